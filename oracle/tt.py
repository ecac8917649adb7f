"""Tensor train of the far coupling (paper Sec. II-D eq. (9), Sec. III eq. (14), (16)-(19)).

The far coupling block, for voxel component chi, reshaped to a 4D tensor
Z^chi[i1, i2, i3, i4] = Z_bc^far[chi, i1 + n1 (i2 + n2 i3), i4] (i4 = far RWG), is written as

    Z^chi[i1,i2,i3,i4] = sum_{j1,j2,j3} G1[i1,j1] G2[j1,i2,j2] G3[j2,i3,j3] G4[j3,i4].

  * tt_svd: the sequence of truncated SVDs of the unfoldings (the quasi-optimal construction the
    paper cites); used to produce cores for tests and to compare ranks with TT-cross.
  * tt_full: the reconstruction, written as the definition above (one einsum).
  * tt_matvec / tt_rmatvec: the dense products Z^chi x and (Z^chi)^T y through the
    reconstruction (no contraction ordering), the reference for eqs. (16)-(19).

Parity: tt_full is the definition; tt_svd is pinned by exact recovery of a tensor of known
TT rank and by the error bound ||A - TT||_F <= eps ||A||_F.
"""
import numpy as np


def tt_svd(A, eps):
    """TT-SVD of a 4D array with relative Frobenius accuracy eps; returns [G1, G2, G3, G4]."""
    d = A.ndim
    n = A.shape
    delta = eps / np.sqrt(d - 1) * np.linalg.norm(A.ravel())
    cores = []
    C = A.reshape(n[0], -1)
    r_prev = 1
    for k in range(d - 1):
        C = C.reshape(r_prev * n[k], -1)
        U, s, Vh = np.linalg.svd(C, full_matrices=False)
        tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]    # tail[r] = ||s[r:]||
        r = len(s)
        for cand in range(1, len(s) + 1):
            if cand == len(s) or tail[cand] <= delta:
                r = cand
                break
        cores.append(U[:, :r].reshape(r_prev, n[k], r))
        C = s[:r, None] * Vh[:r]
        r_prev = r
    cores.append(C.reshape(r_prev, n[-1]))
    G1 = cores[0].reshape(n[0], -1)
    return [G1, cores[1], cores[2], cores[3]]


def tt_full(cores):
    G1, G2, G3, G4 = cores
    return np.einsum("ia,ajb,bkc,cl->ijkl", G1, G2, G3, G4)


def tt_matvec(cores, x):
    """Z^chi x for x (m,) -> (n1, n2, n3) reshaped to i1 fastest flat (n1*n2*n3,)."""
    A = tt_full(cores)
    y = np.einsum("ijkl,l->ijk", A, x)
    return y.transpose(2, 1, 0).ravel()


def tt_rmatvec(cores, y_flat, n):
    """(Z^chi)^T y for y over voxels (i1 fastest) -> (m,)."""
    A = tt_full(cores)
    y = y_flat.reshape(n[2], n[1], n[0]).transpose(2, 1, 0)
    return np.einsum("ijkl,ijk->l", A, y)


def tt_tensor_from_block(block, n):
    """Reshape a coupling block (n_v, m) with voxel index i1 fastest into (n1, n2, n3, m)."""
    m = block.shape[1]
    return block.reshape(n[2], n[1], n[0], m).transpose(2, 1, 0, 3)
