"""Precorrected-FFT projection of near-conductor RWG currents onto the voxel grid
(paper Sec. II-C and Sec. III eq. (13); expansion domain 5 x 5 x 5 voxels, Sec. IV-B).

The paper cites the projection rule without stating it. Reading used here:
  * stencil: for RWG n the 5^3 block of voxels centred on the voxel that contains the midpoint
    of the common edge (base index b = floor((c - origin)/h) - 2 per axis, relative to the body
    grid). Both triangles must lie inside the block, otherwise the projection is refused.
  * weights: the PWC voxel currents J_v on the block reproduce every moment
    int f_n(r) x^a y^b z^c dS for 0 <= a, b, c <= 4. Per axis this is a 5x5 system; its solution
    is W_{n,alpha}(v) = h^-3 int f_{n,alpha}(r) phi_{v1}(x) phi_{v2}(y) phi_{v3}(z) dS with phi_j
    the degree-4 polynomials whose integral over voxel i of the block is delta_ij (times h).
  * interpolation back to the RWG is the transpose W^T, which keeps the operator symmetric.
  * precorrection: for RWG pairs whose blocks lie within Chebyshev distance D voxels, and for
    tissue voxels within D voxels of a block, the grid interaction is replaced by the direct
    entry (Z_cc for conductor pairs; the 8 x 5 point coupling rule for voxel-RWG pairs).

The dual polynomials are computed exactly in rational arithmetic (Fraction) and converted once.

Parity pins (tests): the moment identities sum_v W(v) int_{V_v} x^a = int f x^a (exact), and
exactness under a higher-order surface rule.
"""
from fractions import Fraction

import numpy as np

from .quadrature import collapsed_triangle_rule

STENCIL = 5


class StencilError(ValueError):
    pass


def dual_poly_coeffs():
    """C[j, k]: phi_j(xi) = sum_k C[j, k] xi^k on the centred block coordinate xi in [-2.5, 2.5],
    with int_{voxel i} phi_j dxi = delta_ij (voxel i = [-2.5 + i, -1.5 + i])."""
    half = Fraction(5, 2)
    A = [[None] * 5 for _ in range(5)]   # A[k][i] = int_{voxel i} xi^k
    for k in range(5):
        for i in range(5):
            a, b = -half + i, -half + i + 1
            A[k][i] = (b ** (k + 1) - a ** (k + 1)) / (k + 1)
    # solve A^T C^T = I  ->  C = (A^{-1})  with C[j,k] = (A^{-1})[j,k]
    n = 5
    M = [[A[r][c] for c in range(n)] + [Fraction(int(r == c)) for c in range(n)] for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [x / pv for x in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    Ainv = [row[n:] for row in M]        # Ainv = A^{-1}; A c = mu -> c = Ainv mu
    return np.array([[float(Ainv[j][k]) for k in range(n)] for j in range(n)])


def stencil_bases(rwg, origin, h):
    """Base voxel index (m, 3) of every RWG's 5^3 block, relative to the body grid origin."""
    v = rwg.verts
    c = 0.5 * (v[rwg.edge[:, 0]] + v[rwg.edge[:, 1]])
    k = np.floor((c - origin[None, :]) / h).astype(np.int64)
    base = k - 2
    lo = origin[None, :] + base * h
    hi = lo + STENCIL * h
    for side in (0, 1):
        tv = v[rwg.tris[rwg.tri[:, side]]]          # (m, 3, 3)
        if np.any(tv < lo[:, None, :]) or np.any(tv > hi[:, None, :]):
            raise StencilError("an RWG pair does not fit its 5x5x5 expansion block")
    return base


def stencil_weights(rwg, base, origin, h, nquad=8):
    """W (m, 3, 5, 5, 5) indexed [n, alpha, j3, j2, j1] (i1 fastest)."""
    C = dual_poly_coeffs()
    bary, wq = collapsed_triangle_rule(nquad)
    m = rwg.m
    W = np.zeros((m, 3, 5, 5, 5))
    centre = origin[None, :] + (base + 2.5) * h        # block centre
    for side, s in ((0, 1.0), (1, -1.0)):
        tri = rwg.tri[:, side]
        tv = rwg.verts[rwg.tris[tri]]
        pts = np.einsum("qk,mkc->mqc", bary, tv)                  # (m, nq, 3)
        area = rwg.area[tri]
        f = (pts - rwg.verts[rwg.free[:, side]][:, None, :]) * (s * rwg.length / (2.0 * area))[:, None, None]
        xi = (pts - centre[:, None, :]) / h                        # (m, nq, 3)
        pw = xi[..., None] ** np.arange(5)                          # (m, nq, 3, 5)
        phi = np.einsum("mqck,jk->mqcj", pw, C)                     # (m, nq, 3, 5) phi_j(xi_c)
        wts = wq[None, :] * area[:, None]                           # (m, nq)
        W += np.einsum("mq,mqa,mqz,mqy,mqx->mazyx", wts, f, phi[:, :, 2], phi[:, :, 1], phi[:, :, 0])
    return W / h ** 3


def stencil_voxels(base):
    """Voxel index triples (m, 125, 3) of every block, in [j3, j2, j1] order."""
    j = np.arange(5)
    z, y, x = np.meshgrid(j, j, j, indexing="ij")
    off = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    return base[:, None, :] + off[None, :, :]


def near_rwg_pairs(base, dist):
    """Pairs (m, n) whose blocks are within Chebyshev distance `dist` voxels."""
    b = base
    gap = np.maximum(np.maximum(b[None, :, :] - (b[:, None, :] + 4), b[:, None, :] - (b[None, :, :] + 4)), 0)
    near = gap.max(2) <= dist
    return np.nonzero(near)


def near_voxel_rwg(base, vox, dist):
    """Pairs (voxel list position p, RWG n) with voxel within `dist` of block n."""
    gap = np.maximum(np.maximum(base[None, :, :] - vox[:, None, :], vox[:, None, :] - (base[None, :, :] + 4)), 0)
    near = gap.max(2) <= dist
    return np.nonzero(near)
