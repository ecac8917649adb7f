"""Elimination of the far-conductor currents and the preconditioner of the reduced system.

TEST INFRASTRUCTURE ONLY (imported by tests/, smoke() and the benchmark's CPU baseline): plain
dense formulas, independent of the HIP library.

The paper's conclusion proposes solving for part of the unknowns first and obtaining the
conductor currents afterwards. With the far conductor's RWG currents x_f as the eliminated
block, this is block Gaussian elimination of the coupled system (eqs. (11) and (15)), with the
unknowns split as [x_f | x_r], x_r = [near currents | body currents]:

    Z_ff x_f + Z_fr x_r = b_f
    Z_rf x_f + Z_rr x_r = b_r
    =>  A_S x_r = b_S,   A_S = Z_rr - Z_rf Z_ff^-1 Z_fr,   b_S = b_r - Z_rf Z_ff^-1 b_f,
        x_f = Z_ff^-1 (b_f - Z_fr x_r).

The reduced system is right-preconditioned by a block-diagonal M: on the near currents the
inverse of the reduced near block (direct Galerkin near-near entries minus the eliminated far
block's contribution through the near-far coupling), on the body unknowns the inverse of the
diagonal of the body block (h^3 / chi + h^3 T_aa(0)); the far currents are not unknowns of the
reduced system.

Pins (tests/test_oracle_schur.py): the reduced solve plus recovery reproduces the dense solve of
the full system; det Z = det Z_ff det A_S; A_S is complex-symmetric when Z is; GMRES on the
preconditioned reduced system converges where plain GMRES on the full system stalls.
"""
import numpy as np


def split(Z, mf):
    """The four blocks of Z for the split [far (mf) | rest]."""
    return Z[:mf, :mf], Z[:mf, mf:], Z[mf:, :mf], Z[mf:, mf:]


def reduced_system(Z, b, mf):
    """(A_S, b_S) of the elimination of the first mf unknowns."""
    Zff, Zfr, Zrf, Zrr = split(Z, mf)
    b = np.asarray(b, np.complex128)
    if mf == 0:
        return Zrr.copy(), b.copy()
    X = np.linalg.solve(Zff, np.column_stack([Zfr, b[:mf]]))
    return Zrr - Zrf @ X[:, :-1], b[mf:] - Zrf @ X[:, -1]


def recover_far(Z, b, x_r, mf):
    """x_f = Z_ff^-1 (b_f - Z_fr x_r)."""
    Zff, Zfr, _, _ = split(Z, mf)
    return np.linalg.solve(Zff, np.asarray(b, np.complex128)[:mf] - Zfr @ x_r)


def reduced_near_block(Znn_direct, Znf, Zff, Zfn):
    """The near block the preconditioner inverts: Z_nn (direct) - Z_nf Z_ff^-1 Z_fn."""
    if Zff is None or Zff.shape[0] == 0:
        return Znn_direct.copy()
    return Znn_direct - Znf @ np.linalg.solve(Zff, Zfn)


def block_preconditioner(near_block, body_diag):
    """Dense right preconditioner M = blockdiag(near_block^-1, diag(1 / body_diag)) on [near | body]."""
    mn, nb = near_block.shape[0], len(body_diag)
    M = np.zeros((mn + nb, mn + nb), np.complex128)
    if mn:
        M[:mn, :mn] = np.linalg.inv(near_block)
    M[mn:, mn:] = np.diag(1.0 / np.asarray(body_diag))
    return M
