"""Pins of the oracle's far-current elimination and reduced-system preconditioner (oracle/schur.py)
against exact algebra: block elimination reproduces the full solve, the determinant factorises,
symmetry is kept, and the preconditioned reduced system converges."""
import numpy as np
import pytest

import vsie_synth as synth
from oracle import gmres, schur, system


def _random_symmetric(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return A + A.T + 4 * np.sqrt(n) * np.eye(n)


@pytest.mark.parametrize("mf", [0, 1, 7, 40])
def test_elimination_reproduces_full_solve(mf):
    Z = _random_symmetric(60, 3 + mf)
    rng = np.random.default_rng(11)
    b = rng.standard_normal(60) + 1j * rng.standard_normal(60)
    x = np.linalg.solve(Z, b)
    A_S, b_S = schur.reduced_system(Z, b, mf)
    x_r = np.linalg.solve(A_S, b_S)
    x_f = schur.recover_far(Z, b, x_r, mf)
    assert np.linalg.norm(np.concatenate([x_f, x_r]) - x) <= 1e-12 * np.linalg.norm(x)


@pytest.fixture(scope="module")
def small_direct():
    p = synth.small_case()
    d = system.discretize(p)
    S, blocks = system.assemble_direct(d)
    return d, S, blocks


def test_determinant_factorises(small_direct):
    """det Z = det Z_ff det A_S (the Schur determinant identity), on the coupled small case."""
    d, S, _ = small_direct
    A_S, _ = schur.reduced_system(S.Z, np.zeros(S.Z.shape[0]), d.m_f)
    s1, l1 = np.linalg.slogdet(S.Z)
    s2, l2 = np.linalg.slogdet(S.Z[:d.m_f, :d.m_f])
    s3, l3 = np.linalg.slogdet(A_S)
    assert abs(l1 - (l2 + l3)) <= 1e-9 * abs(l1)
    assert abs(s1 - s2 * s3) <= 1e-8


def test_reduced_operator_is_symmetric(small_direct):
    d, S, _ = small_direct
    A_S, _ = schur.reduced_system(S.Z, np.zeros(S.Z.shape[0]), d.m_f)
    assert np.linalg.norm(A_S - A_S.T) <= 1e-12 * np.linalg.norm(A_S)


def test_preconditioned_reduced_gmres_converges(small_direct):
    """Right-preconditioned GMRES(50) on the reduced system reaches 1e-6 within 60 iterations on
    the coupled small case, where GMRES(50) on the full system is still above 1e-2 after 300;
    the recovered full solution has full-system residual at the same level."""
    d, S, blocks = small_direct
    mf, mn = d.m_f, d.m_n
    Z = S.Z
    b = system.port_rhs(d, 0)[S.red_idx]
    _, it_full, h_full = gmres.gmres(lambda v: Z @ v, b, tol=1e-6, restart=50, max_iter=300)
    assert h_full[-1] > 1e-2
    A_S, b_S = schur.reduced_system(Z, b, mf)
    near = schur.reduced_near_block(blocks["nn"], Z[mf:mf + mn, :mf], Z[:mf, :mf], Z[:mf, mf:mf + mn])
    M = schur.block_preconditioner(near, np.diag(Z)[mf + mn:])
    u, it, h = gmres.gmres(lambda v: A_S @ (M @ v), b_S, tol=1e-6, restart=50, max_iter=200)
    assert it <= 60 and h[-1] <= 1e-6
    x_r = M @ u
    x = np.concatenate([schur.recover_far(Z, b, x_r, mf), x_r])
    assert np.linalg.norm(b - Z @ x) <= 1.5e-6 * np.linalg.norm(b)
