"""Pins of the oracle's voxel Galerkin integrals (paper Sec. II-B, eqs. (4), (5), (7))."""
import mpmath as mp
import numpy as np
import pytest

from oracle import voxel
from oracle.quadrature import gauss01

KAPPA = 2 * np.pi * 297.2e6 / 299792458.0 * 5e-3    # k0 h at 5 mm


def test_trace_identity_exact():
    """sum_a I_ff^{aa}(d) = k0^2 I_vv(d) + dv delta_{d,0}: follows from div grad g = -k^2 g - delta.

    Ties the face integrals (F2) to the volume integral V, singular offsets included."""
    rng = np.random.default_rng(3)
    d = np.concatenate([np.array([[0, 0, 0], [1, 0, 0], [0, 1, 1], [1, 1, 1], [2, 1, 0], [-1, 2, -1]]),
                        rng.integers(-9, 10, (20, 3))]).astype(float)
    for kap in (KAPPA, 0.4):
        V = voxel.V_integral(d, kap)
        F = voxel.face_integrals(d, kap)
        resid = F[:, :3].sum(1) - kap ** 2 * V - (np.abs(d).sum(1) == 0)
        assert np.abs(resid).max() < 2e-15


def _bf_vv(d, kap, n=6):
    x, w = gauss01(n)
    g = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(-1, 3)
    wg = np.einsum("i,j,k->ijk", w, w, w).ravel()
    r = np.linalg.norm(g[:, None, :] - (g[None, :, :] + d), axis=2)
    return (wg[:, None] * wg[None, :] * np.exp(-1j * kap * r) / (4 * np.pi * r)).sum()


def _bf_face(d, a, b, kap, n=8):
    """Definition of I_ff^{ab}: sum over faces of voxel 0 normal to a and faces of voxel d normal
    to b of n_a n'_b int int g (4D tensor Gauss, separated voxels only)."""
    x, w = gauss01(n)
    U, Vv = np.meshgrid(x, x, indexing="ij")
    Wt = np.outer(w, w).ravel()
    U, Vv = U.ravel(), Vv.ravel()
    tot = 0.0
    for sa in (0, 1):
        pa = np.zeros((len(U), 3))
        oth = [i for i in range(3) if i != a]
        pa[:, a] = sa
        pa[:, oth[0]] = U
        pa[:, oth[1]] = Vv
        for sb in (0, 1):
            pb = np.zeros((len(U), 3))
            othb = [i for i in range(3) if i != b]
            pb[:, b] = sb
            pb[:, othb[0]] = U
            pb[:, othb[1]] = Vv
            pb = pb + np.asarray(d, float)
            r = np.linalg.norm(pa[:, None, :] - pb[None, :, :], axis=2)
            val = (Wt[:, None] * Wt[None, :] * np.exp(-1j * kap * r) / (4 * np.pi * r)).sum()
            tot += (2 * sa - 1) * (2 * sb - 1) * val
    return tot


@pytest.mark.parametrize("d", [(3, 2, 1), (0, 0, 5), (4, -3, 2), (-3, 3, 3)])
def test_volume_integral_matches_6d_definition(d):
    """Tent-reduced V(d) equals the plain 6D box x box integral at separated offsets."""
    ref = _bf_vv(np.array(d, float), KAPPA)
    got = voxel.V_integral(np.array([d], float), KAPPA)[0]
    assert abs(got - ref) < 2e-13 * abs(ref)


@pytest.mark.parametrize("d", [(3, 2, 1), (4, -3, 2), (-2, 3, 3)])
def test_face_integrals_match_4d_definition(d):
    """Second-difference and mixed-difference forms equal the face-pair definition."""
    got = voxel.face_integrals(np.array([d], float), KAPPA)[0]
    for comp, (a, b) in enumerate(voxel.COMPONENTS):
        ref = _bf_face(d, a, b, KAPPA)
        assert abs(got[comp] - ref) < 1e-11 * np.abs(got).max(), (comp, got[comp], ref)


def test_singular_self_terms_against_tanh_sinh():
    """V(0) and F2(0; 0, 0) without the Duffy map: the static part with one coordinate
    integrated in closed form, int_0^1 (1 - z)/sqrt(p^2 + z^2) dz = asinh(1/p) - sqrt(p^2 + 1) + p,
    and the remaining log-singular integral by mpmath's double-exponential rule; the bounded
    dynamic remainder (exp(-i kappa r) - 1)/r by a high-order tensor Gauss rule."""
    mp.mp.dps = 20

    def inner(p):
        return mp.asinh(1 / p) - mp.sqrt(p * p + 1) + p

    v_static = 8 * mp.quad(lambda x, y: (1 - x) * (1 - y) * inner(mp.sqrt(x * x + y * y)), [0, 1], [0, 1])
    f_static = 4 * mp.quad(lambda x: (1 - x) * inner(x), [0, 1])
    x, w = gauss01(48)

    def dyn(r):
        return (np.exp(-1j * KAPPA * r) - 1.0) / r

    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W3 = np.einsum("i,j,k->ijk", w, w, w)
    v_dyn = 8 * np.sum(W3 * (1 - X) * (1 - Y) * (1 - Z) * dyn(np.sqrt(X ** 2 + Y ** 2 + Z ** 2)))
    X2, Y2 = np.meshgrid(x, x, indexing="ij")
    f_dyn = 4 * np.sum(np.outer(w, w) * (1 - X2) * (1 - Y2) * dyn(np.sqrt(X2 ** 2 + Y2 ** 2)))
    v_ref = (float(v_static) + v_dyn) / (4 * np.pi)
    f_ref = (float(f_static) + f_dyn) / (4 * np.pi)
    V = voxel.V_integral(np.zeros((1, 3)), KAPPA)[0]
    F = voxel.F2_integral(np.zeros(1), np.zeros((1, 2)), KAPPA)[0]
    assert abs(V - v_ref) < 1e-11 * abs(V)
    assert abs(F - f_ref) < 1e-11 * abs(F)


def test_converged_in_quadrature_order():
    d = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1], [2, 0, 1], [5, 3, 2], [11, 0, 7]], float)
    base = voxel.T_generator(d, KAPPA)
    ref = np.zeros_like(base)
    # raise both the Duffy order and the regular-cell accuracy target
    orig = voxel.cell_integrals.__defaults__
    try:
        voxel.cell_integrals.__defaults__ = (16,) + orig[1:]
        old = voxel._bernstein_order.__defaults__
        voxel._bernstein_order.__defaults__ = (21.0, 3, 20)
        ref = voxel.T_generator(d, KAPPA)
    finally:
        voxel.cell_integrals.__defaults__ = orig
        voxel._bernstein_order.__defaults__ = old
    scale = np.abs(base).max()
    assert np.abs(base - ref).max() < 1e-14 * scale


def test_parity_of_components_and_lookup():
    """Diagonal components even in every axis; ab odd in d_a and d_b; lookup equals direct."""
    rng = np.random.default_rng(5)
    d = rng.integers(-6, 7, (25, 3))
    direct = voxel.T_generator(d.astype(float), KAPPA)
    table = voxel.T_generator_octant((7, 7, 7), KAPPA)
    looked = voxel.T_lookup(table, d)
    assert np.abs(direct - looked).max() < 1e-15 * np.abs(direct).max()


def test_far_field_limit():
    """Far away, V(d) -> K(|d|) (each tent integrates to one)."""
    d = np.array([[40.0, 31.0, 25.0]])
    r = np.linalg.norm(d)
    V = voxel.V_integral(d, KAPPA)[0]
    K = np.exp(-1j * KAPPA * r) / (4 * np.pi * r)
    assert abs(V - K) < 1e-3 * abs(K)
