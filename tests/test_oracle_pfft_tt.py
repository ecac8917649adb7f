"""Pins of the pFFT projection (paper Sec. II-C, eq. (13), 5x5x5 expansion domain) and of the
tensor-train routines (eq. (9), (14))."""
import numpy as np
import pytest

import vsie_synth as synth
from oracle import pfft, tt
from oracle.quadrature import collapsed_triangle_rule
from oracle.rwg import build_rwg


def test_dual_polynomials_histopolate():
    C = pfft.dual_poly_coeffs()
    for j in range(5):
        for i in range(5):
            a, b = -2.5 + i, -1.5 + i
            val = sum(C[j, k] * (b ** (k + 1) - a ** (k + 1)) / (k + 1) for k in range(5))
            assert abs(val - (i == j)) < 1e-13


def _loop():
    p = synth.small_case()
    m = p.meshes[1]
    return p, build_rwg(m.verts, m.tris)


def test_projection_reproduces_moments():
    """sum_v W_n(v) int_{V_v} x^a y^b z^c dV = int f_n x^a y^b z^c dS for 0 <= a, b, c <= 4."""
    p, rwg = _loop()
    g = p.grid
    base = pfft.stencil_bases(rwg, g.origin, g.h)
    W = pfft.stencil_weights(rwg, base, g.origin, g.h)
    bary, wq = collapsed_triangle_rule(10)
    rng = np.random.default_rng(0)
    for n in rng.choice(rwg.m, 6, replace=False):
        centre = g.origin + (base[n] + 2.5) * g.h
        for a, b, c in [(0, 0, 0), (1, 0, 0), (0, 2, 1), (4, 4, 4), (3, 1, 4), (2, 2, 2)]:
            lhs = np.zeros(3)
            scale = np.zeros(3)
            for j3 in range(5):
                for j2 in range(5):
                    for j1 in range(5):
                        lo = np.array([j1, j2, j3]) - 2.5
                        mom = np.prod([((lo[i] + 1) ** (e + 1) - lo[i] ** (e + 1)) / (e + 1)
                                       for i, e in enumerate((a, b, c))]) * g.h ** 3
                        lhs += W[n, :, j3, j2, j1] * mom
                        scale += np.abs(W[n, :, j3, j2, j1] * mom)
            rhs = np.zeros(3)
            for side, s in ((0, 1.0), (1, -1.0)):
                t = rwg.tri[n, side]
                tv = rwg.verts[rwg.tris[t]]
                pts = bary @ tv
                f = s * rwg.length[n] / (2 * rwg.area[t]) * (pts - rwg.verts[rwg.free[n, side]])
                xi = (pts - centre) / g.h
                mono = xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c
                rhs += (wq * rwg.area[t] * mono) @ f
            # tolerance relative to the sum of magnitudes (the signed terms cancel heavily)
            assert np.all(np.abs(lhs - rhs) <= 1e-13 * scale.max())


def test_projection_weights_rule_independent():
    p, rwg = _loop()
    g = p.grid
    base = pfft.stencil_bases(rwg, g.origin, g.h)
    W8 = pfft.stencil_weights(rwg, base, g.origin, g.h, nquad=8)
    W11 = pfft.stencil_weights(rwg, base, g.origin, g.h, nquad=11)
    assert np.abs(W8 - W11).max() < 1e-12 * np.abs(W8).max()


def test_stencil_refuses_oversized_pair():
    p, rwg = _loop()
    with pytest.raises(pfft.StencilError):
        pfft.stencil_bases(rwg, p.grid.origin, 1e-3)       # 1 mm voxels: 5 mm strip cannot fit


def test_tt_svd_recovers_known_rank_tensor():
    rng = np.random.default_rng(1)
    n = (6, 7, 5, 9)
    r = (2, 3, 2)
    cores = [rng.standard_normal((n[0], r[0])) + 1j * rng.standard_normal((n[0], r[0])),
             rng.standard_normal((r[0], n[1], r[1])) + 0j,
             rng.standard_normal((r[1], n[2], r[2])) + 1j * rng.standard_normal((r[1], n[2], r[2])),
             rng.standard_normal((r[2], n[3])) + 0j]
    A = tt.tt_full(cores)
    got = tt.tt_svd(A, 1e-12)
    assert [c.shape[-1] for c in got[:3]] == list(r)
    assert np.linalg.norm(tt.tt_full(got) - A) < 1e-12 * np.linalg.norm(A)


def test_tt_svd_error_bound_and_contractions():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((5, 6, 4, 7)) + 1j * rng.standard_normal((5, 6, 4, 7))
    for eps in (0.3, 0.1, 0.01):
        c = tt.tt_svd(A, eps)
        assert np.linalg.norm(tt.tt_full(c) - A) <= eps * np.linalg.norm(A) * (1 + 1e-12)
    c = tt.tt_svd(A, 0.1)
    x = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    full = tt.tt_full(c)
    ref = np.einsum("ijkl,l->ijk", full, x).transpose(2, 1, 0).ravel()
    assert np.allclose(tt.tt_matvec(c, x), ref, rtol=1e-14, atol=0)
    y = rng.standard_normal(5 * 6 * 4) + 0j
    # bilinear identity y^T (Z x) = x^T (Z^T y)
    assert abs(y @ tt.tt_matvec(c, x) - x @ tt.tt_rmatvec(c, y, (5, 6, 4))) < 1e-12 * np.linalg.norm(full)
