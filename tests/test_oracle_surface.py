"""Pins of the oracle's conductor integrals: closed-form triangle integrals, the 5-point rule,
the EFIE block (paper eqs. (2), (6)) and the coupling dyad (Sec. II-B, Sec. IV-C)."""
from math import factorial

import numpy as np
import pytest

import vsie_synth as synth
from oracle import coupling, surface
from oracle.quadrature import R5_BARY, R5_W, collapsed_triangle_rule, gauss01
from oracle.rwg import MeshError, build_rwg


def test_r5_rule_exact_to_degree_3():
    for i in range(4):
        for j in range(4 - i):
            for k in range(4 - i - j):
                exact = factorial(i) * factorial(j) * factorial(k) * 2.0 / factorial(i + j + k + 2)
                got = np.sum(R5_W * R5_BARY[:, 0] ** i * R5_BARY[:, 1] ** j * R5_BARY[:, 2] ** k)
                assert abs(got - exact) < 1e-15
    assert np.all(R5_W > 0) and abs(R5_W.sum() - 1) < 1e-15 and np.all(R5_BARY > 0)


QTRI = np.array([[0.0, 0, 0], [1.0, 0.1, 0], [0.3, 0.9, 0]])


@pytest.mark.parametrize("r", [(0.3, 0.3, 0.5), (2.0, -1.0, 0.2), (1.5, 1.5, 0.0), (-0.5, 0.05, 0.0),
                               (3, 0.3, 0.01), (0.5, -0.4, 0.0)])
def test_triangle_static_closed_form_off_triangle(r):
    r = np.array(r)
    bary, w = collapsed_triangle_rule(80)
    A = 0.5 * np.linalg.norm(np.cross(QTRI[1] - QTRI[0], QTRI[2] - QTRI[0]))
    pts = bary @ QTRI
    R = np.linalg.norm(pts - r, axis=1)
    s0, s1 = surface.triangle_static(r[None], QTRI[None])
    assert abs(s0[0] - (w * A / R).sum()) < 1e-12
    assert np.abs(s1[0] - ((w * A / R)[:, None] * (pts - r)).sum(0)).max() < 1e-12


def test_triangle_static_point_inside():
    """In-plane point inside the triangle: Duffy-split numerical reference."""
    r = np.array([0.4, 0.3, 0.0])
    x, wx = gauss01(40)
    tot0, tot1 = 0.0, np.zeros(3)
    for a, b in ((0, 1), (1, 2), (2, 0)):
        ar = 0.5 * np.linalg.norm(np.cross(QTRI[a] - r, QTRI[b] - r))
        T, U = np.meshgrid(x, x, indexing="ij")
        W = np.outer(wx, wx)
        P = r + T[..., None] * ((1 - U)[..., None] * (QTRI[a] - r) + U[..., None] * (QTRI[b] - r))
        R = np.linalg.norm(P - r, axis=-1)
        tot0 += (W * T * 2 * ar / R).sum()
        tot1 += ((W * T * 2 * ar / R)[..., None] * (P - r)).sum((0, 1))
    s0, s1 = surface.triangle_static(r[None], QTRI[None])
    assert abs(s0[0] - tot0) < 1e-13 and np.abs(s1[0] - tot1).max() < 1e-13


def test_rwg_rejects_inconsistent_mesh():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float)
    with pytest.raises(MeshError):
        build_rwg(v, np.array([[0, 1, 2], [1, 2, 3]]))        # edge 1->2 listed twice


def test_zcc_symmetric_and_near_rule_converges():
    p = synth.small_case()
    far = p.meshes[0]
    rwg = build_rwg(far.verts, far.tris)
    k = 2 * np.pi * 297.2e6 / 299792458.0
    Z = surface.zcc_block(rwg, rwg, k)
    assert np.abs(Z - Z.T).max() < 1e-14 * np.abs(Z).max()
    # far pairs use the R5xR5 rule: check it against a high-order product rule on a separated pair
    cen = far.verts[far.tris].mean(1)
    j = int(np.argmax(np.linalg.norm(cen - cen[0], axis=1)))
    va = far.verts[far.tris[[0]]]
    vb = far.verts[far.tris[[j]]]
    Aa = np.array([0.5 * np.linalg.norm(np.cross(va[0, 1] - va[0, 0], va[0, 2] - va[0, 0]))])
    Ab = np.array([0.5 * np.linalg.norm(np.cross(vb[0, 1] - vb[0, 0], vb[0, 2] - vb[0, 0]))])
    assert not surface.near_pairs(va, vb)[0]
    B, _ = surface.pair_moments(va, vb, Aa, Ab, k)
    bary, w = collapsed_triangle_rule(12)
    ra, rb = bary @ va[0], bary @ vb[0]
    R = np.linalg.norm(ra[:, None] - rb[None], axis=2)
    ref = np.sum(np.outer(w * Aa[0], w * Ab[0]) * np.exp(-1j * k * R) / (4 * np.pi * R))
    assert abs(B[0] - ref) < 1e-3 * abs(ref)


def test_dyad_matches_finite_differences():
    """(k^2 I + grad grad) g applied to v against central differences of g."""
    k = 6.2
    R = np.array([0.031, -0.017, 0.022])
    v = np.array([0.3 + 0.1j, -0.2, 0.5j])
    got = coupling.dyad_apply(R[None], v[None], k)[0]

    def g(x):
        r = np.linalg.norm(x)
        return np.exp(-1j * k * r) / (4 * np.pi * r)

    hstep = 1e-5
    H = np.zeros((3, 3), complex)
    for i in range(3):
        for j in range(3):
            ei, ej = np.eye(3)[i] * hstep, np.eye(3)[j] * hstep
            H[i, j] = (g(R + ei + ej) - g(R + ei - ej) - g(R - ei + ej) + g(R - ei - ej)) / (4 * hstep ** 2)
    ref = k * k * g(R) * v + H @ v
    assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()
