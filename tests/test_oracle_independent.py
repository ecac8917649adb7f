"""Pins of the oracle's near-field integrals by routes that share nothing with the oracle's own
quadrature code: the face-charge terms of the Toeplitz generator at touching offsets (eq. (5)),
the near and far point rules of the body-conductor coupling (Sec. II-B, Sec. IV-C), and the
Galerkin entries of near conductor pairs (eq. (6) with the quadrature reading Z1).

Each reference below is written from the definitions in this file: a closed-form rectangle
potential with double-exponential outer quadrature for the face terms; the mixed-potential form
(vector potential in the volume, scalar potential on the voxel faces) with high-order rules for
the coupling; a polar-coordinate evaluation of the triangle potential integrals for the
conductor entries. Only the RWG tables (oracle/rwg.py) and the constant rule R5 (which defines
the operator) are taken from the oracle."""
import numpy as np
import pytest

import vsie_synth as synth
from oracle import coupling, surface, voxel
from oracle.quadrature import R5_BARY, R5_W
from oracle.rwg import RWG, build_rwg


# ---------------------------------------------------------------------------------------------
# quadrature written here
def _gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _de01(step):
    """Double-exponential (tanh-sinh) rule on [0, 1]; exponential convergence for integrands with
    integrable end-point singularities such as x log x."""
    t = np.arange(-3.3, 3.3 + 1e-12, step)
    u = 0.5 * np.pi * np.sinh(t)
    x = 0.5 * (1.0 + np.tanh(u))
    w = step * 0.25 * np.pi * np.cosh(t) / np.cosh(u) ** 2
    keep = (x > 0.0) & (x < 1.0)
    return x[keep], w[keep]


def _tri_rule(n):
    """Collapsed Gauss rule on the reference triangle, barycentric points and area fractions."""
    x, w = _gl01(n)
    u, s = np.meshgrid(x, x, indexing="ij")
    wu, ws = np.meshgrid(w, w, indexing="ij")
    l2 = u.ravel()
    l3 = (s * (1.0 - u)).ravel()
    return np.stack([1.0 - l2 - l3, l2, l3], 1), 2.0 * (wu * ws * (1.0 - u)).ravel()


# ---------------------------------------------------------------------------------------------
# A. face-charge terms of the Toeplitz generator at touching offsets
def _rect_static(a1, a2, b1, b2, w):
    """int_{a1}^{a2} int_{b1}^{b2} du dv / sqrt(u^2 + v^2 + w^2) in closed form (the potential of
    a uniformly charged rectangle), vectorised over the corners' arrays."""
    aw = np.abs(w)

    def F(a, b):
        R = np.sqrt(a * a + b * b + aw * aw)

        def xlog(x, y):     # x ln(y + R), stable when y < 0 and with the limit 0 at x = 0
            with np.errstate(divide="ignore", invalid="ignore"):
                arg = np.where(y >= 0, y + R, (x * x + aw * aw) / (R - y))
                v = x * np.log(arg)
            return np.where(x == 0, 0.0, v)

        with np.errstate(divide="ignore", invalid="ignore"):
            at = np.where(aw > 0, aw * np.arctan(a * b / (aw * R)), 0.0)
        return xlog(a, b) + xlog(b, a) - at

    return F(a2, b2) - F(a1, b2) - F(a2, b1) + F(a1, b1)


def test_rectangle_potential_closed_form():
    """The closed form against a plain Gauss product rule at points off the rectangle."""
    x, w = _gl01(60)
    for (px, py, pz) in ((0.3, 0.7, 0.8), (1.7, -0.4, 0.2), (0.5, 0.5, 2.5), (-0.6, 1.4, 0.05)):
        u, v = np.meshgrid(x * 1.0, x * 1.0, indexing="ij")
        ww = np.outer(w, w)
        ref = np.sum(ww / np.sqrt((u - px) ** 2 + (v - py) ** 2 + pz ** 2))
        got = _rect_static(np.array(0.0 - px), np.array(1.0 - px), np.array(0.0 - py), np.array(1.0 - py),
                           np.array(pz))
        assert abs(got - ref) < 1e-11 * abs(ref)


def _face_pair(a, sa, b, sb, d, kappa, step):
    """int_F int_F' K, F = face of the unit voxel at x_a = sa, F' = face of the voxel at offset d
    at x_b = d_b + sb; K = exp(-i kappa rho) / (4 pi rho)."""
    xo, wo = _de01(step)
    oa = [k for k in range(3) if k != a]
    X1, X2 = np.meshgrid(xo, xo, indexing="ij")
    W = np.outer(wo, wo).ravel()
    P = np.zeros((X1.size, 3))
    P[:, a] = sa
    P[:, oa[0]] = X1.ravel()
    P[:, oa[1]] = X2.ravel()
    ob = [k for k in range(3) if k != b]
    wdist = P[:, b] - (d[b] + sb)
    u0, v0 = P[:, ob[0]], P[:, ob[1]]
    stat = _rect_static(d[ob[0]] - u0, d[ob[0]] + 1.0 - u0, d[ob[1]] - v0, d[ob[1]] + 1.0 - v0, wdist)
    static = np.sum(W * stat) / (4.0 * np.pi)
    # bounded remainder (exp(-i kappa rho) - 1) / (4 pi rho): 4D Gauss product, two cells per axis
    x, wg = _gl01(12)
    x = np.concatenate([0.5 * x, 0.5 + 0.5 * x])
    wg = np.concatenate([0.5 * wg, 0.5 * wg])
    g1, g2, g3, g4 = np.meshgrid(x, x, x, x, indexing="ij")
    W4 = np.einsum("i,j,k,l->ijkl", wg, wg, wg, wg).ravel()
    r = np.zeros((g1.size, 3))
    r[:, a] = sa
    r[:, oa[0]] = g1.ravel()
    r[:, oa[1]] = g2.ravel()
    rp = np.zeros((g1.size, 3))
    rp[:, b] = d[b] + sb
    rp[:, ob[0]] = d[ob[0]] + g3.ravel()
    rp[:, ob[1]] = d[ob[1]] + g4.ravel()
    rho = np.linalg.norm(r - rp, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        ph = np.where(rho > 0, (np.exp(-1j * kappa * rho) - 1.0) / rho, -1j * kappa)
    dyn = np.sum(W4 * ph) / (4.0 * np.pi)
    return static + dyn


def _face_term(a, b, d, kappa, step=1.0 / 24):
    """I_ff^{ab}(d) in units of h: the four face pairs with their outward normal signs."""
    tot = 0.0
    for sa in (0, 1):
        for sb in (0, 1):
            tot += (2 * sa - 1) * (2 * sb - 1) * _face_pair(a, sa, b, sb, d, kappa, step)
    return tot


def test_generator_face_terms_touching_offsets():
    """Off-diagonal face-charge components I_ff^{ab} at every offset d in {0, 1}^3 (perpendicular
    faces sharing an edge or a corner: the cases the Duffy-mapped cells handle) against the
    closed-form rectangle potential integrated with a double-exponential rule; the rule is also
    shown converged by halving its step."""
    kappa = 0.031
    ds = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], np.float64)
    ora = voxel.face_integrals(ds, kappa)
    ref = np.zeros((len(ds), 3), np.complex128)
    for comp, (a, b) in enumerate(voxel.COMPONENTS[3:]):
        for i, d in enumerate(ds):
            ref[i, comp] = _face_term(a, b, d, kappa)
    # convergence of the reference on the most singular offset (d = 0)
    c0 = _face_term(0, 1, ds[0], kappa, step=1.0 / 48)
    assert abs(c0 - ref[0, 0]) < 1e-12 * np.abs(ref).max()
    err = np.abs(ora[:, 3:] - ref).max() / np.abs(ref).max()
    assert err < 1e-10, err
    # and on a diagonal component at a face-sharing offset (coplanar faces meeting at an edge)
    dd = np.array([1.0, 0.0, 0.0])
    diag = _face_term(1, 1, dd, kappa)
    assert abs(voxel.face_integrals(dd[None], kappa)[0, 1] - diag) < 1e-10 * abs(diag)


# ---------------------------------------------------------------------------------------------
# B. body-conductor coupling: near and far point rules against the mixed-potential form
def _rwg_parts(rwg, n):
    """Per triangle of RWG n: vertices, area, and f(r) = c (r - p) with c = +-l / (2A), div f."""
    out = []
    for side, s in ((0, 1.0), (1, -1.0)):
        t = rwg.tri[n, side]
        v = rwg.verts[rwg.tris[t]]
        A = rwg.area[t]
        p = rwg.verts[rwg.free[n, side]]
        out.append((v, A, p, s * rwg.length[n] / (2.0 * A), s * rwg.length[n] / A))
    return out


def _potentials(pts, parts, k, order=10):
    """A(r) = int g f dS' and Phi(r) = int g div f dS' at points (P, 3), high-order rule (the
    points are at least a voxel away from the support)."""
    bary, wt = _tri_rule(order)
    Aout = np.zeros((len(pts), 3), np.complex128)
    Pout = np.zeros(len(pts), np.complex128)
    for v, A, p, c, dv in parts:
        q = bary @ v
        R = np.linalg.norm(pts[:, None, :] - q[None], axis=2)
        g = np.exp(-1j * k * R) / (4.0 * np.pi * R) * (wt * A)[None]
        Aout += g @ (c * (q - p))
        Pout += g.sum(1) * dv
    return Aout, Pout


def _zbc_mixed_potential(centre, h, parts, k, nv=8):
    """-[k^2 int_V A dV + oint_dV Phi n dS] for one voxel, Gauss nv per direction."""
    x, w = _gl01(nv)
    x = x - 0.5
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    pts = centre + h * np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    W3 = np.einsum("i,j,k->ijk", w, w, w).ravel() * h ** 3
    Av, _ = _potentials(pts, parts, k)
    vol = (W3[:, None] * Av).sum(0)
    surf = np.zeros(3, np.complex128)
    U, V = np.meshgrid(x, x, indexing="ij")
    W2 = np.outer(w, w).ravel() * h ** 2
    for a in range(3):
        oa = [i for i in range(3) if i != a]
        for s in (-0.5, 0.5):
            q = np.zeros((U.size, 3))
            q[:, a] = s
            q[:, oa[0]] = U.ravel()
            q[:, oa[1]] = V.ravel()
            _, Ph = _potentials(centre + h * q, parts, k)
            surf[a] += np.sign(s) * np.sum(W2 * Ph)
    return -(k * k * vol + surf)


def test_coupling_point_rules_against_mixed_potential_form():
    """Z_bc of separated voxel-RWG pairs: the 8 x 5 near rule and the 1 x 1 far rule against the
    converged mixed-potential integral (no dyad involved). Both rules converge towards it with
    distance, the near rule well inside the far rule's error."""
    p = synth.small_case()
    mesh = p.meshes[1]
    rwg = build_rwg(mesh.verts, mesh.tris)
    k = 2 * np.pi * 297.2e6 / 299792458.0
    h = 5e-3
    n = 7
    parts = _rwg_parts(rwg, n)
    cen = rwg.verts[rwg.edge[n]].mean(0)
    rng = np.random.default_rng(2)
    errs = {}
    for dist in (3, 6, 12):
        dirs = rng.standard_normal((3, 3))
        dirs /= np.linalg.norm(dirs, axis=1)[:, None]
        for j, u in enumerate(dirs):
            c = cen + dist * h * u
            ref = _zbc_mixed_potential(c, h, parts, k)
            sub = RWG(rwg.edge[[n]], rwg.tri[[n]], rwg.free[[n]], rwg.free_local[[n]], rwg.length[[n]],
                      rwg.verts, rwg.tris, rwg.area)
            near = coupling.zbc_block(c[None], h, sub, k, "near")[:, 0, 0]
            far = coupling.zbc_block(c[None], h, sub, k, "far")[:, 0, 0]
            en = np.linalg.norm(near - ref) / np.linalg.norm(ref)
            ef = np.linalg.norm(far - ref) / np.linalg.norm(ref)
            errs.setdefault(dist, []).append((en, ef))
    for dist, v in errs.items():
        en = max(e[0] for e in v)
        ef = max(e[1] for e in v)
        print("distance %d voxels: near rule %.2e, far rule %.2e" % (dist, en, ef))
    en3 = max(e[0] for e in errs[3])
    en12 = max(e[0] for e in errs[12])
    ef3 = max(e[1] for e in errs[3])
    ef12 = max(e[1] for e in errs[12])
    assert en3 < 2e-3 and en12 < 2e-5
    assert ef3 < 0.1 and ef12 < 1e-2
    assert en12 < 0.05 * en3 and ef12 < 0.2 * ef3
    assert all(e[0] < 0.2 * e[1] for v in errs.values() for e in v)


# ---------------------------------------------------------------------------------------------
# C. Galerkin entries of near conductor pairs
def _polar_static(r, tri, nth=64):
    """int_T 1/R dS' and int_T (r' - r)/R dS' for one point r and triangle tri (3, 3): the
    triangle is split at the foot rho of r into three signed triangles with apex rho, each
    integrated in polar coordinates about rho with the radial integrals in closed form. The angle
    is parametrised by tau = asinh(l / t0), l the abscissa along the edge from the foot of rho on
    the edge line and t0 that foot's distance (d theta = d tau / cosh tau), which keeps the
    angular integrand smooth when rho lies close to an edge line; Gauss in tau."""
    e1 = tri[1] - tri[0]
    e2 = tri[2] - tri[0]
    nrm = np.cross(e1, e2)
    nrm /= np.linalg.norm(nrm)
    d = float(np.dot(r - tri[0], nrm))
    ad = abs(d)
    rho = r - d * nrm
    xg, wg = _gl01(nth)
    S0 = 0.0
    S1 = np.zeros(3)
    for i in range(3):
        a, b = tri[i], tri[(i + 1) % 3]
        va, vb = a - rho, b - rho
        ang = np.arctan2(np.dot(np.cross(va, vb), nrm), np.dot(va, vb))
        et = (b - a) / np.linalg.norm(b - a)
        foot = va - np.dot(va, et) * et            # foot of rho on the edge line, relative to rho
        t0 = np.linalg.norm(foot)
        if t0 < 1e-15 * np.linalg.norm(b - a) or abs(ang) == 0.0:
            continue                               # rho on the edge line: a degenerate wedge
        la, lb = np.dot(va, et), np.dot(vb, et)
        ta, tb = np.arcsinh(la / t0), np.arcsinh(lb / t0)
        tau = ta + (tb - ta) * xg
        wt = (tb - ta) * wg / np.cosh(tau)
        ell = t0 * np.sinh(tau)
        smax = t0 * np.cosh(tau)
        dirs = (foot[None, :] + ell[:, None] * et[None, :]) / smax[:, None]
        R = np.sqrt(smax * smax + d * d)
        I0 = R - ad
        if ad > 0:
            I1 = 0.5 * (smax * R - d * d * np.log((smax + R) / ad))
        else:
            I1 = 0.5 * smax * smax
        sg = np.sign(ang)
        S0 += sg * np.sum(wt * I0)
        S1 += sg * (wt * I1) @ dirs
    return S0, S1 - d * nrm * S0


def _zcc_entry(rwg_t, m, rwg_s, n, k, near_fn):
    """Z_cc[m, n] from the RWG definitions: per triangle pair, outer R5 on one triangle, inner
    static part by _polar_static and remainder by R5 for near pairs (averaged over the two
    orderings), R5 x R5 with the full kernel otherwise."""
    tm = _rwg_parts(rwg_t, m)
    tn = _rwg_parts(rwg_s, n)

    def oriented(P, Q):
        (v1, A1, p1, c1, d1), (v2, A2, p2, c2, d2) = P, Q
        q1 = R5_BARY @ v1
        q2 = R5_BARY @ v2
        tot = 0.0
        for i in range(5):
            r = q1[i]
            s0, s1 = _polar_static(r, v2)
            Rr = np.linalg.norm(q2 - r, axis=1)
            with np.errstate(divide="ignore", invalid="ignore"):
                ph = np.where(Rr > 0, (np.exp(-1j * k * Rr) - 1.0) / Rr, -1j * k) * R5_W * A2
            Ig = (s0 + ph.sum()) / (4.0 * np.pi)                          # int g
            Igf = c2 * ((s1 + (r - p2) * s0) + ph @ (q2 - p2)) / (4.0 * np.pi)   # int g f_n
            fm = c1 * (r - p1)
            tot += R5_W[i] * A1 * (-(k * k) * np.dot(fm, Igf) + d1 * d2 * Ig)
        return tot

    def r5r5(P, Q):
        (v1, A1, p1, c1, d1), (v2, A2, p2, c2, d2) = P, Q
        q1 = R5_BARY @ v1
        q2 = R5_BARY @ v2
        R = np.linalg.norm(q1[:, None] - q2[None], axis=2)
        g = np.exp(-1j * k * R) / (4.0 * np.pi * R) * np.outer(R5_W * A1, R5_W * A2)
        f1 = c1 * (q1 - p1)
        f2 = c2 * (q2 - p2)
        return np.sum(g * (-(k * k) * (f1 @ f2.T) + d1 * d2))

    tot = 0.0
    for P in tm:
        for Q in tn:
            if near_fn(P[0], Q[0]):
                tot += 0.5 * (oriented(P, Q) + oriented(Q, P))
            else:
                tot += r5r5(P, Q)
    return tot


def _near(va, vb):
    ca, cb = va.mean(0), vb.mean(0)
    e2 = max(np.sum((va[(i + 1) % 3] - va[i]) ** 2) for i in range(3))
    e2 = max(e2, max(np.sum((vb[(i + 1) % 3] - vb[i]) ** 2) for i in range(3)))
    return np.sum((ca - cb) ** 2) < 16.0 * e2


def test_polar_static_against_product_rule():
    """The polar evaluation against a high-order rule at points well off the triangle."""
    tri = np.array([[0.0, 0.0, 0.0], [1.0, 0.2, 0.0], [0.3, 0.9, 0.1]])
    bary, wt = _tri_rule(40)
    q = bary @ tri
    A = 0.5 * np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0]))
    for r in (np.array([0.4, 0.4, 0.9]), np.array([2.0, -1.0, 0.5]), np.array([0.5, 0.3, 0.3]),
              np.array([-0.3, -0.06 + 1e-5, 0.4])):
        R = np.linalg.norm(q - r, axis=1)
        s0 = np.sum(wt * A / R)
        s1 = (wt * A / R) @ (q - r)
        p0, p1 = _polar_static(r, tri)
        assert abs(p0 - s0) < 1e-11 * abs(s0)
        assert np.linalg.norm(p1 - s1) < 1e-11 * np.linalg.norm(s1)


@pytest.mark.parametrize("mesh_index", [1, 0])
def test_zcc_near_entries_from_definitions(mesh_index):
    """Self, edge-adjacent, vertex-adjacent and near entries of Z_cc (strip loop; coarse closed
    shield) recomputed from the RWG definitions with polar inner integrals: 1e-10 relative."""
    p = synth.small_case()
    mesh = p.meshes[mesh_index]
    rwg = build_rwg(mesh.verts, mesh.tris)
    k = 2 * np.pi * 297.2e6 / 299792458.0
    rng = np.random.default_rng(mesh_index)
    ms = rng.choice(rwg.m, 4, replace=False)
    Z = surface.zcc_block(rwg, rwg, k)
    for m in ms:
        # neighbours through shared triangles and vertices, plus one farther function
        tr = set(rwg.tri[m])
        vt = set(rwg.tris[list(tr)].ravel())
        cand = [n for n in range(rwg.m) if set(rwg.tri[n]) & tr or set(rwg.tris[list(rwg.tri[n])].ravel()) & vt]
        cand = sorted(set(cand))[:8] + [int(rng.integers(rwg.m))]
        for n in cand:
            ref = _zcc_entry(rwg, m, rwg, n, k, _near)
            assert abs(Z[m, n] - ref) <= 1e-10 * abs(ref), (m, n, Z[m, n], ref)
