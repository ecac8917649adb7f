"""Galerkin EFIE matrix of the conductors, Z_cc (paper Sec. II-B, eq. (2) and (6)).

Mixed-potential Galerkin form, rows multiplied by i w eps0 (the same scaling as the body rows):

    Z_cc[m, n] = -k0^2 int_Tm int_Tn f_m . f_n g  +  int_Tm int_Tn (div f_m)(div' f_n) g

derived from E_scat = (k0^2 + grad div) A / (i w eps0), A = int g J, by testing with f_m and
moving one derivative onto the test function.

Quadrature (the paper fixes none for Z_cc; this is a reading), per triangle pair:
  * near pairs (centroid distance < 4 x the longest edge of the two triangles): the outer
    integral uses the 5-point rule R5 on one triangle; the inner integral splits
    g = 1/(4 pi R) + (exp(-i k0 R) - 1)/(4 pi R), the static part and its first moment in closed
    form, the bounded remainder with R5; the entry is the average of both orderings;
  * all other pairs: the R5 x R5 product rule with the full kernel.

Closed forms over a flat triangle T for an observation point r (height d over the plane,
projection rho; per edge: tangent s, outward in-plane normal m, signed endpoint abscissae
s-/s+ relative to the foot of rho, signed distance t0 of rho to the edge line,
R0^2 = t0^2 + d^2, R-/R+ distances to the endpoints):

    int_T 1/R      = sum_edges [ t0 L - |d| (atan(t0 s+ / (R0^2 + |d| R+)) - atan(t0 s- / (R0^2 + |d| R-))) ]
    int_T (rho'-rho)/R = 1/2 sum_edges m [ R0^2 L + s+ R+ - s- R- ],   L = ln((R+ + s+) / (R- + s-)).

Because the outer rule is not exact, the two orderings of a near pair differ slightly; the
entry is their average, so Z_cc is exactly symmetric.

Parity pins (tests): closed forms against high-order numerical quadrature (off the triangle and
in-plane); self, adjacent and near entries recomputed from the RWG definitions with the inner
static integrals in polar coordinates about the foot of the outer point (1e-10); exact
reciprocity Z_cc = Z_cc^T; energy balance of a port-driven closed cavity.
"""
import numpy as np

from .quadrature import R5_BARY, R5_W, tri_points


def _log_ratio(Rp, sp, Rm, sm, R02):
    """ln((R+ + s+)/(R- + s-)) evaluated without cancellation (R + s = R0^2 / (R - s))."""
    with np.errstate(divide="ignore", invalid="ignore"):
        num = np.where(sp >= 0, np.log(Rp + sp), np.log(R02) - np.log(Rp - sp))
        den = np.where(sm >= 0, np.log(Rm + sm), np.log(R02) - np.log(Rm - sm))
        out = num - den
    return np.where(R02 > 0, out, 0.0)


def triangle_static(r, q):
    """Closed-form int_T 1/R dS' and int_T (r' - r)/R dS' for points r (P,3), triangles q (P,3,3)."""
    r = np.asarray(r, np.float64)
    q = np.asarray(q, np.float64)
    nrm = np.cross(q[:, 1] - q[:, 0], q[:, 2] - q[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    d = np.einsum("pc,pc->p", r - q[:, 0], nrm)
    ad = np.abs(d)
    rho = r - d[:, None] * nrm
    s0 = np.zeros(len(r))
    sv = np.zeros((len(r), 3))
    for a, b in ((0, 1), (1, 2), (2, 0)):
        L = q[:, b] - q[:, a]
        s_hat = L / np.linalg.norm(L, axis=1)[:, None]
        m_hat = np.cross(s_hat, nrm)
        sm = np.einsum("pc,pc->p", q[:, a] - rho, s_hat)
        sp = np.einsum("pc,pc->p", q[:, b] - rho, s_hat)
        t0 = np.einsum("pc,pc->p", q[:, a] - rho, m_hat)
        Rm = np.linalg.norm(r - q[:, a], axis=1)
        Rp = np.linalg.norm(r - q[:, b], axis=1)
        R02 = t0 * t0 + d * d
        lg = _log_ratio(Rp, sp, Rm, sm, R02)
        with np.errstate(divide="ignore", invalid="ignore"):
            at = np.where(ad > 0, np.arctan(t0 * sp / (R02 + ad * Rp)) - np.arctan(t0 * sm / (R02 + ad * Rm)), 0.0)
        s0 += np.where(t0 != 0, t0 * lg, 0.0) - ad * at
        sv += 0.5 * m_hat * (R02 * lg + sp * Rp - sm * Rm)[:, None]
    s1 = sv - (d * s0)[:, None] * nrm
    return s0, s1


def _phi(R, k):
    """(exp(-i k R) - 1) / R with its limit -i k at R = 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        v = (-2.0 * np.sin(0.5 * k * R) ** 2 - 1j * np.sin(k * R)) / R
    return np.where(R > 0, v, -1j * k)


def zcc_block(rwg_t, rwg_s, k, chunk=200000):
    """Z_cc block with rows = basis functions of rwg_t and columns = those of rwg_s.

    Assembled over all triangle pairs (testing triangle of rwg_t, source triangle of rwg_s) with
    the symmetric pair moments, then scattered into the (m_t, m_s) matrix.
    """
    Z = np.zeros((rwg_t.m, rwg_s.m), np.complex128)

    def tri_table(rwg):
        rows, loc, sg, coef = [], [], [], []
        for side, s in ((0, 1.0), (1, -1.0)):
            rows.append(np.arange(rwg.m))
            loc.append(rwg.free_local[:, side])
            sg.append(np.full(rwg.m, s))
            coef.append(rwg.tri[:, side])
        return (np.concatenate(rows), np.concatenate(loc), np.concatenate(sg), np.concatenate(coef))

    rt, lt, st, tt = tri_table(rwg_t)
    rs, ls, ss, ts = tri_table(rwg_s)
    # unique triangles used on each side
    ut = np.unique(tt)
    us = np.unique(ts)
    pa, pb = np.meshgrid(ut, us, indexing="ij")
    pa, pb = pa.ravel(), pb.ravel()
    # map (triangle_t, triangle_s) -> pair index
    pos_t = {int(t): i for i, t in enumerate(ut)}
    pos_s = {int(t): i for i, t in enumerate(us)}
    nB = np.zeros(len(pa), np.complex128)
    nA = np.zeros((len(pa), 3, 3), np.complex128)
    for s in range(0, len(pa), chunk):
        B, A = triangle_pair_moments_cross(rwg_t, rwg_s, pa[s:s + chunk], pb[s:s + chunk], k)
        nB[s:s + chunk] = B
        nA[s:s + chunk] = A
    it = np.array([pos_t[int(t)] for t in tt])
    is_ = np.array([pos_s[int(t)] for t in ts])
    rows_per = max(1, (1 << 22) // max(1, len(rs)))
    for s in range(0, len(rt), rows_per):
        I = np.arange(s, min(len(rt), s + rows_per))
        I, J = np.meshgrid(I, np.arange(len(rs)), indexing="ij")
        I, J = I.ravel(), J.ravel()
        pidx = it[I] * len(us) + is_[J]
        lm = rwg_t.length[rt[I]]
        ln = rwg_s.length[rs[J]]
        Am = rwg_t.area[tt[I]]
        An = rwg_s.area[ts[J]]
        sgn = st[I] * ss[J]
        val = sgn * (-(k * k) * lm * ln / (4.0 * Am * An) * nA[pidx, lt[I], ls[J]]
                     + lm * ln / (Am * An) * nB[pidx])
        np.add.at(Z, (rt[I], rs[J]), val)
    return Z


def triangle_pair_moments_cross(rwg_t, rwg_s, ta, tb, k):
    """Symmetric moments for triangles ta of rwg_t's mesh against tb of rwg_s's mesh."""
    va = rwg_t.verts[rwg_t.tris[ta]]
    vb = rwg_s.verts[rwg_s.tris[tb]]
    return pair_moments(va, vb, rwg_t.area[ta], rwg_s.area[tb], k)


def near_pairs(va, vb):
    """Triangle pairs whose centroid distance is below 4 x the longest edge of the pair.

    Squares are summed in a fixed order ((x^2 + y^2) + z^2) with separate roundings, so that the
    decision is reproducible by any IEEE double implementation."""
    ca = (va[:, 0] + va[:, 1] + va[:, 2]) * (1.0 / 3.0)
    cb = (vb[:, 0] + vb[:, 1] + vb[:, 2]) * (1.0 / 3.0)

    def sq(v):
        return (v[..., 0] * v[..., 0] + v[..., 1] * v[..., 1]) + v[..., 2] * v[..., 2]

    d2 = sq(ca - cb)
    e2 = np.zeros(len(va))
    for i in range(3):
        e2 = np.maximum(e2, sq(va[:, (i + 1) % 3] - va[:, i]))
        e2 = np.maximum(e2, sq(vb[:, (i + 1) % 3] - vb[:, i]))
    return d2 < 16.0 * e2


def pair_moments(va, vb, Aa, Ab, k):
    """Symmetric triangle-pair moments B = int int g, A[a,b] = int int (r-va_a).(r'-vb_b) g.

    Near pairs: average of the two orderings of the closed-form rule (_oriented). Other pairs:
    the plain R5 x R5 product rule with the full kernel (symmetric by construction)."""
    P = len(va)
    B = np.zeros(P, np.complex128)
    A = np.zeros((P, 3, 3), np.complex128)
    nr = near_pairs(va, vb)
    if nr.any():
        i = np.nonzero(nr)[0]
        B1, A1 = _oriented(va[i], vb[i], Aa[i], Ab[i], k)
        B2, A2 = _oriented(vb[i], va[i], Ab[i], Aa[i], k)
        B[i] = 0.5 * (B1 + B2)
        A[i] = 0.5 * (A1 + A2.transpose(0, 2, 1))
    if (~nr).any():
        i = np.nonzero(~nr)[0]
        B[i], A[i] = _r5r5(va[i], vb[i], Aa[i], Ab[i], k)
    return B, A


def _r5r5(va, vb, Aa, Ab, k):
    ra = tri_points(va, R5_BARY)
    rb = tri_points(vb, R5_BARY)
    R = np.linalg.norm(ra[:, :, None, :] - rb[:, None, :, :], axis=3)
    gv = np.exp(-1j * k * R) / (4.0 * np.pi * R)
    gv = gv * (R5_W[None, :, None] * Aa[:, None, None]) * (R5_W[None, None, :] * Ab[:, None, None])
    B = gv.sum((1, 2))
    pa = ra[:, :, None, :] - va[:, None, :, :]       # (P, q, a, 3)
    pb = rb[:, :, None, :] - vb[:, None, :, :]       # (P, j, b, 3)
    A = np.einsum("pqj,pqac,pjbc->pab", gv, pa, pb)
    return B, A


def _oriented(va, vb, Aa, Ab, k):
    """One ordering: outer R5 on the testing triangles va, closed-form static + R5 on the
    bounded remainder over the source triangles vb."""
    P = len(va)
    ra = tri_points(va, R5_BARY)
    rb = tri_points(vb, R5_BARY)
    s0, s1 = triangle_static(ra.reshape(-1, 3), np.repeat(vb, 5, axis=0))
    s0 = s0.reshape(P, 5)
    s1 = s1.reshape(P, 5, 3)
    R = np.linalg.norm(ra[:, :, None, :] - rb[:, None, :, :], axis=3)
    ph = _phi(R, k) * (R5_W[None, None, :] * Ab[:, None, None])
    I0 = (s0 + ph.sum(2)) / (4.0 * np.pi)
    M = (ra * s0[:, :, None] + s1 + np.einsum("pqj,pjc->pqc", ph, rb)) / (4.0 * np.pi)
    wq = R5_W[None, :] * Aa[:, None]
    B = (wq * I0).sum(1)
    rM = np.einsum("pqc,pqc->pq", ra, M)
    t_rI = np.einsum("pq,pqc->pc", wq * I0, ra)
    t_M = np.einsum("pq,pqc->pc", wq, M)
    t_I = (wq * I0).sum(1)
    A = ((wq * rM).sum(1)[:, None, None]
         - np.einsum("pc,pbc->pb", t_rI, vb)[:, None, :]
         - np.einsum("pac,pc->pa", va, t_M)[:, :, None]
         + t_I[:, None, None] * np.einsum("pac,pbc->pab", va, vb))
    return B, A
