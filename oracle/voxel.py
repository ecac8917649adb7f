"""Galerkin interaction integrals between piecewise-constant voxel currents.

Paper Sec. II-B: the volume operator of eq. (4)-(5) discretised with PWC basis functions on a
uniform grid (q = 3); its matrix is multilevel block-Toeplitz, i.e. every entry depends only on
the voxel offset d = q - p.

With every row multiplied by i w eps0 and the field equation divided by chi, the entry for
voxel p, component alpha against voxel q, component beta is

    Z_bb[p a, q b] = dv * delta_pq delta_ab / chi_p - k0^2 delta_ab I_vv(d) + I_ff^{ab}(d)

    I_vv(d)     = int_{V_p} int_{V_q} g(r - r')                                (vector potential)
    I_ff^{ab}(d) = oint_{dV_p} oint_{dV_q} g(r - r') n_a(r) n'_b(r')           (face charges)

The face term follows from nabla nabla . acting on a PWC current: its divergence is a surface
charge on voxel faces; integrating by parts on both sides gives the face-face integral. With all
lengths in units of h, kappa = k0 h, and K(rho) = exp(-i kappa rho) / (4 pi rho):

  * the convolution of two unit boxes is the tent (1 - |t|) per axis, so
        I_vv(d) = h^5 V(d),   V(d) = int_{[-1,1]^3} K(|t + d|) prod (1 - |t_i|) dt;
  * two parallel faces normal to axis a reduce to a 2D tent integral
        F2(s; e) = int_{[-1,1]^2} K(sqrt(s^2 + |t + e|^2)) prod (1 - |t_i|) dt,
    and summing the four face pairs with their normal signs gives a second difference
        I_ff^{aa}(d) = h^3 [2 F2(d_a) - F2(d_a - 1) - F2(d_a + 1)]   (e = the other two d's);
  * two perpendicular faces (normals a != b) share the third axis c, which reduces to a tent:
        G(m, n; d_c) = int_m^{m+1} dX int_n^{n+1} dY int_{-1}^{1} (1-|t|) K(sqrt(X^2+Y^2+(t-d_c)^2))
        I_ff^{ab}(d) = -h^3 [G(d_a, d_b) - G(d_a-1, d_b) - G(d_a, d_b-1) + G(d_a-1, d_b-1)].

Quadrature (no rule is given in the paper; the integrals are converged to ~1e-15 so that two
independent codes agree): every domain is a union of unit cells. A cell that has the singular
point at a corner is mapped with the Duffy transform (pyramids for 3D, triangles for 2D), which
cancels the 1/rho singularity, then integrated with 12-point Gauss-Legendre per direction. Every
other cell lies at least one cell away from the singular point and is integrated with a tensor
Gauss-Legendre rule whose order follows from the Bernstein-ellipse bound for that distance.

Parity pins (tests): the trace identity sum_a I_ff^{aa} = k0^2 I_vv + dv delta_{d0} (exact), the
6D/4D brute-force definitions at separated offsets, an independent tanh-sinh evaluation of the
singular self terms, the off-diagonal face terms at every touching offset d in {0, 1}^3 from the
closed-form potential of a rectangle integrated by a double-exponential rule (1e-10), and
convergence in the quadrature order.
"""
import numpy as np

from .quadrature import gauss01

COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))   # xx yy zz xy xz yz


def _bernstein_order(dist, digits=17.0, nmin=3, nmax=16):
    """Gauss order per direction for a unit cell at distance `dist` (cells) from the singularity.

    Worst case is a singularity at distance D perpendicular to the cell's end: in the cell's
    [-1,1] coordinate it sits at z = -1 + 2 D i; Gauss error decays like rho^(-2N) with rho the
    Bernstein ellipse parameter through z.
    """
    z = -1.0 + 2.0j * np.asarray(dist, dtype=np.float64)
    s = np.sqrt(z * z - 1.0)
    rho = np.maximum(np.abs(z + s), np.abs(z - s))
    n = np.ceil(digits * np.log(10.0) / (2.0 * np.log(rho)))
    return np.clip(n, nmin, nmax).astype(np.int64)


def _kernel(r, kappa):
    return np.exp(-1j * kappa * r) / (4.0 * np.pi * r)


def _tent(x, tent):
    w = np.ones(x.shape[:-1])
    for i, t in enumerate(tent):
        if t:
            w = w * (1.0 - np.abs(x[..., i]))
    return w


def _tensor_nodes(n, dim):
    x, w = gauss01(n)
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    wgrids = np.meshgrid(*([w] * dim), indexing="ij")
    nodes = np.stack([g.ravel() for g in grids], axis=1)
    wt = np.prod(np.stack([g.ravel() for g in wgrids], axis=1), axis=1)
    return nodes, wt


def _duffy_nodes(n, dim):
    """Nodes y in [0,1]^dim (singular corner at 0) and weights (including the Jacobian) of the
    Duffy map: one pyramid (3D) or triangle (2D) per principal axis."""
    x, w = gauss01(n)
    nodes, wts = [], []
    if dim == 3:
        t, u, v = np.meshgrid(x, x, x, indexing="ij")
        wt = np.einsum("i,j,k->ijk", w, w, w)
        t, u, v, wt = t.ravel(), u.ravel(), v.ravel(), wt.ravel()
        for j in range(3):
            y = np.empty((t.size, 3))
            others = [k for k in range(3) if k != j]
            y[:, j] = t
            y[:, others[0]] = t * u
            y[:, others[1]] = t * v
            nodes.append(y)
            wts.append(wt * t * t)
    else:
        t, u = np.meshgrid(x, x, indexing="ij")
        wt = np.einsum("i,j->ij", w, w).ravel()
        t, u = t.ravel(), u.ravel()
        for j in range(2):
            y = np.empty((t.size, 2))
            y[:, j] = t
            y[:, 1 - j] = t * u
            nodes.append(y)
            wts.append(wt * t)
    return np.concatenate(nodes), np.concatenate(wts)


def cell_integrals(lo, c, delta, tent, kappa, n_sing=12, chunk_points=1 << 22):
    """Integrals over unit cells [lo, lo+1]^D of K(sqrt(|x - c|^2 + delta^2)) * prod w_i(x_i).

    lo, c: (P, D) arrays; delta: (P,) array; tent[i] says whether axis i carries (1 - |x_i|).
    A cell is singular when the point (c, delta) touches it; c must then be one of its corners.
    """
    lo = np.asarray(lo, np.float64)
    c = np.asarray(c, np.float64)
    delta = np.asarray(delta, np.float64)
    P, D = lo.shape
    gap = np.maximum(np.maximum(lo - c, c - lo - 1.0), 0.0)
    dist = np.sqrt((gap ** 2).sum(1) + delta ** 2)
    out = np.zeros(P, np.complex128)

    sing = dist == 0.0
    if sing.any():
        idx = np.nonzero(sing)[0]
        cl, cc = lo[idx], c[idx]
        at_lo = cc == cl
        at_hi = cc == cl + 1.0
        if not np.all(at_lo | at_hi):
            raise ValueError("singular point must be a cell corner")
        sigma = np.where(at_lo, 1.0, -1.0)
        y, wy = _duffy_nodes(n_sing, D)
        per = max(1, chunk_points // len(wy))
        for s in range(0, len(idx), per):
            sl = slice(s, s + per)
            x = cc[sl, None, :] + sigma[sl, None, :] * y[None, :, :]
            r = np.sqrt((y ** 2).sum(1))[None, :]
            f = _kernel(r, kappa) * _tent(x, tent) * wy[None, :]
            out[idx[sl]] = f.sum(1)

    reg = ~sing
    if reg.any():
        ridx = np.nonzero(reg)[0]
        order = _bernstein_order(dist[ridx])
        for n in np.unique(order):
            idx = ridx[order == n]
            nodes, wt = _tensor_nodes(int(n), D)
            per = max(1, chunk_points // len(wt))
            for s in range(0, len(idx), per):
                ii = idx[s:s + per]
                x = lo[ii, None, :] + nodes[None, :, :]
                r = np.sqrt(((x - c[ii, None, :]) ** 2).sum(2) + delta[ii, None] ** 2)
                f = _kernel(r, kappa) * _tent(x, tent) * wt[None, :]
                out[ii] = f.sum(1)
    return out


def V_integral(d, kappa):
    """V(d) = int_{[-1,1]^3} K(|t + d|) prod(1 - |t_i|) dt for integer offsets d (P, 3)."""
    d = np.asarray(d, np.float64).reshape(-1, 3)
    corners = np.array([[a, b, e] for e in (-1, 0) for b in (-1, 0) for a in (-1, 0)], np.float64)
    P = len(d)
    lo = np.repeat(corners[None], P, 0).reshape(-1, 3)
    c = np.repeat(-d, 8, 0)
    vals = cell_integrals(lo, c, np.zeros(len(lo)), (True, True, True), kappa)
    return vals.reshape(P, 8).sum(1)


def F2_integral(s, e, kappa):
    """F2(s; e) = int_{[-1,1]^2} K(sqrt(s^2 + |t + e|^2)) prod(1-|t_i|) dt; s (P,), e (P, 2)."""
    s = np.asarray(s, np.float64).ravel()
    e = np.asarray(e, np.float64).reshape(-1, 2)
    corners = np.array([[a, b] for b in (-1, 0) for a in (-1, 0)], np.float64)
    P = len(s)
    lo = np.repeat(corners[None], P, 0).reshape(-1, 2)
    c = np.repeat(-e, 4, 0)
    dl = np.repeat(np.abs(s), 4)
    vals = cell_integrals(lo, c, dl, (True, True), kappa)
    return vals.reshape(P, 4).sum(1)


def G_integral(m, n, dc, kappa):
    """G(m, n; dc) = int_m^{m+1} dX int_n^{n+1} dY int_{-1}^{1} (1-|t|) K(|(X, Y, t - dc)|) dt."""
    m = np.asarray(m, np.float64).ravel()
    n = np.asarray(n, np.float64).ravel()
    dc = np.asarray(dc, np.float64).ravel()
    P = len(m)
    lo = np.zeros((P, 2, 3))
    lo[:, :, 0] = m[:, None]
    lo[:, :, 1] = n[:, None]
    lo[:, 0, 2] = -1.0
    lo[:, 1, 2] = 0.0
    c = np.zeros((P, 2, 3))
    c[:, :, 2] = dc[:, None]
    vals = cell_integrals(lo.reshape(-1, 3), c.reshape(-1, 3), np.zeros(2 * P),
                          (False, False, True), kappa)
    return vals.reshape(P, 2).sum(1)


def face_integrals(d, kappa):
    """Dimensionless I_ff^{ab}(d) / h^3 for the six components (P, 6) in COMPONENTS order."""
    d = np.asarray(d, np.float64).reshape(-1, 3)
    P = len(d)
    out = np.zeros((P, 6), np.complex128)
    for a in range(3):
        oth = [k for k in range(3) if k != a]
        e = d[:, oth]
        f0 = F2_integral(d[:, a], e, kappa)
        fm = F2_integral(d[:, a] - 1.0, e, kappa)
        fp = F2_integral(d[:, a] + 1.0, e, kappa)
        out[:, a] = 2.0 * f0 - fm - fp
    for comp, (a, b) in enumerate(COMPONENTS[3:], start=3):
        c = 3 - a - b
        da, db, dc = d[:, a], d[:, b], d[:, c]
        g00 = G_integral(da, db, dc, kappa)
        g10 = G_integral(da - 1.0, db, dc, kappa)
        g01 = G_integral(da, db - 1.0, dc, kappa)
        g11 = G_integral(da - 1.0, db - 1.0, dc, kappa)
        out[:, comp] = -(g00 - g10 - g01 + g11)
    return out


def T_generator(d, kappa):
    """Dimensionless Toeplitz generator T~_ab(d) = -kappa^2 delta_ab V(d) + I_ff^{ab}(d)/h^3.

    The physical Galerkin matrix of the volume operator (without the 1/chi diagonal) is
    h^3 * T~(q - p). Returns (P, 6) in COMPONENTS order.
    """
    d = np.asarray(d, np.float64).reshape(-1, 3)
    t = face_integrals(d, kappa)
    v = V_integral(d, kappa)
    t[:, :3] -= (kappa ** 2) * v[:, None]
    return t


def T_generator_octant(extent, kappa):
    """T~ on all offsets d with 0 <= d_i < extent_i, shape (e3, e2, e1, 6)."""
    e1, e2, e3 = extent
    z, y, x = np.meshgrid(np.arange(e3), np.arange(e2), np.arange(e1), indexing="ij")
    d = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    return T_generator(d, kappa).reshape(e3, e2, e1, 6)


def T_lookup(octant, d):
    """T~ at arbitrary integer offsets d (P, 3) from an octant table using the exact parities:
    diagonal components are even in every axis; component ab (a != b) is odd in d_a and d_b."""
    d = np.asarray(d, np.int64).reshape(-1, 3)
    ad = np.abs(d)
    vals = octant[ad[:, 2], ad[:, 1], ad[:, 0]].copy()
    sg = np.sign(d)
    for comp, (a, b) in enumerate(COMPONENTS[3:], start=3):
        vals[:, comp] *= sg[:, a] * sg[:, b]
    return vals
