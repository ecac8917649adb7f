"""Dense assembly of the coupled hybrid system (paper Sec. III, eq. (11) and eq. (15)).

Unknown vector (full length N = m_f + m_n + 3 n_v):
    [ j_far (m_f) | j_near (m_n) | j_body^x (n_v) | j_body^y | j_body^z ],  voxels i1 fastest.

Only tissue voxels enter the dense matrix; air voxels carry identity rows and columns.

  * assemble_direct: eq. (11) fully assembled (every block by direct quadrature).
  * assemble_same  : eq. (15) densified -- Z_cc^ff dense, Z_cc^fn = U V^* from given factors,
    the far coupling from given TT cores, the near 2x2 block as the precorrected-FFT operator
    W^T T W + corrections (eq. (13)), and the same dense volume block.

Port right-hand side (delta gap, Sec. II-A after eq. (2)): b_m = s_m i w eps0 V0 l_m for the port
edges, V0 = 1 V. Port current I = sum_m s_m l_m x_m.
"""
from dataclasses import dataclass

import numpy as np

from . import coupling, pfft, surface, tt, voxel
from .constants import chi as chi_of, k0 as k0_of, omega, row_scale
from .rwg import build_rwg, port_signs

NEAR, FAR = 0, 1


def merge(meshes, domain):
    """Concatenate the meshes of one domain (input order); port ids renumbered globally later."""
    vs, ts, pe, pid, counts = [], [], [], [], []
    off = 0
    for m in meshes:
        if m.domain != domain:
            continue
        vs.append(m.verts)
        ts.append(m.tris + off)
        pe.append(m.port_edges + off)
        pid.append(m.port_id)
        counts.append(m.n_ports)
        off += len(m.verts)
    if not vs:
        return None
    return (np.concatenate(vs), np.concatenate(ts), np.concatenate(pe).reshape(-1, 2),
            pid, counts)


@dataclass
class Disc:
    problem: object
    k: float
    h: float
    origin: np.ndarray
    n: tuple
    chi: np.ndarray          # flat (n_v,) complex, 0 in air
    tissue: np.ndarray       # flat indices of tissue voxels
    far: object              # RWG or None
    near: object
    ports: list              # list of (domain, rwg indices, signs)

    @property
    def m_f(self):
        return 0 if self.far is None else self.far.m

    @property
    def m_n(self):
        return 0 if self.near is None else self.near.m

    @property
    def n_v(self):
        return int(np.prod(self.n))

    @property
    def N(self):
        return self.m_f + self.m_n + 3 * self.n_v

    def centres(self, flat_idx):
        n1, n2, _ = self.n
        i1 = flat_idx % n1
        i2 = (flat_idx // n1) % n2
        i3 = flat_idx // (n1 * n2)
        idx = np.stack([i1, i2, i3], axis=1)
        return self.origin[None, :] + (idx + 0.5) * self.h, idx


def discretize(problem):
    g = problem.grid
    f = problem.freq_hz
    chi = chi_of(g.eps_r, g.sigma, f).ravel()
    tissue = np.nonzero(chi != 0)[0]
    far = merge(problem.meshes, FAR)
    near = merge(problem.meshes, NEAR)
    rf = build_rwg(far[0], far[1]) if far else None
    rn = build_rwg(near[0], near[1]) if near else None
    ports = []
    for dom, merged, rwg in ((FAR, far, rf), (NEAR, near, rn)):
        if merged is None:
            continue
        pe, pids, counts = merged[2], merged[3], merged[4]
        edge_pos = 0
        for pid_arr, cnt in zip(pids, counts):
            for p in range(cnt):
                sel = np.nonzero(pid_arr == p)[0] + edge_pos
                idx, sg = port_signs(rwg, pe[sel])
                ports.append((dom, idx, sg))
            edge_pos += len(pid_arr)
    return Disc(problem, k0_of(f), g.h, np.asarray(g.origin, np.float64), tuple(g.n), chi, tissue, rf, rn,
                _order_ports(problem, ports))


def _order_ports(problem, ports):
    """Ports in the order of the problem's mesh list (then port id)."""
    far_ports = [p for p in ports if p[0] == FAR]
    near_ports = [p for p in ports if p[0] == NEAR]
    out = []
    fi = ni = 0
    for mesh in problem.meshes:
        for _ in range(mesh.n_ports):
            if mesh.domain == FAR:
                out.append(far_ports[fi]); fi += 1
            else:
                out.append(near_ports[ni]); ni += 1
    return out


def port_rhs(disc, port, V0=1.0):
    """Full-length right-hand side for one port."""
    dom, idx, sg = disc.ports[port]
    b = np.zeros(disc.N, np.complex128)
    rwg = disc.far if dom == FAR else disc.near
    off = 0 if dom == FAR else disc.m_f
    b[off + idx] = sg * row_scale(disc.problem.freq_hz) * V0 * rwg.length[idx]
    return b


def port_current(disc, port, x):
    dom, idx, sg = disc.ports[port]
    rwg = disc.far if dom == FAR else disc.near
    off = 0 if dom == FAR else disc.m_f
    return np.sum(sg * rwg.length[idx] * x[off + idx])


def plane_wave_rhs(disc):
    """Body rows i w eps0 int_{V_p} E_inc for E_inc = x e^{-i k0 z} (conductor rows zero)."""
    b = np.zeros(disc.N, np.complex128)
    c, _ = disc.centres(disc.tissue)
    k, h = disc.k, disc.h
    val = h * h * np.exp(-1j * k * c[:, 2]) * (2.0 * np.sin(0.5 * k * h) / k)
    b[disc.m_f + disc.m_n + disc.tissue] = row_scale(disc.problem.freq_hz) * val
    return b


class DenseSystem:
    """Dense reduced matrix over [far | near | tissue x,y,z] with identity air rows."""

    def __init__(self, disc, Z):
        self.disc = disc
        self.Z = Z
        nt = len(disc.tissue)
        off = disc.m_f + disc.m_n
        self.red_idx = np.concatenate([np.arange(off)] + [off + a * disc.n_v + disc.tissue for a in range(3)])
        assert Z.shape == (off + 3 * nt, off + 3 * nt)

    def matvec(self, x):
        y = np.array(x, np.complex128, copy=True)      # identity on air rows
        y[self.red_idx] = self.Z @ np.asarray(x)[self.red_idx]
        return y

    def solve(self, b):
        x = np.array(b, np.complex128, copy=True)
        x[self.red_idx] = np.linalg.solve(self.Z, np.asarray(b)[self.red_idx])
        return x


def body_block(disc, table):
    """Dense Z_bb over tissue voxels: h^3 (delta/chi + T~(q - p))."""
    _, idx = disc.centres(disc.tissue)
    nt = len(idx)
    d = (idx[None, :, :] - idx[:, None, :]).reshape(-1, 3)
    Tv = voxel.T_lookup(table, d).reshape(nt, nt, 6)
    h3 = disc.h ** 3
    Z = np.zeros((3 * nt, 3 * nt), np.complex128)
    for comp, (a, b) in enumerate(voxel.COMPONENTS):
        blk = h3 * Tv[:, :, comp]
        Z[a * nt:(a + 1) * nt, b * nt:(b + 1) * nt] = blk
        if a != b:
            Z[b * nt:(b + 1) * nt, a * nt:(a + 1) * nt] = blk
    diag = h3 / disc.chi[disc.tissue]
    for a in range(3):
        Z[a * nt + np.arange(nt), a * nt + np.arange(nt)] += diag
    return Z


def generator_table(disc, extent):
    return voxel.T_generator_octant(extent, disc.k * disc.h)


def _blocks_direct(disc):
    k = disc.k
    c, _ = disc.centres(disc.tissue)
    nt = len(disc.tissue)
    out = {}
    if disc.far is not None:
        out["ff"] = surface.zcc_block(disc.far, disc.far, k)
        out["bf"] = coupling.zbc_block(c, disc.h, disc.far, k, "far").reshape(3 * nt, disc.m_f)
    if disc.near is not None:
        out["nn"] = surface.zcc_block(disc.near, disc.near, k)
        out["bn"] = coupling.zbc_block(c, disc.h, disc.near, k, "near").reshape(3 * nt, disc.m_n)
    if disc.far is not None and disc.near is not None:
        out["nf"] = surface.zcc_block(disc.near, disc.far, k)
    return out


def _compose(disc, blocks, Zbb):
    mf, mn, nt3 = disc.m_f, disc.m_n, Zbb.shape[0]
    Nr = mf + mn + nt3
    Z = np.zeros((Nr, Nr), np.complex128)
    f, n, b = slice(0, mf), slice(mf, mf + mn), slice(mf + mn, Nr)
    if "ff" in blocks:
        Z[f, f] = blocks["ff"]
        Z[b, f] = blocks["bf"]
        Z[f, b] = blocks["bf"].T
    if "nn" in blocks:
        Z[n, n] = blocks["nn"]
        Z[b, n] = blocks["bn"]
        Z[n, b] = blocks["bn"].T
    if "nf" in blocks:
        Z[n, f] = blocks["nf"]
        Z[f, n] = blocks["nf_T"] if "nf_T" in blocks else blocks["nf"].T
    Z[b, b] = Zbb
    return Z


def needed_extent(disc, bases=None):
    """Largest |offset| + 1 per axis over body-body, body-stencil and stencil-stencil pairs."""
    lo = np.zeros(3, np.int64)
    hi = np.array(disc.n, np.int64) - 1
    if bases is not None and len(bases):
        lo = np.minimum(lo, bases.min(0))
        hi = np.maximum(hi, bases.max(0) + 4)
    return tuple(int(v) for v in (hi - lo + 1))


def assemble_direct(disc, table=None):
    if table is None:
        table = generator_table(disc, tuple(disc.n))
    blocks = _blocks_direct(disc)
    return DenseSystem(disc, _compose(disc, blocks, body_block(disc, table))), blocks


def pfft_parts(disc, table, pc_dist):
    """Grid operator pieces of eq. (13): W^T T W (near-near), T W at tissue voxels, and the
    precorrection pair lists."""
    rn = disc.near
    base = pfft.stencil_bases(rn, disc.origin, disc.h)
    W = pfft.stencil_weights(rn, base, disc.origin, disc.h)        # (m, 3, 5, 5, 5)
    vox = pfft.stencil_voxels(base)                                   # (m, 125, 3)
    allv = vox.reshape(-1, 3)
    uniq, inv = np.unique(allv, axis=0, return_inverse=True)
    S = len(uniq)
    m = rn.m
    WS = np.zeros((3 * S, m))
    Wf = W.reshape(m, 3, 125)
    inv = inv.reshape(m, 125)
    for a in range(3):
        for n_ in range(m):
            WS[a * S + inv[n_], n_] += Wf[n_, a]
    h3 = disc.h ** 3

    def Tmat(rows, cols):
        d = (cols[None, :, :] - rows[:, None, :]).reshape(-1, 3)
        Tv = voxel.T_lookup(table, d).reshape(len(rows), len(cols), 6) * h3
        M = np.zeros((3 * len(rows), 3 * len(cols)), np.complex128)
        R, C = len(rows), len(cols)
        for comp, (a, b) in enumerate(voxel.COMPONENTS):
            M[a * R:(a + 1) * R, b * C:(b + 1) * C] = Tv[:, :, comp]
            if a != b:
                M[b * R:(b + 1) * R, a * C:(a + 1) * C] = Tv[:, :, comp]
        return M

    TSS = Tmat(uniq, uniq)
    WTW = WS.T @ (TSS @ WS)
    _, tidx = disc.centres(disc.tissue)
    TW = Tmat(tidx, uniq) @ WS                                          # (3 nt, m)
    pairs_nn = pfft.near_rwg_pairs(base, pc_dist)
    pairs_bn = pfft.near_voxel_rwg(base, tidx, pc_dist)
    return dict(base=base, W=W, WTW=WTW, TW=TW, pairs_nn=pairs_nn, pairs_bn=pairs_bn)


def assemble_same(disc, tt_cores=None, aca=None, pc_dist=2, table=None, direct_blocks=None):
    """The hybrid operator of eq. (15) as a dense matrix.

    tt_cores: list over chi of [G1, G2, G3, G4] for the far coupling (full box tensors);
    aca: (U, V) with Z_cc^fn ~ U V^*.
    """
    if direct_blocks is None:
        direct_blocks = _blocks_direct(disc)
    blocks = dict(direct_blocks)
    bases = None
    parts = None
    if disc.near is not None:
        bases = pfft.stencil_bases(disc.near, disc.origin, disc.h)
    ext = needed_extent(disc, bases)
    if table is None or any(table.shape[2 - i] < ext[i] for i in range(3)):
        table = generator_table(disc, ext)
    if disc.near is not None:
        parts = pfft_parts(disc, table, pc_dist)
        nn = parts["WTW"].copy()
        i, j = parts["pairs_nn"]
        nn[i, j] = direct_blocks["nn"][i, j]
        blocks["nn"] = nn
        bn = parts["TW"].copy()
        p, n_ = parts["pairs_bn"]
        nt = len(disc.tissue)
        for a in range(3):
            bn[a * nt + p, n_] = direct_blocks["bn"][a * nt + p, n_]
        blocks["bn"] = bn
    if disc.far is not None:
        if tt_cores is not None:
            nt = len(disc.tissue)
            bf = np.zeros((3 * nt, disc.m_f), np.complex128)
            for a in range(3):
                A = tt.tt_full(tt_cores[a])                      # (n1, n2, n3, m_f)
                flat = A.transpose(2, 1, 0, 3).reshape(-1, disc.m_f)
                bf[a * nt:(a + 1) * nt] = flat[disc.tissue]
            blocks["bf"] = bf
        if aca is not None and disc.near is not None:
            U, V = aca
            blocks["nf"] = U @ V.conj().T
            blocks["nf_T"] = V.conj() @ U.T
    Zbb = body_block(disc, table)
    return DenseSystem(disc, _compose(disc, blocks, Zbb)), blocks, parts


def far_coupling_tensor(disc, chi_comp):
    """Brute-force far coupling over the full box for one component: (n1, n2, n3, m_f)."""
    allv = np.arange(disc.n_v)
    c, _ = disc.centres(allv)
    blk = coupling.zbc_block(c, disc.h, disc.far, disc.k, "far")[chi_comp]
    return tt.tt_tensor_from_block(blk, disc.n)
