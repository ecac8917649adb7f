"""Triangle meshes of conductors: strip loops (flat or conformal to a cylinder) and cylindrical
shields (closed with capped ends, or an open tube).

Every mesh is consistently oriented (each interior edge is listed once in each direction by its
two triangles). Ports are cuts across a strip: a list of directed interior edges ``(a, b)`` that
share a port id; positive port current flows out of the triangle listing ``a`` then ``b``.
"""
from dataclasses import dataclass, field

import numpy as np

NEAR = 0
FAR = 1


@dataclass
class Mesh:
    verts: np.ndarray            # float64 [nv, 3]
    tris: np.ndarray             # int32 [nt, 3]
    domain: int = NEAR           # NEAR (pFFT) or FAR (TT / ACA / dense)
    port_edges: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    port_id: np.ndarray = field(default_factory=lambda: np.zeros((0,), np.int32))

    @property
    def n_ports(self):
        return int(self.port_id.max()) + 1 if len(self.port_id) else 0


def _grid_lines(length, width, step):
    """Parameter lines across a frame side: [0, w/2, w, ..uniform.., L-w, L-w/2, L]."""
    inner = length - 2.0 * width
    k = max(1, int(round(inner / step)))
    mid = width + inner * np.arange(k + 1) / k
    return np.concatenate([[0.0, 0.5 * width], mid, [length - 0.5 * width, length]])


def _frame(W, H, w, step):
    """Conforming triangulation of the rectangular frame [0,W]x[0,H] minus (w,W-w)x(w,H-w).

    Returns parameter-plane vertices (u, v), CCW triangles, and the index grid of vertices.
    """
    us = _grid_lines(W, w, step)
    vs = _grid_lines(H, w, step)
    nu, nv = len(us), len(vs)
    vid = -np.ones((nu, nv), np.int64)
    pts, tris = [], []

    def vertex(i, j):
        if vid[i, j] < 0:
            vid[i, j] = len(pts)
            pts.append((us[i], vs[j]))
        return vid[i, j]

    for i in range(nu - 1):
        for j in range(nv - 1):
            uc = 0.5 * (us[i] + us[i + 1])
            vc = 0.5 * (vs[j] + vs[j + 1])
            if w < uc < W - w and w < vc < H - w:
                continue
            a, b = vertex(i, j), vertex(i + 1, j)
            c, d = vertex(i + 1, j + 1), vertex(i, j + 1)
            if (i + j) % 2 == 0:
                tris += [(a, b, c), (a, c, d)]
            else:
                tris += [(a, b, d), (b, c, d)]
    return np.array(pts), np.array(tris, np.int32), vid, us, vs


def _frame_port(vid, us, n_across=2):
    """Directed edges of the cut across the bottom side (v in [0, w]) at the middle u line.

    The cut runs from the outer edge inward; orienting each edge (lower v -> higher v) makes the
    cell on its left (lower u) the triangle that lists a then b, so positive current flows +u.
    """
    i = len(us) // 2
    edges = [(vid[i, j], vid[i, j + 1]) for j in range(n_across)]
    return np.array(edges, np.int32)


def strip_loop_flat(centre, side=60e-3, width=5e-3, step=5e-3, port_id=0):
    """Square strip loop in the plane x = centre[0], edges along y and z, one delta-gap port."""
    pts, tris, vid, us, vs = _frame(side, side, width, step)
    c = np.asarray(centre, np.float64)
    verts = np.stack([np.full(len(pts), c[0]), c[1] - 0.5 * side + pts[:, 0],
                      c[2] - 0.5 * side + pts[:, 1]], axis=1)
    pe = _frame_port(vid, us)
    return Mesh(verts, tris, NEAR, pe, np.full(len(pe), port_id, np.int32))


def strip_loop_on_cylinder(radius, phi0, arc, z0, length, width=5e-3, step=2e-3, port_id=0):
    """Rectangular strip loop conformal to a cylinder of the given radius (axis = z).

    The loop spans azimuth [phi0, phi0 + arc/radius] and z in [z0, z0 + length]."""
    pts, tris, vid, us, vs = _frame(arc, length, width, step)
    phi = phi0 + pts[:, 0] / radius
    verts = np.stack([radius * np.cos(phi), radius * np.sin(phi), z0 + pts[:, 1]], axis=1)
    pe = _frame_port(vid, us)
    return Mesh(verts, tris, NEAR, pe, np.full(len(pe), port_id, np.int32))


def loop_array(n_loops=8, radius=0.12, length=0.1, gap=10e-3, width=5e-3, step=2e-3, z_centre=0.0,
               phi_offset=0.0):
    """n_loops conformal strip loops evenly pitched around a cylinder, one port each, one mesh."""
    pitch = 2.0 * np.pi * radius / n_loops
    arc = pitch - gap
    verts, tris, pe, pid = [], [], [], []
    off = 0
    for k in range(n_loops):
        phi0 = phi_offset + 2.0 * np.pi * k / n_loops + 0.5 * gap / radius
        m = strip_loop_on_cylinder(radius, phi0, arc, z_centre - 0.5 * length, length, width, step, k)
        verts.append(m.verts)
        tris.append(m.tris + off)
        pe.append(m.port_edges + off)
        pid.append(m.port_id)
        off += len(m.verts)
    return Mesh(np.concatenate(verts), np.concatenate(tris).astype(np.int32), NEAR,
                np.concatenate(pe).astype(np.int32), np.concatenate(pid).astype(np.int32))


def cylinder_shield(radius, length, n_around, n_along, closed=True, cap_rings=3, z_centre=0.0,
                    phi_offset=0.0):
    """Cylindrical PEC shield around the z axis, outward-oriented; closed with flat caps or open."""
    phi = phi_offset + 2.0 * np.pi * np.arange(n_around) / n_around
    zs = z_centre - 0.5 * length + length * np.arange(n_along + 1) / n_along
    verts = []
    side = np.zeros((n_along + 1, n_around), np.int64)
    for j, z in enumerate(zs):
        for i, p in enumerate(phi):
            side[j, i] = len(verts)
            verts.append((radius * np.cos(p), radius * np.sin(p), z))
    tris = []
    for j in range(n_along):
        for i in range(n_around):
            i2 = (i + 1) % n_around
            a, b, c, d = side[j, i], side[j, i2], side[j + 1, i2], side[j + 1, i]
            if (i + j) % 2 == 0:
                tris += [(a, b, c), (a, c, d)]
            else:
                tris += [(a, b, d), (b, c, d)]
    if closed:
        for end, z in ((0, zs[0]), (n_along, zs[-1])):
            rings = [side[end]]
            for k in range(cap_rings - 1, 0, -1):
                r = radius * k / cap_rings
                ids = []
                for p in phi:
                    ids.append(len(verts))
                    verts.append((r * np.cos(p), r * np.sin(p), z))
                rings.append(np.array(ids))
            centre = len(verts)
            verts.append((0.0, 0.0, z))
            top = end != 0
            for k in range(len(rings) - 1):
                o, n = rings[k], rings[k + 1]
                for i in range(n_around):
                    i2 = (i + 1) % n_around
                    if top:   # outward normal +z: counter-clockwise seen from above
                        tris += [(o[i], o[i2], n[i2]), (o[i], n[i2], n[i])]
                    else:
                        tris += [(o[i2], o[i], n[i]), (o[i2], n[i], n[i2])]
            last = rings[-1]
            for i in range(n_around):
                i2 = (i + 1) % n_around
                tris.append((last[i], last[i2], centre) if top else (last[i2], last[i], centre))
    return Mesh(np.array(verts, np.float64), np.array(tris, np.int32), FAR)
