"""Rao-Wilton-Glisson basis functions on triangle meshes (paper Sec. II-B).

One basis function per interior edge (an edge shared by exactly two triangles). Ordering: edges
sorted by (min vertex, max vertex). For edge (a, b) with a < b, T+ is the triangle listing a then
b in cyclic order and T- the one listing b then a; f = l/(2 A+) (r - p+) on T+ and
l/(2 A-) (p- - r) on T-, div f = +l/A+ on T+ and -l/A- on T-.

Port excitation (delta gap, Sec. II-A after eq. (2)): a port edge (a, b) carries unit voltage;
positive current leaves the triangle listing a then b, so the basis function's sign relative to
the port is +1 when a < b and -1 otherwise.

Parity: pinned indirectly (PEC/loop physics tests, reciprocity of Z_cc).
"""
from dataclasses import dataclass

import numpy as np


class MeshError(ValueError):
    pass


@dataclass
class RWG:
    edge: np.ndarray        # (m, 2) vertex ids a < b
    tri: np.ndarray         # (m, 2) triangle ids [T+, T-]
    free: np.ndarray        # (m, 2) free-vertex ids [p+, p-]
    free_local: np.ndarray  # (m, 2) local index (0..2) of the free vertex inside T+/T-
    length: np.ndarray      # (m,)
    verts: np.ndarray
    tris: np.ndarray
    area: np.ndarray        # per triangle

    @property
    def m(self):
        return len(self.length)


def build_rwg(verts, tris):
    verts = np.asarray(verts, np.float64)
    tris = np.asarray(tris, np.int64)
    directed = {}
    for t, (i, j, k) in enumerate(tris):
        for a, b, fl in ((i, j, 2), (j, k, 0), (k, i, 1)):
            key = (int(a), int(b))
            if key in directed:
                raise MeshError("inconsistent orientation or non-manifold edge %s" % (key,))
            directed[key] = (t, fl)
    edges = []
    for (a, b), (t, fl) in directed.items():
        if a < b and (b, a) in directed:
            tm, flm = directed[(b, a)]
            edges.append((a, b, t, tm, fl, flm))
    edges.sort()
    e = np.array(edges, np.int64).reshape(-1, 6)
    v = verts
    cr = np.cross(v[tris[:, 1]] - v[tris[:, 0]], v[tris[:, 2]] - v[tris[:, 0]])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    if np.any(area <= 0):
        raise MeshError("degenerate triangle")
    free = np.stack([tris[e[:, 2], e[:, 4]], tris[e[:, 3], e[:, 5]]], axis=1)
    length = np.linalg.norm(v[e[:, 1]] - v[e[:, 0]], axis=1)
    return RWG(e[:, :2], e[:, 2:4], free, e[:, 4:6], length, v, tris, area)


def port_signs(rwg, port_edges):
    """Indices into the RWG list and +/-1 signs for directed port edges (a, b)."""
    lookup = {(int(a), int(b)): i for i, (a, b) in enumerate(rwg.edge)}
    idx, sgn = [], []
    for a, b in np.asarray(port_edges, np.int64).reshape(-1, 2):
        key = (min(a, b), max(a, b))
        if key not in lookup:
            raise MeshError("port edge %s is not an interior edge" % (key,))
        idx.append(lookup[key])
        sgn.append(1.0 if a < b else -1.0)
    return np.array(idx, np.int64), np.array(sgn)
