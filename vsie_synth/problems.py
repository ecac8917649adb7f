"""Named problem instances: voxel grid + conductor meshes + frequency.

  * ``tiny_case``  : 16^3 voxels at 5 mm, homogeneous sphere r = 35 mm (eps_r 52, sigma 0.55),
                     one 60 mm square strip loop about 10 mm from the sphere (near, one port),
                     closed cylindrical shield r = 150 mm, L = 300 mm, 2000 triangles (far).
  * ``small_case`` : a scaled-down variant of the same layout for quick tests.
  * ``two_mm_case``: 96x112x128 voxels at 2 mm, head-like phantom (seed 0), eight conformal
                     loops on a 120 mm cylinder (near, eight ports), open tube shield
                     r = 340 mm, L = 1.2 m, about 20k triangles (far).
  * ``one_mm_case``: 192x224x256 voxels at 1 mm, head-like phantom (seed 7), 32 loops in two rings
                     of 16 (near, 32 ports), the same shield meshed with about 40k triangles (far).
  * ``mie_case``   : the sphere alone (plane-wave excitation is built by the consumer).
"""
from dataclasses import dataclass, field

import numpy as np

from .meshes import FAR, NEAR, cylinder_shield, loop_array, strip_loop_flat
from .phantoms import Grid, head_phantom, sphere_phantom

LARMOR_7T_HZ = 297.2e6


@dataclass
class Problem:
    grid: Grid
    meshes: list = field(default_factory=list)
    freq_hz: float = LARMOR_7T_HZ
    name: str = ""

    def n_ports(self):
        return sum(m.n_ports for m in self.meshes)


def tiny_case():
    g = sphere_phantom((16, 16, 16), 5e-3, 35e-3, 52.0, 0.55)
    # small offsets keep RWG edge midpoints off voxel faces (stencil base selection is a floor)
    loop = strip_loop_flat((45.5e-3, 0.37e-3, -0.41e-3), side=60e-3, width=5e-3, step=5e-3)
    shield = cylinder_shield(0.150, 0.300, 40, 20, closed=True, cap_rings=3)
    return Problem(g, [shield, loop], LARMOR_7T_HZ, "tiny")


def small_case(n=8, shield_around=12, shield_along=6):
    """8^3 voxels at 5 mm, sphere r = 17 mm, 30 mm loop, coarse closed shield (fast tests)."""
    g = sphere_phantom((n, n, n), 5e-3, 17e-3, 52.0, 0.55)
    loop = strip_loop_flat((25.5e-3, 0.37e-3, -0.41e-3), side=30e-3, width=5e-3, step=5e-3)
    shield = cylinder_shield(0.080, 0.160, shield_around, shield_along, closed=True, cap_rings=2)
    return Problem(g, [shield, loop], LARMOR_7T_HZ, "small")


def two_mm_case(seed=0, n=(96, 112, 128), h=2e-3, n_loops=8, shield_around=128, shield_along=78):
    g = head_phantom(seed, n, h)
    coil = loop_array(n_loops, radius=0.12, length=0.1, gap=10e-3, width=5e-3, step=2e-3,
                      z_centre=0.37e-3, phi_offset=0.0013)
    shield = cylinder_shield(0.340, 1.2, shield_around, shield_along, closed=False)
    return Problem(g, [shield, coil], LARMOR_7T_HZ, "2mm")


def one_mm_case(seed=7, n=(192, 224, 256), h=1e-3, loops_per_ring=16, shield_around=180, shield_along=111):
    """192x224x256 voxels at 1 mm, head-like phantom (seed 7), 32 conformal loops in two rings of 16
    on the 120 mm cylinder (4 mm strips meshed at 1 mm along and 2 mm across, so that every RWG pair
    fits its 5x5x5 pFFT block at h = 1 mm), open tube shield r = 340 mm, L = 1.2 m, about 40k
    triangles."""
    from .meshes import Mesh
    g = head_phantom(seed, n, h)
    rings = [loop_array(loops_per_ring, radius=0.12, length=0.1, gap=10e-3, width=4e-3, step=1e-3,
                        z_centre=zc, phi_offset=0.0013 + 0.5 * ring * 2 * np.pi / loops_per_ring)
             for ring, zc in enumerate((-55.37e-3, 55.37e-3))]
    nv0 = len(rings[0].verts)
    coil = Mesh(np.concatenate([r.verts for r in rings]),
                np.concatenate([rings[0].tris, rings[1].tris + nv0]).astype(np.int32), NEAR,
                np.concatenate([rings[0].port_edges, rings[1].port_edges + nv0]).astype(np.int32),
                np.concatenate([rings[0].port_id, rings[1].port_id + rings[0].n_ports]).astype(np.int32))
    shield = cylinder_shield(0.340, 1.2, shield_around, shield_along, closed=False)
    return Problem(g, [shield, coil], LARMOR_7T_HZ, "1mm")


def uneven_phantom_set(h=2e-3):
    """Six head-like phantoms of uneven grids at 2 mm inside one shared open shield (r = 340 mm,
    L = 1.2 m, about 20k triangles, the same mesh object for all): 48^3 (seed 10), 64x72x80 (11),
    80x96x96 (12), 96x112x128 (13 and 14), 112x128x144 (15); loop arrays of 8, 8, 16, 16, 16 and 32
    (two rings of 16) channels on a cylinder 20 mm outside the larger in-plane half-extent (at least
    120 mm)."""
    from .meshes import Mesh
    shield = cylinder_shield(0.340, 1.2, 128, 78, closed=False)
    spec = [((48, 48, 48), 10, 8), ((64, 72, 80), 11, 8), ((80, 96, 96), 12, 16), ((96, 112, 128), 13, 16),
            ((96, 112, 128), 14, 16), ((112, 128, 144), 15, 32)]
    out = []
    for n, seed, nl in spec:
        g = head_phantom(seed, n, h)
        radius = max(0.12, 0.5 * max(n[0], n[1]) * h + 0.02)
        if nl <= 16:
            coil = loop_array(nl, radius=radius, length=0.1, gap=10e-3, width=5e-3, step=2e-3, z_centre=0.37e-3,
                              phi_offset=0.0013)
        else:
            rings = [loop_array(16, radius=radius, length=0.1, gap=10e-3, width=5e-3, step=2e-3, z_centre=zc,
                                phi_offset=0.0013 + 0.5 * ring * 2 * np.pi / 16)
                     for ring, zc in enumerate((-55.37e-3, 55.37e-3))]
            nv0 = len(rings[0].verts)
            coil = Mesh(np.concatenate([r.verts for r in rings]),
                        np.concatenate([rings[0].tris, rings[1].tris + nv0]).astype(np.int32), NEAR,
                        np.concatenate([rings[0].port_edges, rings[1].port_edges + nv0]).astype(np.int32),
                        np.concatenate([rings[0].port_id, rings[1].port_id + rings[0].n_ports]).astype(np.int32))
        out.append(Problem(g, [shield, coil], LARMOR_7T_HZ, "%dx%dx%d" % n))
    return out


def mie_case(n=16, h=5e-3, radius=35e-3):
    return Problem(sphere_phantom((n, n, n), h, radius, 52.0, 0.55), [], LARMOR_7T_HZ, "mie")


__all__ = ["Problem", "tiny_case", "small_case", "two_mm_case", "one_mm_case", "uneven_phantom_set", "mie_case",
           "NEAR", "FAR", "LARMOR_7T_HZ"]
