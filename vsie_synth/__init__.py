"""Seeded synthetic inputs for the hybrid VSIE: voxel phantoms, conductor meshes, test vectors.

This package holds no electromagnetic arithmetic. It only builds geometry (voxel grids with
material maps, triangle meshes with port edges) and random vectors, so that the CPU oracle and
the GPU library can be driven with identical inputs. Everything is deterministic in its seed
(numpy PCG64).

Conventions shared by every consumer:
  * lengths in metres, frequency in Hz, conductivity in S/m;
  * a voxel grid is ``n = (n1, n2, n3)`` voxels of edge ``h`` whose lower corner is ``origin``;
    voxel ``(i1, i2, i3)`` spans ``origin + [i, i+1) * h`` and flat index ``i1 + n1*(i2 + n2*i3)``
    (i1 fastest); material arrays are numpy arrays of shape ``(n3, n2, n1)``;
  * a mesh is ``verts`` (float64, [nv, 3]) and ``tris`` (int32, [nt, 3]) with a consistent
    orientation; ports are directed vertex pairs ``(a, b)`` of interior edges plus a port id;
    positive port current flows out of the triangle that lists ``a`` then ``b`` in cyclic order.
"""
from .phantoms import Grid, sphere_phantom, head_phantom, random_block
from .meshes import Mesh, strip_loop_flat, strip_loop_on_cylinder, loop_array, cylinder_shield
from .vectors import complex_normal
from .problems import Problem, tiny_case, two_mm_case, one_mm_case, small_case, mie_case, uneven_phantom_set

__all__ = [
    "Grid", "sphere_phantom", "head_phantom", "random_block", "Mesh", "strip_loop_flat", "strip_loop_on_cylinder",
    "loop_array", "cylinder_shield", "complex_normal", "Problem", "tiny_case", "two_mm_case",
    "small_case", "mie_case", "one_mm_case", "uneven_phantom_set",
]
