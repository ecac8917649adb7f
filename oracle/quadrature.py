"""Quadrature rules used by the oracle.

  * Gauss-Legendre on [0, 1] (numpy's leggauss, a library primitive).
  * The 5-point triangle rule R5 that defines the "5 surface points" of the coupling integrals
    (paper Sec. IV-C). The paper names only the point count. This rule is exact for polynomials
    of total degree <= 3, has positive weights and is mirror-symmetric about the median through
    the first vertex. Its values are fixed here and in the GPU library alike because the rule is
    part of the operator's definition. Pinned by an exactness test.
  * 2x2x2 Gauss-Legendre in a voxel: the "8 volume points" of the same passage.
  * A collapsed (Duffy) Gauss product rule on the triangle for exact integration of
    polynomials (pFFT projection weights).
"""
import numpy as np

# barycentric coordinates (l1, l2, l3) and weights as fractions of the triangle area
R5_BARY = np.array([
    [1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0],
    [0.66, 0.17, 0.17],
    [0.082832331329325317301, 0.45858383433533734135, 0.45858383433533734135],
    [0.2, 0.70704891655600176715, 0.092951083443998232846],
    [0.2, 0.092951083443998232846, 0.70704891655600176715],
])
R5_W = np.array([0.03, 0.33127923434407885754, 0.19677027567856090582,
                 0.22097524498868011832, 0.22097524498868011832])


def gauss01(n):
    """n-point Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def tri_points(v, bary):
    """Points of a rule on triangles v (..., 3 vertices, 3 coords) -> (..., npts, 3)."""
    return np.einsum("qk,...kc->...qc", bary, v)


def collapsed_triangle_rule(n):
    """Barycentric points and area-fraction weights of the n x n collapsed Gauss rule.

    Map (u, s) in [0,1]^2 to l2 = u, l3 = s (1 - u), l1 = 1 - l2 - l3 with Jacobian (1 - u); exact
    for total degree <= 2n - 2. Weights sum to 1 (fractions of the area).
    """
    x, w = gauss01(n)
    u, s = np.meshgrid(x, x, indexing="ij")
    wu, ws = np.meshgrid(w, w, indexing="ij")
    l2 = u.ravel()
    l3 = (s * (1.0 - u)).ravel()
    l1 = 1.0 - l2 - l3
    wt = (wu * ws * (1.0 - u)).ravel() * 2.0
    return np.stack([l1, l2, l3], axis=1), wt


def voxel_gauss2():
    """Offsets (in units of h, from the voxel centre) and weights (fractions of h^3) of the
    2x2x2 Gauss-Legendre rule."""
    a = 0.5 / np.sqrt(3.0)
    o = np.array([[sx, sy, sz] for sz in (-a, a) for sy in (-a, a) for sx in (-a, a)])
    return o, np.full(8, 1.0 / 8.0)
