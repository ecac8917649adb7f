"""Conductor-to-body coupling matrix (paper Sec. II-B after eq. (8); quadrature Sec. IV-C).

Petrov-Galerkin: RWG source functions, voxel-PWC testing. With rows multiplied by i w eps0 and
the body equation tested with the field, the entry for voxel p, component a, against RWG n is

    Z_bc[p a, n] = - int_{V_p} [ (k0^2 I + grad grad) int_{T_n} g(r - r') f_n(r') dS' ]_a dV

    (k0^2 I + grad grad) g(R) = g(R) [ (k0^2 - i k0/R - 1/R^2) I + (3/R^2 + 3 i k0/R - k0^2) R^R^ ].

The integrals are point rules, as the paper states: 8 volume points (2x2x2 Gauss-Legendre) and
5 surface points (rule R5) for the near conductors; 1 volume point (voxel centre) and 1 surface
point (triangle centroid) for the far conductors. The coil rows of eq. (8) are the transpose.

Parity pins (tests): the dyad against finite differences of g; both point rules against the
converged mixed-potential form of the same entry (k0^2 times the vector potential integrated over
the voxel plus the scalar potential of div f integrated over its faces, high-order rules; no dyad
involved) at 3, 6 and 12 voxels from the RWG, where the near rule's error falls from 2e-3 to 3e-6
and stays below a fifth of the far rule's; reciprocity of the assembled system.
"""
import numpy as np

from .quadrature import R5_BARY, R5_W, voxel_gauss2


def dyad_apply(R, v, k):
    """[(k^2 I + grad grad) g](R) v for R (..., 3), v (..., 3)."""
    r = np.linalg.norm(R, axis=-1)
    g = np.exp(-1j * k * r) / (4.0 * np.pi * r)
    a = k * k - 1j * k / r - 1.0 / (r * r)
    b = 3.0 / (r * r) + 3j * k / r - k * k
    rv = np.einsum("...c,...c->...", R, v) / (r * r)
    return g[..., None] * (a[..., None] * v + (b * rv)[..., None] * R)


def zbc_block(centres, h, rwg, k, rule, chunk=1 << 21):
    """Coupling block for voxel centres (P, 3) against all RWGs of `rwg`: returns (3, P, m).

    rule = "near" (8 x 5 points) or "far" (1 x 1 point).
    """
    centres = np.asarray(centres, np.float64)
    if rule == "near":
        vo, vw = voxel_gauss2()
        sb, sw = R5_BARY, R5_W
    elif rule == "far":
        vo, vw = np.zeros((1, 3)), np.ones(1)
        sb, sw = np.full((1, 3), 1.0 / 3.0), np.ones(1)
    else:
        raise ValueError(rule)
    P, m = len(centres), rwg.m
    out = np.zeros((3, P, m), np.complex128)
    vpts = centres[:, None, :] + h * vo[None, :, :]                 # (P, nv, 3)
    for side, s in ((0, 1.0), (1, -1.0)):
        tri = rwg.tri[:, side]
        tv = rwg.verts[rwg.tris[tri]]                              # (m, 3, 3)
        spts = np.einsum("qk,mkc->mqc", sb, tv)                     # (m, ns, 3)
        free = rwg.verts[rwg.free[:, side]]                         # (m, 3)
        # f = s * l/(2A) (r - p); the surface weight carries A, so the product is s*l/2
        fv = (spts - free[:, None, :]) * (s * 0.5 * rwg.length)[:, None, None]
        per = max(1, chunk // (m * len(vo) * len(sb)))
        for p0 in range(0, P, per):
            vp = vpts[p0:p0 + per]
            R = vp[:, None, :, None, :] - spts[None, :, None, :, :]   # (p, m, nv, ns, 3)
            F = np.broadcast_to(fv[None, :, None, :, :], R.shape)
            D = dyad_apply(R, F, k)
            wts = (vw[:, None] * sw[None, :]) * h ** 3
            acc = np.einsum("pmvsc,vs->cpm", D, wts)
            out[:, p0:p0 + per, :] -= acc
    return out
