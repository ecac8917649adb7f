"""Mie series for a homogeneous dielectric sphere under a plane wave (textbook closed form).

Used as a physics pin of the volume operator: the discretised current-based VIE (eq. (4)) with a
plane-wave right-hand side must approach the exact interior field as the grid is refined.

The series is written for the exp(-i w t) convention, E_inc = x e^{i k z}, internal field
    E_1 = sum_n E_n (c_n M_o1n^(1) - i d_n N_e1n^(1)),   E_n = i^n (2n+1)/(n(n+1)),
scattered field
    E_s = sum_n E_n (i a_n N_e1n^(3) - b_n M_o1n^(3)),
and returned for exp(+i w t) by conjugation: the caller's incident field is x e^{-i k z} and the
relative index uses eps_r - i sigma/(w eps0); under conjugation that becomes eps_r + i sigma/(w eps0).

Parity pins (tests): Rayleigh limit E_1 -> 3/(eps + 2) for k a -> 0, continuity of the
tangential field at r = a (internal vs incident + scattered), convergence in n_max.
"""
import numpy as np
from scipy.special import spherical_jn, spherical_yn


def _pi_tau(nmax, mu):
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros_like(pi)
    pi[1] = 1.0
    for n in range(2, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
    for n in range(1, nmax + 1):
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi, tau


def _coeffs(x, m, nmax):
    n = np.arange(1, nmax + 1)
    jx = spherical_jn(n, x)
    djx = spherical_jn(n, x, derivative=True)
    yx = spherical_yn(n, x)
    dyx = spherical_yn(n, x, derivative=True)
    hx = jx + 1j * yx
    dhx = djx + 1j * dyx
    mx = m * x
    jm = spherical_jn(n, mx)
    djm = spherical_jn(n, mx, derivative=True)
    psi_x, dpsi_x = x * jx, jx + x * djx
    xi_x, dxi_x = x * hx, hx + x * dhx
    psi_m, dpsi_m = mx * jm, jm + mx * djm
    a = (m * psi_m * dpsi_x - psi_x * dpsi_m) / (m * psi_m * dxi_x - xi_x * dpsi_m)
    b = (psi_m * dpsi_x - m * psi_x * dpsi_m) / (psi_m * dxi_x - m * xi_x * dpsi_m)
    c = (jx * dxi_x - hx * dpsi_x) / (jm * dxi_x - hx * dpsi_m)
    d = m * (jx * dxi_x - hx * dpsi_x) / (m * m * jm * dxi_x - hx * dpsi_m)
    return n, a, b, c, d


def _field(points, k, m_rel, nmax, kind, a_rad):
    """Field (exp(-i w t) convention) of the internal/incident/scattered series at points."""
    p = np.asarray(points, np.float64)
    r = np.linalg.norm(p, axis=1)
    th = np.arccos(np.clip(p[:, 2] / np.where(r > 0, r, 1.0), -1.0, 1.0))
    ph = np.arctan2(p[:, 1], p[:, 0])
    mu = np.cos(th)
    pi, tau = _pi_tau(nmax, mu)
    n, a, b, c, d = _coeffs(k * a_rad, m_rel, nmax)
    En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
    if kind == "int":
        rho = m_rel * k * r
    else:
        rho = k * r
    Er = np.zeros(len(p), complex)
    Et = np.zeros(len(p), complex)
    Ep = np.zeros(len(p), complex)
    for idx, nn in enumerate(n):
        if kind == "sca":
            z = spherical_jn(nn, rho) + 1j * spherical_yn(nn, rho)
            dz = spherical_jn(nn, rho, derivative=True) + 1j * spherical_yn(nn, rho, derivative=True)
            cM, cN = -b[idx], 1j * a[idx]
        else:
            z = spherical_jn(nn, rho)
            dz = spherical_jn(nn, rho, derivative=True)
            if kind == "int":
                cM, cN = c[idx], -1j * d[idx]
            else:
                cM, cN = 1.0, -1j
        dd = z + rho * dz                      # [rho z]'
        # M_o1n and N_e1n (exp(-iwt) textbook form)
        Mt = np.cos(ph) * pi[nn] * z
        Mp = -np.sin(ph) * tau[nn] * z
        with np.errstate(divide="ignore", invalid="ignore"):
            Nr = np.cos(ph) * nn * (nn + 1) * np.sin(th) * pi[nn] * np.where(rho != 0, z / rho, 0.0)
            Nt = np.cos(ph) * tau[nn] * np.where(rho != 0, dd / rho, 0.0)
            Np = -np.sin(ph) * pi[nn] * np.where(rho != 0, dd / rho, 0.0)
        Er += En[idx] * cN * Nr
        Et += En[idx] * (cM * Mt + cN * Nt)
        Ep += En[idx] * (cM * Mp + cN * Np)
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    ex = Er * st * cp + Et * ct * cp - Ep * sp
    ey = Er * st * sp + Et * ct * sp + Ep * cp
    ez = Er * ct - Et * st
    return np.stack([ex, ey, ez], axis=1), (Er, Et, Ep)


def sphere_internal_field(points, freq_hz, radius, eps_r, sigma, nmax=None):
    """Total internal E (exp(+i w t)) for incident x e^{-i k0 z}, unit amplitude; points (P,3)
    relative to the sphere centre, all inside the sphere."""
    from .constants import EPS0, k0, omega
    k = k0(freq_hz)
    eps_c = eps_r + 1j * sigma / (omega(freq_hz) * EPS0)   # exp(-iwt) form
    m_rel = np.sqrt(eps_c)
    if nmax is None:
        x = k * radius
        nmax = int(np.ceil(x + 4.05 * x ** (1.0 / 3.0) + 2)) + 10
    E, _ = _field(points, k, m_rel, nmax, "int", radius)
    return np.conj(E)


def sphere_fields_spherical(points, freq_hz, radius, eps_r, sigma, nmax, kind):
    """(E_r, E_theta, E_phi) in the exp(-i w t) convention, for boundary-condition tests."""
    from .constants import EPS0, k0, omega
    k = k0(freq_hz)
    m_rel = np.sqrt(eps_r + 1j * sigma / (omega(freq_hz) * EPS0))
    _, sph = _field(points, k, m_rel, nmax, kind, radius)
    return sph
