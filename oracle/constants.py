"""Physical constants and material conversion (paper Sec. II-A, eq. (1)).

Parity: pinned by the Mie-series tests (a wrong sign or factor in chi moves the interior field).
"""
import numpy as np

EPS0 = 8.8541878128e-12      # F/m
MU0 = 1.25663706212e-6       # H/m
C0 = 1.0 / np.sqrt(EPS0 * MU0)


def omega(freq_hz):
    return 2.0 * np.pi * freq_hz


def k0(freq_hz):
    """Free-space wavenumber."""
    return omega(freq_hz) / C0


def chi(eps_r, sigma, freq_hz):
    """Complex electric susceptibility for exp(+i w t): eps_r - 1 - i sigma / (w eps0).

    eq. (1) defines chi_e = eps_r - 1 for lossless media; conductivity enters as the imaginary
    part of the complex permittivity.
    """
    return (np.asarray(eps_r) - 1.0) - 1j * np.asarray(sigma) / (omega(freq_hz) * EPS0)


def row_scale(freq_hz):
    """The factor i w eps0 applied to every row of the coupled system."""
    return 1j * omega(freq_hz) * EPS0
