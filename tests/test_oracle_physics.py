"""Physics pins of the assembled oracle system: the Mie series (volume operator, constants and
signs), reciprocity (eq. (8) symmetric), energy balance of a port-driven closed cavity, the
hybrid operator of eq. (15) against the fully assembled eq. (11), and GMRES against LU."""
import numpy as np
import pytest

import vsie_synth as synth
from oracle import gmres, mie, system, tt
from oracle.constants import EPS0, omega

F = 297.2e6


def test_mie_rayleigh_limit_and_continuity():
    a = 1e-4
    E = mie.sphere_internal_field(np.array([[1e-5, 2e-5, -1e-5]]), F, a, 52.0, 0.55)
    epsc = 52.0 - 1j * 0.55 / (omega(F) * EPS0)
    assert abs(E[0, 0] - 3 / (epsc + 2)) < 1e-3 * abs(3 / (epsc + 2))
    a = 35e-3
    th = np.linspace(0.2, 2.9, 9)
    ph = np.linspace(0.1, 5, 9)
    pts = a * np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    Ei = mie.sphere_fields_spherical(pts, F, a, 52.0, 0.55, 30, "int")
    Eo = mie.sphere_fields_spherical(pts, F, a, 52.0, 0.55, 30, "inc")
    Es = mie.sphere_fields_spherical(pts, F, a, 52.0, 0.55, 30, "sca")
    for c in (1, 2):
        assert np.abs(Ei[c] - Eo[c] - Es[c]).max() < 1e-12
    epsbh = 52.0 + 1j * 0.55 / (omega(F) * EPS0)
    assert np.abs(epsbh * Ei[0] - Eo[0] - Es[0]).max() < 1e-12


def _vie_mie_error(n, h, radius, eps=52.0, sig=0.55):
    p = synth.Problem(synth.sphere_phantom((n, n, n), h, radius, eps, sig), [], F, "mie")
    d = system.discretize(p)
    S, _ = system.assemble_direct(d)
    x = S.solve(system.plane_wave_rhs(d))
    c, idx = d.centres(d.tissue)
    J = x[d.m_f + d.m_n:].reshape(3, -1)[:, d.tissue].T
    E = J / (1j * omega(F) * EPS0 * d.chi[d.tissue][:, None])
    # equal-volume sphere radius of the staircase, interior voxels only (surface layer excluded)
    r_eq = (len(d.tissue) * h ** 3 * 3 / (4 * np.pi)) ** (1 / 3)
    inner = np.linalg.norm(c, axis=1) < radius - 1.5 * h
    Em = mie.sphere_internal_field(c[inner], F, r_eq, eps, sig)
    return np.linalg.norm(E[inner] - Em) / np.linalg.norm(Em)


def test_vie_matches_mie_low_contrast():
    """eps_r = 2: the PWC current-based VIE reproduces the Mie interior field to ~1% and the
    error falls under refinement."""
    e_coarse = _vie_mie_error(10, 5e-3, 20e-3, 2.0, 0.0)
    e_fine = _vie_mie_error(18, 2.5e-3, 20e-3, 2.0, 0.0)
    assert e_coarse < 0.02
    assert e_fine < 0.7 * e_coarse


def test_vie_mie_high_contrast_converges_first_order():
    """eps_r = 52, sigma = 0.55 (the tissue of the tiny case): the staircased sphere converges
    at first order (error roughly halves when h halves)."""
    e_coarse = _vie_mie_error(10, 5e-3, 20e-3)
    e_fine = _vie_mie_error(18, 2.5e-3, 20e-3)
    # measured 47 % and 24 %: PWC currents on a staircased sphere of contrast 52 converge at first
    # order from a large error, so the pin is the rate together with both levels
    assert e_coarse < 0.5 and e_fine < 0.27
    assert e_fine < 0.56 * e_coarse


@pytest.fixture(scope="module")
def small():
    p = synth.small_case()
    d = system.discretize(p)
    S, blocks = system.assemble_direct(d)
    return p, d, S, blocks


def test_reciprocity_and_energy_balance(small):
    p, d, S, _ = small
    assert np.abs(S.Z - S.Z.T).max() < 1e-13 * np.abs(S.Z).max()
    x = S.solve(system.port_rhs(d, 0))
    I = system.port_current(d, 0, x)
    jb = x[d.m_f + d.m_n:].reshape(3, -1)[:, d.tissue]
    E = jb / (1j * omega(F) * EPS0 * d.chi[d.tissue])
    sig = p.grid.sigma.ravel()[d.tissue]
    p_abs = 0.5 * np.sum(sig * np.sum(np.abs(E) ** 2, 0)) * d.h ** 3
    p_in = 0.5 * np.real(1.0 * np.conj(I))
    assert p_in > 0
    assert abs(p_in - p_abs) < 1e-3 * p_in          # closed PEC shield: no radiation


def test_free_space_body_decouples(small):
    """eps_r = 1, sigma = 0 everywhere: no body unknowns, identity rows, zero body current."""
    p = synth.small_case()
    p.grid.eps_r[:] = 1.0
    p.grid.sigma[:] = 0.0
    d = system.discretize(p)
    S, _ = system.assemble_direct(d)
    x = S.solve(system.port_rhs(d, 0))
    assert np.all(x[d.m_f + d.m_n:] == 0)


def test_hybrid_operator_close_to_full_assembly(small):
    """eq. (15) with TT (1e-3) far coupling, low-rank near-far block and pFFT near block solves
    within 1% of the fully assembled system (the paper reports 0.08-0.52% for PWC)."""
    p, d, S, blocks = small
    cores = [tt.tt_svd(system.far_coupling_tensor(d, a), 1e-3) for a in range(3)]
    U, sv, Vh = np.linalg.svd(blocks["nf"], full_matrices=False)
    r = int(np.sum(sv > 1e-4 * sv[0]))
    S2, _, _ = system.assemble_same(d, cores, (U[:, :r] * sv[:r], Vh[:r].conj().T), 2, direct_blocks=blocks)
    assert np.abs(S2.Z - S2.Z.T).max() < 1e-13 * np.abs(S2.Z).max()
    b = system.port_rhs(d, 0)
    x1, x2 = S.solve(b), S2.solve(b)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-2


def test_gmres_matches_direct(small):
    """The coupled system inherits the low-frequency ill-conditioning of the EFIE (condition
    number ~1e7), so a long restart is used here; restart 50 stagnates on this case."""
    _, d, S, _ = small
    b = system.port_rhs(d, 0)
    x, it, hist = gmres.gmres(S.matvec, b, tol=1e-8, restart=1000, max_iter=2000)
    assert np.linalg.norm(S.matvec(x) - b) / np.linalg.norm(b) < 1e-8
    assert np.linalg.norm(x - S.solve(b)) / np.linalg.norm(x) < 1e-4


def test_gmres_restart_equals_dimension_terminates():
    rng = np.random.default_rng(0)
    n = 40
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n) + 0j
    x, it, _ = gmres.gmres(lambda v: A @ v, b, tol=1e-12, restart=n, max_iter=n)
    assert it <= n
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-10
