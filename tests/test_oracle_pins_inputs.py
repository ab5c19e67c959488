"""Pins of the oracle's synthetic ionic terms and position operator against
closed forms and exact symmetries that do not reuse the oracle's grid code:

  * the Gaussian wells integrate to -D (2 pi w^2)^(3/2) per atom (the grid sum of
    a well-resolved periodic Gaussian equals its integral to exponential accuracy);
  * moving every atom by one grid step moves the potential by one grid step
    (a circular roll: pins the image sum and the axis mapping);
  * the projectors' unnormalised profile, summed over a fine 3-D grid, equals a
    1-D radial quadrature of the stated profile (s and p channels);
  * moving the electrons by one grid step along x raises Tr(P M_x) by N_e h,
    less the cell length times the charge that crosses the sawtooth jump, and
    leaves Tr(P M_y), Tr(P M_z) unchanged (pins axis, sign and jump location).

Each pin is also run against a planted mistake in the oracle (on the CPU) and
must reject it.  Sec. Overview of RMG (potential terms, nonlocal
pseudopotentials, grid quadrature); Sec. Algorithm (position operator of the
field, sawtooth on the periodic cell)."""

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import grid, hamiltonian, system

from conftest import c1_ground_state, c1_system


# ---------------------------------------------------------------------------
# Local wells
# ---------------------------------------------------------------------------
def _wells(n=32, h=0.35, seed=11):
    # several atoms, one of them close to a cell face so the image sum matters
    s = synth.make_system(n, h, 5, 1, 1, seed=seed, region=(0.25, 0.75))
    s.pos[0] = np.array([0.4, 0.5 * n * h, 0.3 * n * h])
    return s


def _integral_error(s, v):
    exact = -np.sum(s.depth * (2.0 * np.pi * s.width ** 2) ** 1.5)
    return abs(s.h ** 3 * np.sum(v) - exact) / abs(exact)


def test_local_wells_integrate_to_closed_form():
    s = _wells()
    assert _integral_error(s, system.v_ion(s)) < 1e-12


def test_local_wells_integral_rejects_planted_width_convention():
    # exp(-d^2 / w^2) instead of exp(-d^2 / (2 w^2)) is the same as w -> w / sqrt(2)
    s = _wells()
    s.width = s.width / np.sqrt(2.0)
    assert _integral_error(_wells(), system.v_ion(s)) > 0.5


def _shifted(s, dx):
    t = synth.make_system(s.n, s.h, s.n_atoms, s.n_occ, s.n_virt, seed=s.seed)
    t.pos, t.depth, t.width, t.nl_D, t.nl_rank, t.n_images = s.pos.copy(), s.depth, s.width, s.nl_D, s.nl_rank, s.n_images
    t.pos[:, 0] += dx
    return t


def _roll_error(s, vfun):
    v0 = vfun(s)
    v1 = vfun(_shifted(s, s.h))
    return np.max(np.abs(v1 - np.roll(v0, 1, axis=2))) / np.max(np.abs(v0))


def test_local_wells_translate_as_a_grid_roll():
    s = _wells()
    assert _roll_error(s, system.v_ion) < 1e-13
    # the face atom really does wrap: without images the roll would not hold
    t = _wells()
    t.n_images = 0
    assert _roll_error(t, system.v_ion) > 1e-3


def test_local_wells_roll_rejects_planted_axis_swap(monkeypatch):
    s = _wells()
    orig = system.grid_xyz

    def swapped(sys):
        x, y, z = orig(sys)
        return z, y, x

    monkeypatch.setattr(system, "grid_xyz", swapped)
    assert _roll_error(s, system.v_ion) > 1e-2


# ---------------------------------------------------------------------------
# Projector radial profile
# ---------------------------------------------------------------------------
def _stated_profile(s, sigma=0.6, rc=2.0):
    """The profile as specified: exp(-s^2 / (2 sigma^2)) (1 - s^2 / r_c^2)^2 on s < r_c."""
    return np.exp(-s * s / (2 * sigma ** 2)) * (1.0 - (s / rc) ** 2) ** 2


def _radial_moments(rc=2.0):
    """1-D quadratures of the stated profile: int 4 pi s^2 g, int 4 pi s^2 g^2,
    int 4 pi s^4 g / 3, int 4 pi s^4 g^2 / 3 (x^2 averages to s^2/3 on a sphere)."""
    q = lambda f: quad(f, 0.0, rc, epsabs=0, epsrel=1e-13, limit=200)[0]
    g = _stated_profile
    return (q(lambda r: 4 * np.pi * r * r * g(r)),
            q(lambda r: 4 * np.pi * r * r * g(r) ** 2),
            q(lambda r: 4 * np.pi * r ** 4 * g(r) / 3),
            q(lambda r: 4 * np.pi * r ** 4 * g(r) ** 2 / 3))


def _projector_moment_errors():
    """Errors of the grid moments of the normalised projectors against the
    radial quadratures, on a fine grid (h = 0.08) with the atom on a point.
    Point coordinates are built here, not taken from the oracle."""
    n, h = 56, 0.08
    s = synth.make_system(n, h, 1, 1, 1, seed=0, nl_rank=4)
    c = np.array([28, 27, 29])
    s.pos = (c * h)[None, :].astype(float)
    s.nl_D = np.array([[1.0, 1.0, 1.0, 1.0]])
    idx, beta, _ = system.projectors(s)[0]
    # flat index = (k n + j) n + i for point (i, j, k) = (x, y, z)
    i, j, k = idx % n, (idx // n) % n, idx // (n * n)
    x, y, z = (i - c[0]) * h, (j - c[1]) * h, (k - c[2]) * h
    m0, m0sq, m2, m2sq = _radial_moments()
    dv = h ** 3
    err = []
    # s channel: h^3 sum beta_1 = int g / sqrt(int g^2)
    err.append(abs(dv * np.sum(beta[:, 0]) - m0 / np.sqrt(m0sq)) / (m0 / np.sqrt(m0sq)))
    # p channels: h^3 sum beta_(1+q) r_q = int r_q^2 g / sqrt(int r_q^2 g^2); other directions vanish
    ref = m2 / np.sqrt(m2sq)
    for q, cq in enumerate((x, y, z)):
        err.append(abs(dv * np.sum(beta[:, 1 + q] * cq) - ref) / ref)
        for r, d in enumerate((x, y, z)):
            if r != q:
                err.append(abs(dv * np.sum(beta[:, 1 + q] * d)) / ref)
    return max(err)


def test_projector_profile_matches_radial_quadrature():
    assert _projector_moment_errors() < 1e-6


@pytest.mark.parametrize("planted", ["linear_cutoff", "sigma_convention"])
def test_projector_profile_pin_rejects_planted_profiles(monkeypatch, planted):
    if planted == "linear_cutoff":
        bad = lambda s2, sigma, rc: np.exp(-s2 / (2 * sigma ** 2)) * (1.0 - np.sqrt(s2) / rc) ** 2
    else:
        bad = lambda s2, sigma, rc: np.exp(-s2 / sigma ** 2) * (1.0 - s2 / rc ** 2) ** 2
    monkeypatch.setattr(system, "radial_profile", bad)
    assert _projector_moment_errors() > 1e-2


def test_projector_moment_pin_rejects_planted_axis_swap(monkeypatch):
    orig = system.grid_xyz

    def swapped(sys):
        x, y, z = orig(sys)
        return z, y, x

    monkeypatch.setattr(system, "grid_xyz", swapped)
    assert _projector_moment_errors() > 1e-2


# ---------------------------------------------------------------------------
# Position operator (sawtooth) and dipole
# ---------------------------------------------------------------------------
def _dipole_shift_errors():
    """Move every ground-state orbital of the 32^3 parity molecule by one grid
    step along +x and take mu = Tr(P_0 M_q) from the oracle's model before and
    after.  Returns (error of the x shift against N_e h - L Q_jump, largest
    change of mu_y, mu_z)."""
    s = c1_system()
    psi, _ = c1_ground_state()
    nx, ny, nz = s.n
    f = s.occupations()
    P = np.diag(f)
    orb = psi.reshape(s.n_orb, nz, ny, nx)
    mu0 = hamiltonian.Model(s, psi).dipole(P)
    mu1 = hamiltonian.Model(s, np.roll(orb, 1, axis=3).reshape(s.n_orb, -1)).dipole(P)
    n_e = np.sum(f)
    # electrons on the last x-plane wrap to the first and their coordinate drops by L - h
    rho0 = np.sum(f[:, None] * psi.reshape(s.n_orb, -1) ** 2, axis=0).reshape(nz, ny, nx)
    q_jump = s.h ** 3 * np.sum(rho0[:, :, nx - 1])
    expect = n_e * s.h - nx * s.h * q_jump
    return abs(mu1[0] - mu0[0] - expect), max(abs(mu1[1] - mu0[1]), abs(mu1[2] - mu0[2]))


def test_dipole_shift_pins_axis_sign_and_jump():
    ex, eyz = _dipole_shift_errors()
    assert ex < 1e-11 and eyz < 1e-11


def test_dipole_centred_sawtooth_averages_to_zero():
    s = c1_system()
    for q in range(3):
        assert abs(np.sum(grid.dipole_coordinate(s, q))) < 1e-9


@pytest.mark.parametrize("planted", ["axis_swap", "sign", "jump_inside"])
def test_dipole_shift_pin_rejects_planted_mistakes(monkeypatch, planted):
    orig = grid.dipole_coordinate

    def bad(sys, axis):
        if planted == "axis_swap":
            return orig(sys, 2 - axis)
        if planted == "sign":
            return -orig(sys, axis)
        # sawtooth jump moved into the cell (coordinate wrapped at the centre)
        q = orig(sys, axis)
        L = sys.n[axis] * sys.h
        return np.where(q > 0, q - L, q)

    monkeypatch.setattr(hamiltonian, "dipole_coordinate", bad)
    ex, eyz = _dipole_shift_errors()
    assert ex > 1e-4 or eyz > 1e-4
