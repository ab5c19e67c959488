"""Pins of the oracle's sawtooth coordinate with a movable jump and of the
vacuum dipole correction (Sec. Algorithm, time-dependent field: a sawtooth
potential with a dipole correction in the vacuum, after Bengtsson, Phys. Rev. B
59, 12301 (1999)).  Closed forms of one-dimensional electrostatics, the
variational identity dE/dP = H, and planted mistakes.  No GPU."""

import dataclasses

import numpy as np
import pytest

import oracle
import synth
from oracle import grid, hamiltonian


def _slab_cell(axis, mask, jump):
    """A thin periodic cell, long along `axis` (96 points of 0.25 bohr)."""
    n = [4, 4, 4]
    n[axis] = 96
    s = synth.make_system(tuple(n), 0.25, 1, 1, 1, seed=0)
    j = [0, 0, 0]
    j[axis] = jump
    # electrons only: the one synthetic atom carries no point charge here
    return dataclasses.replace(s, saw_jump=tuple(j), dipole_correction=mask, ion_charge=np.zeros(1))


def _sheets(s, axis, a, b, amp, w):
    """Neutral pair of Gaussian sheets normal to `axis`: amp (g(z - a) - g(z - b)),
    g of unit integral and width w; the per-area dipole is amp (a - b)."""
    z = np.arange(s.n[axis]) * s.h
    g = lambda c: np.exp(-((z - c) ** 2) / (2 * w * w)) / np.sqrt(2 * np.pi * w * w)
    prof = amp * (g(a) - g(b))
    shape = [1, 1, 1]
    shape[2 - axis] = s.n[axis]
    nx, ny, nz = s.n
    return np.broadcast_to(prof.reshape(shape), (nz, ny, nx)).ravel().copy()


def _profile(v, s, axis):
    nx, ny, nz = s.n
    return v.reshape(nz, ny, nx).mean(axis=tuple(k for k in range(3) if k != 2 - axis))


# sheets at 8 and 11 bohr (width 0.75), jump plane at 19 bohr (index 76) of a 24 bohr cell
A_POS, B_POS, AMP, WID, JUMP = 8.0, 11.0, 0.7, 0.75, 76


def _slab_errors(axis, mask=None):
    """(slope error of the corrected vacuum field, step error, periodic slope error)."""
    mask = (1 << axis) if mask is None else mask
    s = _slab_cell(axis, mask, JUMP)
    rho = _sheets(s, axis, A_POS, B_POS, AMP, WID)
    d_area = AMP * (A_POS - B_POS)  # closed form of the per-area dipole
    L = s.n[axis] * s.h
    h = s.h
    z = np.arange(s.n[axis]) * h
    v, _ = hamiltonian.electrostatic(rho, s)
    prof = _profile(v, s, axis)
    right = (z > B_POS + 5.5) & (z < JUMP * h - 0.01)       # vacuum between the pair and the jump
    left = (z >= JUMP * h) | (z < A_POS - 5.5)               # vacuum past the jump (wraps round)
    slope_err = max(np.ptp(prof[right]), np.ptp(prof[left]))
    step_err = abs((prof[right].mean() - prof[left].mean()) - 4 * np.pi * d_area)
    # periodic Hartree alone: uniform vacuum field -4 pi d / L
    s0 = dataclasses.replace(s, dipole_correction=0)
    v0 = _profile(hamiltonian.electrostatic(rho, s0)[0], s0, axis)
    zr = z[right]
    slope = np.polyfit(zr, v0[right], 1)[0]
    per_err = abs(slope + 4 * np.pi * d_area / L)
    return slope_err, step_err, per_err


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_slab_dipole_correction_flattens_vacuum_and_steps_by_4pi_d(axis):
    slope_err, step_err, per_err = _slab_errors(axis)
    assert slope_err < 1e-9
    assert step_err < 1e-9
    assert per_err < 1e-9


def test_correction_along_an_axis_without_dipole_changes_nothing():
    s = _slab_cell(2, 1 | 2, JUMP)  # correction along x and y; the density varies along z only
    rho = _sheets(s, 2, A_POS, B_POS, AMP, WID)
    vdc, edc = hamiltonian.dipole_correction(rho, s)
    assert np.max(np.abs(vdc)) < 1e-14 and abs(edc) < 1e-28


def test_correction_energy_is_half_the_density_weighted_potential():
    s = _slab_cell(2, 4, JUMP)
    rho = _sheets(s, 2, A_POS, B_POS, AMP, WID) + 0.01
    vdc, edc = hamiltonian.dipole_correction(rho, s)
    d_area = AMP * (A_POS - B_POS)
    area = s.n[0] * s.n[1] * s.h ** 2
    # the uniform part carries no dipole about the centred sawtooth; E = (2 pi / Omega) d^2
    omega = area * s.n[2] * s.h
    assert abs(edc - 2 * np.pi * (area * d_area) ** 2 / omega) < 1e-10 * edc
    assert abs(edc - 0.5 * s.h ** 3 * np.sum(rho * vdc)) < 1e-12 * edc


@pytest.mark.parametrize("n,j0", [(7, 0), (7, 3), (8, 5), (12, 11)])
def test_sawtooth_with_jump_plane(n, j0):
    s = synth.make_system((n, 5, 6), 0.3, 1, 1, 1, seed=0)
    s = dataclasses.replace(s, saw_jump=(j0, 0, 0))
    q = grid.dipole_coordinate(s, 0)[0, 0, :]
    steps = np.diff(np.concatenate([q, q[:1]]))  # periodic successive differences
    # rises by h everywhere except one drop of (n - 1) h, from plane j0 - 1 to j0
    drop = (j0 - 1) % n
    for i in range(n):
        want = -(n - 1) * s.h if i == drop else s.h
        assert abs(steps[i] - want) < 1e-12
    assert abs(np.sum(q)) < 1e-12
    assert abs(q[j0] + 0.5 * (n - 1) * s.h) < 1e-12


def _small_model_dc(mask, jump, seed=11, n_orb=6):
    s = synth.make_system(16, 0.4, 2, n_orb // 2, n_orb - n_orb // 2, seed=seed, nl_rank=4,
                          region=(0.3, 0.7))
    s = dataclasses.replace(s, saw_jump=jump, dipole_correction=mask)
    psi = synth.lowpass_orbitals(16, 0.4, n_orb, seed)
    q, _ = np.linalg.qr(psi.reshape(n_orb, -1).T)
    psi = q.T / np.sqrt(s.h ** 3)
    return s, oracle.Model(s, psi)


def _energy_derivative_error(mask=7, jump=(2, 14, 5)):
    s, m = _small_model_dc(mask, jump)
    rng = np.random.default_rng(5)
    N = m.N
    A = rng.standard_normal((N, N))
    S = np.diag(s.occupations()) + 0.05 * (A + A.T)
    B = rng.standard_normal((N, N))
    P = S + 1j * 0.05 * (B - B.T)
    H, _ = m.h_of_p(P)
    X = rng.standard_normal((N, N))
    X = X + X.T
    eps = 1e-5

    def E(Pm):
        return m.energy(Pm, m.h_of_p(Pm)[1])

    dE = (E(P + eps * X) - E(P - eps * X)) / (2 * eps)
    return abs(dE - np.sum(X * H)) / max(1.0, abs(dE)), m, P


def test_energy_derivative_is_the_hamiltonian_with_dipole_correction():
    err, m, P = _energy_derivative_error()
    assert err < 1e-8
    # and the correction is not negligible here: it moves H by more than the test resolves
    s0 = dataclasses.replace(m.sys, dipole_correction=0)
    m0 = oracle.Model(s0, m.psi)
    assert np.max(np.abs(m.h_of_p(P)[0] - m0.h_of_p(P)[0])) > 1e-4


def _symmetric_blob_field():
    """Largest |v_dc| for a charged blob centred opposite the jump plane
    (mirror-symmetric about the sawtooth's zero): it has no dipole."""
    s = _slab_cell(2, 4, JUMP)
    z0 = ((JUMP + 0.5 * (s.n[2] - 1)) % s.n[2]) * s.h
    z = np.arange(s.n[2]) * s.h
    prof = np.exp(-((z - z0) ** 2) / (2 * 0.7 ** 2))
    nx, ny, nz = s.n
    rho = np.broadcast_to(prof.reshape(nz, 1, 1), (nz, ny, nx)).ravel().copy()
    vdc, _ = hamiltonian.dipole_correction(rho, s)
    return float(np.max(np.abs(vdc)))


def test_blob_without_dipole_gets_no_correction():
    assert _symmetric_blob_field() < 1e-12


def _blob_cell(jump_x, shift, charge=None):
    """A 48 x 8 x 8 cell (h = 0.25) with one ion at x = 5 bohr of charge 2 and a
    Gaussian electron blob of 2 electrons centred at 5 + shift."""
    s = synth.make_system((48, 8, 8), 0.25, 1, 1, 1, seed=0)
    pos = np.array([[5.0, 1.0, 1.0]])
    s = dataclasses.replace(s, pos=pos, saw_jump=(jump_x, 0, 0), dipole_correction=1,
                            ion_charge=charge)
    x = np.arange(48) * s.h
    prof = np.exp(-((x - 5.0 - shift) ** 2) / (2 * 0.5 ** 2))
    prof *= 2.0 / (np.sum(prof) * s.h * (8 * s.h) ** 2)
    rho = np.broadcast_to(prof.reshape(1, 1, 48), (8, 8, 48)).ravel().copy()
    return s, rho


def _ion_errors():
    """(closed-form energy error of a displaced blob, jump dependence of a neutral cell's energy)."""
    shift = 0.4
    s, rho = _blob_cell(40, shift)  # default charge: 2 electrons on the one atom
    _, e = hamiltonian.dipole_correction(rho, s)
    omega = float(np.prod(s.cell))
    closed = 2 * np.pi * (2.0 * shift) ** 2 / omega  # d = N_e * shift
    err_closed = abs(e - closed) / closed
    s2, rho2 = _blob_cell(38, shift)
    _, e2 = hamiltonian.dipole_correction(rho2, s2)
    return err_closed, abs(e2 - e) / closed


def test_displaced_electrons_against_point_ions_closed_form_and_jump_invariance():
    err_closed, err_jump = _ion_errors()
    assert err_closed < 1e-9
    assert err_jump < 1e-12


def test_explicit_ion_charges_equal_the_default_share():
    s, rho = _blob_cell(40, 0.3)
    s2, _ = _blob_cell(40, 0.3, charge=np.array([2.0]))
    a = hamiltonian.dipole_correction(rho, s)
    b = hamiltonian.dipole_correction(rho, s2)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


@pytest.mark.parametrize("planted", ["sign", "factor_2pi", "energy_4pi", "uncentred", "ions_dropped", "ion_sign"])
def test_dipole_pins_reject_planted_mistakes(monkeypatch, planted):
    orig_coord = grid.dipole_coordinate

    def bad(rho, sys):
        mask = int(sys.dipole_correction)
        if not mask:
            return 0.0, 0.0
        omega = float(np.prod(sys.cell))
        v = np.zeros(sys.ng)
        e = 0.0
        for q in range(3):
            if (mask >> q) & 1:
                c = orig_coord(sys, q).ravel()
                if planted == "uncentred":  # measured from the jump plane, not the centre
                    c = c + 0.5 * (sys.n[q] - 1) * sys.h
                d = sys.h ** 3 * float(np.sum(rho * c))
                if planted != "ions_dropped" and sys.n_atoms:
                    zi = hamiltonian.ion_charges(sys) * hamiltonian.sawtooth_at(sys.pos[:, q], sys, q)
                    d += (1.0 if planted == "ion_sign" else -1.0) * float(np.sum(zi))
                k = {"sign": -4.0, "factor_2pi": 2.0}.get(planted, 4.0)
                v += (k * np.pi / omega) * d * c
                e += ((4.0 if planted == "energy_4pi" else 2.0) * np.pi / omega) * d * d
        return v, e

    monkeypatch.setattr(hamiltonian, "dipole_correction", bad)
    slope_err, step_err, _ = _slab_errors(2)
    d_err, _, _ = _energy_derivative_error()
    blob = _symmetric_blob_field()
    ion_closed, ion_jump = _ion_errors()
    assert (slope_err > 1e-4 or step_err > 1e-4 or d_err > 1e-6 or blob > 1e-4 or ion_closed > 1e-4
            or ion_jump > 1e-4)
