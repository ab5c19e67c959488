"""Pins of the CPU oracle against what the paper and the mathematics fix
(closed forms, invariants, special cases, brute force), independent of the
oracle's own code paths.  No GPU."""

import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth
from oracle import grid, hamiltonian, propagate, system
from oracle.ground_state import dense_ground_state, ground_state

from conftest import GOLDEN, c1_ground_state, c1_model, c1_oracle_run, c1_system


# ---------------------------------------------------------------------------
# Finite-difference Laplacian (Sec. Overview of RMG, central difference formula)
# ---------------------------------------------------------------------------
def test_fd_coefficients_match_published_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fd8_coefficients.txt")) if l.strip() and l[0] != "#"]
    table = [Fraction(r[1]) for r in rows]
    assert grid.fd_coefficients(4) == table


@pytest.mark.parametrize("n_half", [1, 2, 3, 4])
def test_fd_exact_on_polynomials_up_to_degree_2n(n_half):
    a = grid.fd_coefficients(n_half)
    for deg in range(0, 2 * n_half + 2):
        for x0 in (Fraction(0), Fraction(3, 7), Fraction(-5, 3)):
            approx = a[0] * x0 ** deg + sum(a[k] * ((x0 + k) ** deg + (x0 - k) ** deg) for k in range(1, n_half + 1))
            exact = deg * (deg - 1) * x0 ** (deg - 2) if deg >= 2 else Fraction(0)
            if deg <= 2 * n_half + 1:
                assert approx == exact, (n_half, deg, x0)
    # and not exact one degree higher than the symmetric order allows
    deg = 2 * n_half + 2
    approx = a[0] * 0 + sum(a[k] * 2 * Fraction(k) ** deg for k in range(1, n_half + 1))
    assert approx != 0


def test_fd_moment_identities():
    a = grid.fd_coefficients(4)
    assert a[0] + 2 * sum(a[1:]) == 0
    assert 2 * sum(Fraction(k * k) * a[k] for k in range(1, 5)) == 2


def test_fd_plane_wave_dispersion_closed_form():
    s = synth.make_system((16, 12, 20), 0.35, 1, 1, 1, seed=0)
    nx, ny, nz = s.n
    c = grid.fd_coefficients_float(4)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for m in [(1, 0, 0), (3, 2, 1), (8, 6, 10), (5, 1, 7)]:
        k = [2 * np.pi * m[0] / (nx * s.h), 2 * np.pi * m[1] / (ny * s.h), 2 * np.pi * m[2] / (nz * s.h)]
        f = np.cos(k[0] * x * s.h + k[1] * y * s.h + k[2] * z * s.h + 0.3)
        lap = grid.laplacian(f, s.h, c)
        lam = grid.fd_dispersion(k, s.h, c)
        assert np.max(np.abs(lap - lam * f)) < 1e-11 * max(1.0, abs(lam))
    # long waves approach the continuum -k^2
    k = [2 * np.pi / (nx * s.h), 0, 0]
    assert abs(grid.fd_dispersion(k, s.h, c) + k[0] ** 2) < 1e-6 * k[0] ** 2


def test_fd_mixed_order_blend_still_exact_for_quadratics():
    a = grid.fd_coefficients_float(4, mix_M=0.7)
    f = lambda x: 1.0 + 2.0 * x + 3.0 * x * x  # noqa: E731
    approx = a[0] * f(0.0) + sum(a[k] * (f(k) + f(-k)) for k in range(1, 5))
    assert abs(approx - 6.0) < 1e-12


# ---------------------------------------------------------------------------
# Hartree, exchange, energy
# ---------------------------------------------------------------------------
def test_hartree_matches_direct_fourier_series_of_gaussian_charge():
    s = synth.make_system((20, 24, 16), 0.4, 1, 1, 1, seed=0)
    nx, ny, nz = s.n
    L = s.cell
    R = np.array([3.1, 4.7, 2.9])
    sig, Q = 0.9, 2.5
    X, Y, Z = system.grid_xyz(s)
    rho = np.zeros_like(X)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                d2 = (X - R[0] - i * L[0]) ** 2 + (Y - R[1] - j * L[1]) ** 2 + (Z - R[2] - k * L[2]) ** 2
                rho += Q * np.exp(-d2 / (2 * sig ** 2)) / (2 * np.pi * sig ** 2) ** 1.5
    vh = hamiltonian.hartree(rho.ravel(), s).reshape(nz, ny, nx)
    omega = L.prod()
    gx = 2 * np.pi * np.fft.fftfreq(nx, d=s.h)
    gy = 2 * np.pi * np.fft.fftfreq(ny, d=s.h)
    gz = 2 * np.pi * np.fft.fftfreq(nz, d=s.h)
    G = np.stack(np.meshgrid(gx, gy, gz, indexing="ij"), -1).reshape(-1, 3)
    g2 = np.sum(G * G, axis=1)
    G, g2 = G[g2 > 0], g2[g2 > 0]
    coef = 4 * np.pi * Q * np.exp(-g2 * sig ** 2 / 2) / (g2 * omega)
    for (iz, iy, ix) in [(0, 0, 0), (3, 7, 11), (15, 23, 19), (8, 12, 10)]:
        r = np.array([ix * s.h, iy * s.h, iz * s.h])
        direct = np.sum(coef * np.cos(G @ (r - R)))
        assert abs(direct - vh[iz, iy, ix]) < 1e-11
    assert abs(np.mean(vh)) < 1e-13


def test_lda_exchange_pointwise_and_derivative():
    rho = np.array([8 * np.pi / 3, 1e-3, 0.37, -1e-14, 0.0])
    vx, ex = hamiltonian.lda_x(rho)
    assert abs(vx[0] + 2.0) < 1e-14
    assert vx[3] == 0.0 and ex[3] == 0.0
    np.testing.assert_allclose(ex[:3], 0.75 * rho[:3] * vx[:3], rtol=1e-14)
    for r in (0.37, 1e-3, 2.0):
        e = 1e-6 * r
        d = (hamiltonian.lda_x(np.array([r + e]))[1] - hamiltonian.lda_x(np.array([r - e]))[1]) / (2 * e)
        assert abs(d[0] - hamiltonian.lda_x(np.array([r]))[0][0]) < 1e-8


def _small_model(nl_rank=4, seed=11, n_orb=6):
    s = synth.make_system(16, 0.4, 2, n_orb // 2, n_orb - n_orb // 2, seed=seed, nl_rank=nl_rank,
                          region=(0.3, 0.7))
    rng = np.random.default_rng(seed)
    psi = synth.lowpass_orbitals(16, 0.4, n_orb, seed)
    q, _ = np.linalg.qr(psi.reshape(n_orb, -1).T)
    psi = q.T / np.sqrt(s.h ** 3)
    return s, oracle.Model(s, psi), rng


def test_energy_derivative_is_the_hamiltonian():
    s, m, rng = _small_model()
    N = m.N
    A = rng.standard_normal((N, N))
    S = np.diag(s.occupations()) + 0.05 * (A + A.T)
    B = rng.standard_normal((N, N))
    Ai = 0.05 * (B - B.T)
    P = S + 1j * Ai
    H, aux = m.h_of_p(P)
    X = rng.standard_normal((N, N))
    X = X + X.T
    eps = 1e-5

    def E(Pm):
        return m.energy(Pm, m.h_of_p(Pm)[1])

    dE = (E(P + eps * X) - E(P - eps * X)) / (2 * eps)
    assert abs(dE - np.sum(X * H)) < 1e-8 * max(1.0, abs(dE))


# ---------------------------------------------------------------------------
# Separable projectors
# ---------------------------------------------------------------------------
def test_projector_operator_spectrum_is_D():
    s = synth.make_system(16, 0.35, 1, 1, 1, seed=0, nl_rank=4)
    s.pos = np.array([[8 * 0.35, 7 * 0.35, 9 * 0.35]])  # on a grid point: parity makes the columns orthogonal
    s.nl_D = np.array([[0.5, 1.25, 1.75, 2.0]])
    projs = system.projectors(s)
    idx, beta, D = projs[0]
    np.testing.assert_allclose(np.sum(beta * beta, axis=0) * s.h ** 3, 1.0, rtol=1e-13)
    A = system.apply_vnl(np.eye(s.ng), projs, s.h)
    assert np.max(np.abs(A - A.T)) < 1e-13
    w = np.linalg.eigvalsh(A)
    nz = np.sort(w[np.abs(w) > 1e-8])
    np.testing.assert_allclose(nz, np.sort(s.nl_D[0]), rtol=1e-10)
    assert np.sum(np.abs(w) > 1e-8) == 4


def test_projector_sphere_has_expected_point_count():
    s = synth.make_system(48, 0.3, 1, 1, 1, seed=0, nl_rank=4)
    idx, beta, D = system.projectors(s)[0]
    expect = 4.0 / 3.0 * np.pi * (2.0 / 0.3) ** 3
    assert abs(len(idx) - expect) / expect < 0.03


# ---------------------------------------------------------------------------
# Propagator (Magnus midpoint, exponential, commutator series, kick)
# ---------------------------------------------------------------------------
def _rand_h(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) * scale
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("dt", [0.05, 0.7])
def test_spectral_exponential_matches_pade_expm(dt):
    H = _rand_h(10, 1, 2.0)
    U = propagate.expm_herm(H, dt)
    np.testing.assert_allclose(U, scipy.linalg.expm(-1j * dt * H), atol=1e-13)


@pytest.mark.parametrize("dt,seed", [(0.05, 2), (0.4, 3), (-0.3, 4)])
def test_commutator_series_equals_exact_propagation(dt, seed):
    H = _rand_h(12, seed, 1.0)  # dt * spectral width of a few units, as in real steps
    rng = np.random.default_rng(seed + 10)
    A = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
    P = A @ A.conj().T
    P1, k = propagate.propagate_series(H, P, dt, 1e-15)
    P2 = propagate.propagate_exact(H, P, dt)
    assert np.max(np.abs(P1 - P2)) < 1e-13 * np.max(np.abs(P))
    assert k > 3


def test_series_stationary_state_stops_after_one_term():
    H = np.diag(np.linspace(-1, 1, 8))
    P = np.diag([2.0] * 4 + [0.0] * 4).astype(complex)
    P1, k = propagate.propagate_series(H, P, 0.05, 1e-15)
    assert k == 1 and np.max(np.abs(P1 - P)) == 0.0


def test_kick_is_unitary():
    _, m, _ = _small_model(nl_rank=0)
    P0 = np.diag(m.sys.occupations()).astype(complex)
    P = oracle.kick(P0, m.M[0], 0.3)
    assert abs(np.trace(P) - np.trace(P0)) < 1e-13
    assert np.max(np.abs(P - P.conj().T)) < 1e-14
    assert np.max(np.abs(P @ P - 2 * P)) < 1e-13
    assert np.max(np.abs(P - P0)) > 1e-3


# ---------------------------------------------------------------------------
# Whole time loop on the 32^3 parity molecule
# ---------------------------------------------------------------------------
def test_ground_state_fixture_is_self_consistent_eigenbasis():
    psi, eps = c1_ground_state()
    m = c1_model()
    s = c1_system()
    H, _ = m.h_of_p(np.diag(s.occupations()).astype(complex))
    assert np.max(np.abs(H - np.diag(eps[: m.N]))) < 1e-9
    G = s.h ** 3 * psi.reshape(m.N, -1) @ psi.reshape(m.N, -1).T
    assert np.max(np.abs(G - np.eye(m.N))) < 1e-12
    assert eps[s.n_occ] - eps[s.n_occ - 1] > 1e-3 and eps[m.N] - eps[m.N - 1] > 1e-6


def test_frozen_hxc_dipole_closed_form():
    s = c1_system()
    psi, eps = c1_ground_state()
    base = c1_model()
    rho_gs = hamiltonian.density(np.diag(s.occupations()), base.psi)
    m = oracle.Model(s, psi, frozen_rho=rho_gs)
    rp = synth.config_run("c1_parity_32", n_steps=100)
    out = oracle.run(m, rp)
    P0 = np.diag(s.occupations()).astype(complex)
    Pk = oracle.kick(P0, m.M[0], rp.kappa)
    e = eps[: m.N]
    t = rp.dt * np.arange(rp.n_steps + 1)
    ph = np.exp(-1j * (e[:, None] - e[None, :])[None] * t[:, None, None])
    mu = np.real(np.einsum("tij,ji->t", Pk[None] * ph, m.M[0]))
    assert np.max(np.abs(mu - out["mu"][:, 0])) < 1e-9
    assert np.all(out["scf"][1:] <= 2)


def test_dipole_initial_slope_is_double_commutator():
    s = c1_system()
    psi, eps = c1_ground_state()
    out = c1_oracle_run()
    m = c1_model()
    kappa, dt = 1e-3, 0.05
    M = m.M[0]
    H0 = np.diag(eps[: m.N])
    P0 = np.diag(s.occupations())
    trk = np.trace(P0 @ (M @ (H0 @ M - M @ H0) - (H0 @ M - M @ H0) @ M))
    t = dt * np.arange(9)
    c = np.polyfit(t, out["mu"][:9, 0] - out["mu"][0, 0], 4)
    assert trk > 0
    assert abs(c[-2] - (-kappa * trk)) < 1e-4 * kappa * trk


def test_energy_and_trace_conserved_no_drift():
    out = c1_oracle_run()
    E = out["E"]
    t = 0.05 * np.arange(len(E))
    slope = np.polyfit(t[1:], E[1:] - E[1], 1)[0]
    assert abs(slope) < 1e-11
    assert np.max(np.abs(E - E[0])) < 1e-10
    assert np.max(np.abs(out["trace"] - 16.0)) < 1e-12
    P = out["P"]
    assert np.max(np.abs(P @ P - 2 * P)) < 1e-11


def test_time_reversal_of_a_step_pair():
    m = c1_model()
    rp = synth.config_run("c1_parity_32", n_steps=10)
    out = oracle.run(m, rp, record_p=True)
    Pj = out["Ps"][5]
    fwd = oracle.run(m, synth.config_run("c1_parity_32", n_steps=1), P_start=Pj)
    back = oracle.run(m, synth.config_run("c1_parity_32", n_steps=1, dt=-0.05), P_start=fwd["P"])
    assert np.max(np.abs(fwd["P"] - Pj)) > 1e-7
    assert np.max(np.abs(back["P"] - Pj)) < 1e-11


def test_series_route_matches_exact_route():
    m = c1_model()
    rp = synth.config_run("c1_parity_32", n_steps=15)
    a = oracle.run(m, rp, method="exact")
    b = oracle.run(m, rp, method="series")
    assert np.max(np.abs(a["mu"] - b["mu"])) < 1e-12
    assert np.max(np.abs(a["E"] - b["E"])) < 1e-12


def test_complete_active_space_equals_grid_propagation():
    """Brute force: with all Ng orbitals active the density-matrix step must
    equal propagating the occupied grid orbitals with exp(-i dt Hbar_grid)."""
    s = synth.make_system(8, 0.6, 1, 2, 0, seed=21, region=(0.4, 0.6), depth_range=(2.0, 3.0))
    s.n_images = 1
    d = dense_ground_state(s)
    ng = s.ng
    s.n_virt = ng - s.n_occ
    psi = d["psi_all"]
    m = oracle.Model(s, psi)
    rp = synth.RunParams(dt=0.1, n_steps=4, kappa=0.05, axis=0, h_thrs=1e-11)
    out = oracle.run(m, rp)
    # grid route
    dv = s.h ** 3
    T_nl = d["H_grid"] - np.diag(np.diag(d["H_grid"]))
    vion = system.v_ion(s).ravel()
    kin_diag = np.diag(d["H_grid"]) - (vion + hamiltonian.hartree(d["rho"], s) + hamiltonian.lda_x(d["rho"])[0])
    H_static = T_nl + np.diag(kin_diag + vion)
    x = grid.dipole_coordinate(s, 0).ravel()
    phi = (psi[: s.n_occ] * np.exp(-1j * rp.kappa * x)[None, :]).T  # [ng, n_occ]

    def hgrid(ph):
        rho = 2.0 * np.sum(np.abs(ph) ** 2, axis=1)
        return H_static + np.diag(hamiltonian.hartree(rho, s) + hamiltonian.lda_x(rho)[0]), rho

    mu = [dv * np.sum(x * 2.0 * np.sum(np.abs(phi) ** 2, axis=1))]
    Hcur, _ = hgrid(phi)
    for j in range(rp.n_steps):
        Hnew = Hcur.copy()
        for _ in range(60):
            U = scipy.linalg.expm(-1j * rp.dt * 0.5 * (Hcur + Hnew))
            ph1 = U @ phi
            Hn, _ = hgrid(ph1)
            r = np.max(np.abs(Hn - Hnew))
            Hnew = Hn
            if r < 1e-12:
                break
        phi, Hcur = ph1, Hnew
        mu.append(dv * np.sum(x * 2.0 * np.sum(np.abs(phi) ** 2, axis=1)))
    assert np.max(np.abs(np.array(mu) - out["mu"][:, 0])) < 1e-9
    assert abs(mu[-1] - mu[0]) > 1e-3


@pytest.mark.slow
def test_iterative_ground_state_matches_dense():
    s = synth.make_system(10, 0.5, 1, 2, 2, seed=5, region=(0.4, 0.6), depth_range=(2.0, 3.0))
    s.n_images = 1
    d = dense_ground_state(s)
    g = ground_state(s, tol_rho=1e-10, tol_res=1e-9)
    np.testing.assert_allclose(g["eps"][:4], d["eps"][:4], atol=1e-8)


# ---------------------------------------------------------------------------
# Spectrum
# ---------------------------------------------------------------------------
def test_spectrum_sum_rule_on_analytic_signal():
    kappa, dt = 1e-3, 0.05
    w0 = np.array([0.4, 0.9, 1.7])
    c = np.array([0.3, 1.1, 0.2])
    t = dt * np.arange(40000)
    mu = 5.0 - 4 * kappa * np.sum(c[:, None] * np.sin(w0[:, None] * t[None]), axis=0)
    om = np.linspace(0.0005, 6.0, 12000)
    S = oracle.spectrum.spectrum(mu, 5.0, dt, kappa, om, gamma=0.01)
    integral = np.trapezoid(S, om)
    assert abs(integral - np.sum(4 * w0 * c)) < 0.02 * np.sum(4 * w0 * c)
    for w in w0:
        assert S[np.argmin(np.abs(om - w))] > 0


def test_spectrum_integral_of_a_kicked_run_is_the_trk_sum():
    """The dipole strength of a real self-consistent run integrates to the
    Thomas-Reiche-Kuhn sum Tr(P0 [M, [H0, M]]) of the active space (the local
    Hartree-exchange kernel adds nothing to the double commutator).  With damping
    gamma the spectrum keeps a Lorentzian tail above the highest transition: for a
    response with dmu(0) = 0 and dmu'(0) = -kappa TRK it decays as
    4 gamma TRK / (pi w^2), so the integral up to w_max is
    TRK (1 - 4 gamma / (pi w_max)).  A wrong time scale in the propagator, kick
    strength or spectrum normalisation moves the integral by its own factor."""
    import synth

    s = c1_system()
    _, eps = c1_ground_state()
    m = c1_model()
    M = m.M[0]
    H0 = np.diag(eps[: m.N])
    P0 = np.diag(s.occupations())
    trk = np.trace(P0 @ (M @ (H0 @ M - M @ H0) - (H0 @ M - M @ H0) @ M))
    # 30 a.u.: the damped response has fallen to e^-6 of its size by the end
    rp = synth.config_run("c1_parity_32", n_steps=150, h_thrs=1e-9, dt=0.2)
    out = oracle.run(m, rp)
    mu = out["mu"][:, 0]
    gamma, w_max = 0.2, 3.0
    assert w_max > 3 * (eps[m.N - 1] - eps[0])  # above every transition of the active space
    om = np.linspace(1e-4, w_max, 30000)
    S = oracle.spectrum.spectrum(mu, mu[0], rp.dt, rp.kappa, om, gamma=gamma)
    got = np.trapezoid(S, om)
    want = trk * (1 - 4 * gamma / (np.pi * w_max))
    assert abs(got - want) < 5e-3 * trk, (got, want, trk)


# ---------------------------------------------------------------------------
# External field V_j = sum_q E_q(t_j) M_q in the midpoint (Algorithm 1)
# ---------------------------------------------------------------------------
def _frozen_c1():
    s = c1_system()
    psi, eps = c1_ground_state()
    base = c1_model()
    rho_gs = hamiltonian.density(np.diag(s.occupations()), base.psi)
    return s, eps, oracle.Model(s, psi, frozen_rho=rho_gs)


def test_constant_field_frozen_hxc_closed_form():
    """With the Hartree-exchange potential frozen, H = diag(eps) is constant; a
    constant field E0 along x makes the midpoint step exact, so
    P(t) = exp(-i (H + E0 M_x) t) P0 exp(+i (H + E0 M_x) t)."""
    s, eps, m = _frozen_c1()
    rp = synth.config_run("c1_parity_32", n_steps=60)
    rp.kappa = 0.0
    E0 = 2e-3
    out = oracle.run(m, rp, field=lambda t: (E0, 0.0, 0.0))
    Htot = np.diag(eps[: m.N]) + E0 * m.M[0]
    w, W = np.linalg.eigh(Htot)
    P0 = np.diag(s.occupations()).astype(complex)
    for j in (1, 17, 60):
        U = (W * np.exp(-1j * w * j * rp.dt)[None, :]) @ W.T
        mu = np.real(np.trace(U @ P0 @ U.conj().T @ m.M[0]))
        assert abs(mu - out["mu"][j, 0]) < 1e-9
    assert abs(out["mu"][60, 0] - out["mu"][0, 0]) > 1e-5  # the field did act


def test_pulse_midpoint_converges_at_second_order():
    """Trapezoid field average + first Magnus term: local error O(dt^3), so the
    dipole at a fixed time converges as dt^2 (frozen Hxc, sin^2 pulse)."""
    from oracle.propagate import pulse

    s, eps, m = _frozen_c1()
    T = 2.0
    f = lambda t: pulse(t, 5e-3, 1.0, T, 0.3, (1.0, 0.5, 0.0))  # noqa: E731

    def mu_end(dt):
        rp = synth.config_run("c1_parity_32", n_steps=int(round(T / dt)), dt=dt)
        rp.kappa = 0.0
        return oracle.run(m, rp, field=f)["mu"][-1]

    ref = mu_end(T / 1280)
    errs = [np.max(np.abs(mu_end(T / n) - ref)) for n in (40, 80, 160)]
    for a, b in zip(errs, errs[1:]):
        assert 3.7 < a / b < 4.3, errs


def test_weak_pulse_response_is_linear_in_amplitude():
    from oracle.propagate import pulse

    s, eps, m = _frozen_c1()
    rp = synth.config_run("c1_parity_32", n_steps=60)
    rp.kappa = 0.0
    resp = []
    for a in (1e-4, 2e-4):
        out = oracle.run(m, rp, field=lambda t, a=a: pulse(t, a, 2.0, 2.0, 0.0, (0.0, 1.0, 0.0)))
        resp.append(out["mu"] - out["mu"][0])
    d1, d2 = resp
    assert np.max(np.abs(d1)) > 1e-8
    assert np.max(np.abs(d2 - 2 * d1)) < 1e-3 * np.max(np.abs(d1))


# ---------------------------------------------------------------------------
# Fourth-order Magnus: Omega = Omega_1 + (dt^2/12)[H_0, H_1]
# ---------------------------------------------------------------------------
def test_magnus4_reduces_to_midpoint_when_hamiltonians_commute():
    """Frozen Hartree-exchange and no field: H_0 = H_1 at every step, Omega_2 = 0."""
    s, eps, m = _frozen_c1()
    rp = synth.config_run("c1_parity_32", n_steps=30)
    a = oracle.run(m, rp)
    b = oracle.run(m, rp, magnus_order=4)
    assert np.max(np.abs(a["mu"] - b["mu"])) < 1e-11  # rounding of the complex eigensolver path


def test_magnus4_converges_at_fourth_order_for_a_linear_hamiltonian():
    """H(t) = H + alpha t M_x is linear in t (frozen Hxc, field ramp): the two-term
    Magnus step has local error O(dt^5), the midpoint O(dt^3)."""
    s, eps, m = _frozen_c1()
    T, alpha = 2.0, 0.05
    ramp = lambda t: (alpha * t, 0.0, 0.0)  # noqa: E731

    def mu_end(n, order):
        rp = synth.config_run("c1_parity_32", n_steps=n, dt=T / n)
        rp.kappa = 0.0
        return oracle.run(m, rp, field=ramp, magnus_order=order)["mu"][-1]

    ref = mu_end(640, 4)
    e4 = [np.max(np.abs(mu_end(n, 4) - ref)) for n in (10, 20, 40)]
    e2 = [np.max(np.abs(mu_end(n, 2) - ref)) for n in (10, 20, 40)]
    for a, b in zip(e4, e4[1:]):
        assert 13.0 < a / b < 19.0, e4
    for a, b in zip(e2, e2[1:]):
        assert 3.5 < a / b < 4.5, e2
    assert e4[-1] < 1e-2 * e2[-1]


def test_magnus4_self_consistent_run_keeps_trace_and_idempotency():
    rp = synth.config_run("c1_parity_32", n_steps=20, dt=0.2)
    out = oracle.run(c1_model(), rp, magnus_order=4, record_p=True, method="series")
    assert np.max(np.abs(out["trace"] - 16.0)) < 1e-12
    for P in out["Ps"][::5]:
        assert np.max(np.abs(P @ P / 2.0 - P)) < 1e-11


# ---------------------------------------------------------------------------
# Non-orthogonal basis: dP^(k) = (1/k)(-i dt)(S^-1 Hbar dP - dP Hbar S^-1)
# (eq. commutator-expansion-nonort; Appendix, propagation in a non-orthogonal basis)
# ---------------------------------------------------------------------------
def _rand_spd(n, seed):
    A = synth.basis_mixing(n, seed, strength=0.6)
    return A @ A.T


@pytest.mark.parametrize("dt,seed", [(0.05, 21), (0.3, 22), (-0.2, 23)])
def test_nonorthogonal_step_matches_pade_exponential(dt, seed):
    """For constant Hbar, eq. LvN_nonort is solved by
    P(dt) = exp(-i dt S^-1 H) P exp(+i dt H S^-1); scipy's Pade exponential of the
    non-symmetric S^-1 H is an independent route to both the series and the
    orthonormal-basis transform."""
    n = 10
    S = _rand_spd(n, seed)
    H = _rand_h(n, seed + 1)
    rng = np.random.default_rng(seed + 2)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    P = A @ A.conj().T
    G = np.linalg.solve(S, H)
    ref = scipy.linalg.expm(-1j * dt * G) @ P @ scipy.linalg.expm(1j * dt * G.T)
    ser, k = propagate.propagate_series(H, P, dt, 1e-15, Sinv=np.linalg.inv(S))
    ex = propagate.propagate_exact_nonorth(H, P, dt, S)
    scale = np.max(np.abs(P))
    assert np.max(np.abs(ser - ref)) < 1e-12 * scale
    assert np.max(np.abs(ex - ref)) < 1e-12 * scale
    assert k > 3


def test_nonorthogonal_series_with_unit_overlap_is_the_commutator_series():
    H = _rand_h(8, 31)
    P = propagate.kick(np.diag([2.0] * 3 + [0.0] * 5), _rand_h(8, 32), 0.3)
    a, ka = propagate.propagate_series(H, P, 0.2, 1e-15)
    b, kb = propagate.propagate_series(H, P, 0.2, 1e-15, Sinv=np.eye(8))
    assert ka == kb
    assert np.max(np.abs(a - b)) < 1e-15


def test_nonorthogonal_ground_density_is_idempotent_in_the_metric():
    """P_0 = R^-1 diag(f) L^-1 with f in {0, 2}: (P S)^2 = 2 P S, Tr(P S) = N_e."""
    S = _rand_spd(9, 41)
    occ = np.array([2.0] * 4 + [0.0] * 5)
    P = propagate.ground_density_nonorth(occ, S)
    PS = P @ S
    assert np.max(np.abs(PS @ PS - 2.0 * PS)) < 1e-12
    assert abs(np.trace(PS) - 8.0) < 1e-12


def _nonorth_c1(mixing_seed, lower):
    """The 32^3 parity molecule in the basis Phi = A Psi, with its overlap."""
    psi, _ = c1_ground_state()
    s = c1_system()
    N = psi.shape[0]
    A = synth.basis_mixing(N, mixing_seed, strength=0.4, lower=lower)
    phi = A @ psi.reshape(N, -1)
    S = s.h ** 3 * (phi @ phi.T)
    return A, oracle.Model(s, phi.reshape(psi.shape)), 0.5 * (S + S.T)


def test_nonorthogonal_run_reproduces_orthonormal_physics_lower_triangular_basis():
    """Phi = A Psi with A unit lower triangular: the Cholesky factor of Phi's overlap
    is A, so the default P_0 occupies the same orbitals; mu(t), E(t) and the
    electron count must equal the orthonormal run (basis-invariant observables,
    Appendix trace identities)."""
    A, m, S = _nonorth_c1(51, lower=True)
    assert np.max(np.abs(np.linalg.cholesky(S) - A)) < 1e-10
    rp = synth.config_run("c1_parity_32", n_steps=20, h_thrs=1e-12)
    ref = c1_oracle_run(n_steps=20)
    for method in ("exact", "series"):
        out = oracle.run(m, rp, method=method, S=S)
        assert np.max(np.abs(out["mu"] - ref["mu"])) < 1e-10, method
        assert np.max(np.abs(out["E"] - ref["E"])) < 1e-9, method
        assert np.max(np.abs(out["trace"] - 16.0)) < 1e-11, method


def test_nonorthogonal_run_reproduces_orthonormal_physics_general_basis():
    """A general mixing A: the ground state in Phi is P_0 = A^-T diag(f) A^-1; kicked
    through S it must give the orthonormal run's dipole history."""
    A, m, S = _nonorth_c1(52, lower=False)
    rp = synth.config_run("c1_parity_32", n_steps=20, h_thrs=1e-12)
    Ai = np.linalg.inv(A)
    P0 = Ai.T @ np.diag(c1_system().occupations()) @ Ai
    P = propagate.kick(P0, m.M[rp.axis], rp.kappa, S)
    out = oracle.run(m, rp, method="series", S=S, P_start=P)
    ref = c1_oracle_run(n_steps=20)
    assert np.max(np.abs(out["mu"] - ref["mu"])) < 1e-10
    assert np.max(np.abs(out["trace"] - 16.0)) < 1e-11


# ---------------------------------------------------------------------------
# Quadratic first guess 3 H_0 - 3 H_-1 + H_-2 (a predictor option: same fixed point)
# ---------------------------------------------------------------------------
def _guess_errors(dt, t_end, predictor):
    """max |guess - converged H| at the steps that end near t_end, on a tightly
    converged trajectory of the parity molecule."""
    n = int(round(t_end / dt))
    rp = synth.config_run("c1_parity_32", n_steps=n + 1, dt=dt, h_thrs=1e-13)
    m = c1_model()
    out = oracle.run(m, rp, record_p=True)
    H = [m.h_of_p(P)[0] for P in out["Ps"]]
    j = n
    if predictor == "linear":
        g = 2 * H[j - 1] - H[j - 2]
    else:
        g = 3 * H[j - 1] - 3 * H[j - 2] + H[j - 3]
    return np.max(np.abs(g - H[j]))


def test_quadratic_guess_error_is_third_order_in_dt():
    """The linear guess misses the converged H by O(dt^2), the quadratic one by
    O(dt^3): halving dt at a fixed time divides them by ~4 and ~8."""
    el = [_guess_errors(dt, 1.6, "linear") for dt in (0.2, 0.1)]
    eq = [_guess_errors(dt, 1.6, "quadratic") for dt in (0.2, 0.1)]
    assert 3.0 < el[0] / el[1] < 5.0, el
    assert 6.0 < eq[0] / eq[1] < 10.0, eq
    assert eq[1] < 0.2 * el[1]


def test_quadratic_predictor_keeps_the_fixed_point_and_saves_updates():
    tight = synth.config_run("c1_parity_32", n_steps=40, dt=0.2, h_thrs=1e-12)
    a = oracle.run(c1_model(), tight)
    b = oracle.run(c1_model(), tight, predictor="quadratic")
    assert np.max(np.abs(a["mu"] - b["mu"])) < 1e-10
    paper = synth.config_run("c1_parity_32", n_steps=40, dt=0.2, h_thrs=1e-7)
    lin = oracle.run(c1_model(), paper)
    quad = oracle.run(c1_model(), paper, predictor="quadratic")
    assert np.mean(quad["scf"][3:]) < np.mean(lin["scf"][3:]) - 0.3, (np.mean(lin["scf"][3:]), np.mean(quad["scf"][3:]))
    assert np.max(np.abs(quad["mu"] - a["mu"])) < 1e-6
