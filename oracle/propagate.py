"""Density-matrix propagation (oracle; test infrastructure only).

Paper passages:
  * Magnus expansion, first term for a Hamiltonian linear over the step:
    Omega_1 = -i dt (H_0 + H_1)/2 (Sec. Magnus expansion, eq. omega1a).
  * Spectral propagator U = W exp(omega) W^dagger from the eigenpairs of Omega
    (same section) and P(t) = U P(0) U^dagger (Sec. Density matrix propagation,
    eq. UxP0xU).
  * Commutator expansion P(t + dt) = P + sum_k dP^(k),
    dP^(k) = (1/k)(-i dt)[Hbar, dP^(k-1)] for an orthonormal basis
    (eq. commutator-expansion-ort), stopped when max|dP| <= dP_thrs (Algorithm 1).
  * Self-consistent midpoint loop of Algorithm 1: predictor H_1 = 2 H_0 - H_-1
    (or, as an option that changes only the number of updates, the quadratic
    extrapolation 3 H_0 - 3 H_-1 + H_-2 through the last three steps),
    repeat { Omega from (H_0 + H_1)/2; propagate; H_1 <- DFT(rho(P_1)) } until
    the update of H_1 is below H_thrs; then shift H_-1 <- H_0, H_0 <- H_1,
    P_0 <- P_1.
  * Delta-kick perturbation (Sec. Numerical Results, kick equation).
  * External field (Algorithm 1 inputs and Magnus line): V_j = sum_q E_q(t_j) M_q
    enters the midpoint as Omega = -i dt (H_0 + H_1 + V_(j-1) + V_j)/2, t_j = j dt.
  * Fourth-order Magnus (Sec. Magnus expansion, eq. omega2 for a Hamiltonian
    linear over the step): Omega = Omega_1 + Omega_2, Omega_2 = (dt^2/12)[H_0, H_1];
    the series becomes dP^(k) = (1/k)(Omega dP^(k-1) + dP^(k-1) Omega^dagger)
    (eq. commutator-expansion-general).
  * Non-orthogonal basis with overlap S (Sec. Density matrix propagation,
    eq. LvN_nonort and eq. commutator-expansion-nonort; Appendix, propagation
    in a non-orthogonal basis): dP^(k) = (1/k)(-i dt)(S^-1 Hbar dP^(k-1) -
    dP^(k-1) Hbar S^-1).  The exact reference goes through the orthonormal
    basis of the Appendix's transformation rules with S = L R, R = L^T
    (Cholesky): H_o = L^-1 H_n R^-1, P_o = R P_n L, back by P_n = R^-1 P_o L^-1.

Readings where the paper is silent:
  * The kick is an instantaneous unitary at t = 0+, P(0+) = e^{-i kappa M_q}
    P_0 e^{+i kappa M_q}; afterwards the field is zero.  H_0 = H[P(0+)],
    H_-1 = H_0.
  * The self-consistency residual compares each new H_1 with the H_1 that built
    Omega, so every step does at least one Hamiltonian update.
  * The series is not stopped before k >= ceil(dt * w), w the Gershgorin width
    of Hbar, so a term on the rising part of the series cannot end it.
  * The field's time origin is the kick (t_0 = 0); the self-consistency residual
    compares Kohn-Sham Hamiltonians only (the field matrix is known exactly).
  * Pulse shape (the paper names no shape): E(t) = a sin^2(pi t / tau)
    sin(omega t + phase) along a fixed direction for 0 <= t <= tau, zero after.
  * Omega_2 takes the full endpoint Hamiltonians including the field,
    [H_0 + V_(j-1), H_1 + V_j]; its series stop floor is the Gershgorin width of
    the Hermitian matrix i Omega.
  * Non-orthogonal basis: the initial density matrix occupies the first n_occ
    vectors of the basis orthonormalised by the Cholesky factor of S (the basis
    transform the paper names), P_0 = R^-1 diag(f) L^-1; the kick and the field
    act through S^-1 M_q like the Hamiltonian; the electron count is Tr(P S);
    the series stop floor is the Gershgorin width of S^-1 Hbar (row discs; its
    eigenvalues, those of the pencil (Hbar, S), are real).  Fourth-order Magnus
    is not combined with a non-orthogonal basis here.
"""

import math

import numpy as np


class NoConvergence(RuntimeError):
    pass


def expm_herm(Hbar: np.ndarray, dt: float) -> np.ndarray:
    """U = exp(-i dt Hbar) for real symmetric Hbar, spectral form W e^{-i dt w} W^T."""
    w, W = np.linalg.eigh(Hbar)
    return (W * np.exp(-1j * dt * w)[None, :]) @ W.T


def propagate_exact(Hbar: np.ndarray, P: np.ndarray, dt: float) -> np.ndarray:
    """P -> U P U^dagger with the exact exponential of Omega_1 = -i dt Hbar."""
    U = expm_herm(Hbar, dt)
    return U @ P @ U.conj().T


def gershgorin_width(A: np.ndarray) -> float:
    """Width of the interval spanned by the Gershgorin row discs of real A (centre
    a_ii, radius sum_j!=i |a_ij|); it encloses the spectrum when that is real
    (A symmetric, or A = S^-1 H with S positive definite and H symmetric)."""
    d = np.diag(A)
    r = np.sum(np.abs(A), axis=1) - np.abs(d)
    return float(np.max(d + r) - np.min(d - r))


def propagate_omega_exact(omega: np.ndarray, P: np.ndarray) -> np.ndarray:
    """P -> U P U^dagger, U = exp(Omega) for anti-Hermitian Omega, from the eigenpairs
    of the Hermitian matrix i Omega (spectral form of the Magnus propagator)."""
    w, W = np.linalg.eigh(1j * omega)
    U = (W * np.exp(-1j * w)[None, :]) @ W.conj().T
    return U @ P @ U.conj().T


def overlap_factor(S: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor L of the overlap, S = L L^T (so R = L^T)."""
    return np.linalg.cholesky(S)


def propagate_exact_nonorth(Hbar: np.ndarray, P: np.ndarray, dt: float, S: np.ndarray) -> np.ndarray:
    """Exact step in a non-orthogonal basis: to the orthonormal basis by the
    Appendix's rules (H_o = L^-1 H R^-1, P_o = R P L), the spectral propagator
    there, and back (P = R^-1 P_o L^-1), with S = L R, R = L^T."""
    L = overlap_factor(S)
    Li = np.linalg.inv(L)
    Ho = Li @ Hbar @ Li.T
    Po = L.T @ P @ L
    Po = propagate_exact(0.5 * (Ho + Ho.T), Po, dt)
    return Li.T @ Po @ Li


def ground_density_nonorth(occ: np.ndarray, S: np.ndarray) -> np.ndarray:
    """P_0 = R^-1 diag(f) L^-1: occupations of the Cholesky-orthonormalised basis,
    written in the non-orthogonal basis."""
    Li = np.linalg.inv(overlap_factor(S))
    return Li.T @ np.diag(occ) @ Li


def gershgorin_width_herm(X: np.ndarray) -> float:
    """Width of the Gershgorin interval of a Hermitian matrix (centres Re x_ii)."""
    d = np.real(np.diag(X))
    r = np.sum(np.abs(X), axis=1) - np.abs(np.diag(X))
    return float(np.max(d + r) - np.min(d - r))


def omega2(A0: np.ndarray, A1: np.ndarray, dt: float) -> np.ndarray:
    """Second Magnus term for a Hamiltonian linear over the step: (dt^2/12)[A0, A1]."""
    return dt * dt / 12.0 * (A0 @ A1 - A1 @ A0)


def propagate_series(Hbar: np.ndarray, P: np.ndarray, dt: float, thrs: float, max_terms: int = 200,
                     B: np.ndarray = None, Sinv: np.ndarray = None):
    """Commutator series for P(t + dt): dP^(0) = P,
    dP^(k) = (1/k) (Omega dP^(k-1) + dP^(k-1) Omega^dagger) with Omega = -i dt Hbar (+ B,
    the real antisymmetric Omega_2 when given), i.e. (1/k)[Omega, dP^(k-1)]; summed
    until max|dP^(k)| <= thrs.  With the inverse overlap Sinv of a non-orthogonal
    basis, Omega = -i dt Sinv Hbar, and Omega dP + dP Omega^dagger is
    -i dt (S^-1 Hbar dP - dP Hbar S^-1).  Returns (P(t + dt), number of terms)."""
    omega = -1j * dt * Hbar
    if Sinv is not None:
        if B is not None:
            raise NotImplementedError("Omega_2 with a non-orthogonal basis")
        G = Sinv @ Hbar
        omega = -1j * dt * G
        k_min = math.ceil(abs(dt) * gershgorin_width(G))
    elif B is None:
        k_min = math.ceil(dt * gershgorin_width(Hbar))
    else:
        omega = omega + B
        k_min = math.ceil(gershgorin_width_herm(1j * omega))
    P1 = P.astype(np.complex128).copy()
    dP = P1.copy()
    k = 0
    while True:
        k += 1
        if k > max_terms:
            raise NoConvergence("commutator series exceeded max_terms")
        dP = (omega @ dP + dP @ omega.conj().T) / k
        P1 += dP
        if k >= k_min and np.max(np.abs(dP)) <= thrs:
            return P1, k


def kick(P0: np.ndarray, M: np.ndarray, kappa: float, S: np.ndarray = None) -> np.ndarray:
    """Instantaneous delta kick: P(0+) = exp(-i kappa M) P_0 exp(+i kappa M)
    (through the orthonormal basis when the overlap S is given)."""
    if S is not None:
        return propagate_exact_nonorth(M, P0.astype(np.complex128), kappa, S)
    return propagate_exact(M, P0.astype(np.complex128), kappa)


def pulse(t: float, amp: float, omega: float, tau: float, phase: float = 0.0, direction=(1.0, 0.0, 0.0)):
    """Field vector (E_x, E_y, E_z) of a sin^2-envelope pulse at time t."""
    if t < 0.0 or t > tau:
        return np.zeros(3)
    return amp * math.sin(math.pi * t / tau) ** 2 * math.sin(omega * t + phase) * np.asarray(direction, float)


def field_matrix(model, e3) -> np.ndarray:
    """V = E_x M_x + E_y M_y + E_z M_z (Algorithm 1, perturbation matrix)."""
    return e3[0] * model.M[0] + e3[1] * model.M[1] + e3[2] * model.M[2]


def run(model, rp, method: str = "exact", predictor: str = "linear", record_p: bool = False,
        P_start=None, H_start=None, field=None, magnus_order: int = 2, S=None):
    """Self-consistent midpoint time loop (Algorithm 1, time integration block).

    method: "exact" (spectral exponential, the fixed point the method converges
    to) or "series" (the commutator series of Algorithm 1).
    field: optional callable t -> (E_x, E_y, E_z); V(t) = sum_q E_q(t) M_q is
    added to the midpoint Hamiltonian as (V(t_(j-1)) + V(t_j))/2.
    magnus_order: 2 (Omega_1, the paper's midpoint) or 4 (adds Omega_2).
    S: overlap of a non-orthogonal basis (the model's orbitals), or None for an
    orthonormal one; then P_0 = R^-1 diag(f) L^-1, every step goes through
    S^-1, and trace reports Tr(P S).
    Returns a dict with per-step dipole mu[j, 3], energy E[j], trace N[j],
    update counts scf[j] and series terms.
    """
    N = model.N
    if S is not None and magnus_order == 4:
        raise NotImplementedError("Omega_2 with a non-orthogonal basis")
    Sinv = None if S is None else np.linalg.inv(S)
    if P_start is None:
        occ = model.sys.occupations()[:N]
        P0 = (np.diag(occ) if S is None else ground_density_nonorth(occ, S)).astype(np.complex128)
        P = kick(P0, model.M[rp.axis], rp.kappa, S) if rp.kappa else P0
    else:
        P = P_start.astype(np.complex128)

    def electrons(P):
        return float(np.real(np.trace(P if S is None else P @ S)))

    H0, aux = model.h_of_p(P)
    if H_start is not None:
        Hm1 = H_start
    else:
        Hm1 = H0.copy()
    Hm2 = Hm1.copy()
    mu = [model.dipole(P)]
    E = [model.energy(P, aux)]
    tr = [electrons(P)]
    scf, terms = [0], [0]
    Ps = [P.copy()] if record_p else None
    for j in range(1, rp.n_steps + 1):
        if predictor == "linear":
            H1 = 2.0 * H0 - Hm1
        elif predictor == "quadratic":
            H1 = 3.0 * H0 - 3.0 * Hm1 + Hm2
        else:
            H1 = H0.copy()
        n_terms = 0
        Va = Vb = 0.0
        if field is not None:
            Va, Vb = field_matrix(model, field((j - 1) * rp.dt)), field_matrix(model, field(j * rp.dt))
        Vbar = 0.5 * (Va + Vb)
        for m in range(1, rp.max_scf + 1):
            Hbar = 0.5 * (H0 + H1) + Vbar
            B = omega2(H0 + Va, H1 + Vb, rp.dt) if magnus_order == 4 else None
            if method == "exact":
                if S is not None:
                    P1 = propagate_exact_nonorth(Hbar, P, rp.dt, S)
                elif B is None:
                    P1 = propagate_exact(Hbar, P, rp.dt)
                else:
                    P1 = propagate_omega_exact(-1j * rp.dt * Hbar + B, P)
            else:
                P1, kk = propagate_series(Hbar, P, rp.dt, rp.dp_thrs, rp.max_terms, B, Sinv)
                n_terms += kk
            Hn, aux = model.h_of_p(P1)
            r = float(np.max(np.abs(Hn - H1)))
            H1 = Hn
            if r <= rp.h_thrs:
                break
        else:
            raise NoConvergence(f"self-consistent loop did not converge at step {j}")
        Hm2, Hm1, H0, P = Hm1, H0, H1, P1
        mu.append(model.dipole(P))
        E.append(model.energy(P, aux))
        tr.append(electrons(P))
        scf.append(m)
        terms.append(n_terms)
        if record_p:
            Ps.append(P.copy())
    out = dict(mu=np.array(mu), E=np.array(E), trace=np.array(tr), scf=np.array(scf),
               terms=np.array(terms), P=P, H0=H0, Hm1=Hm1)
    if record_p:
        out["Ps"] = Ps
    return out
