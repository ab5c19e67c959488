"""Kohn-Sham Hamiltonian in the orbital basis as a function of the density
matrix, H[P] = DFT(rho(P)) (oracle; test infrastructure only).

Paper passages:
  * Eq. DFT (Sec. Overview of RMG): H = kinetic + V_eff with V_eff = ionic
    (local + nonlocal) + Hartree + exchange-correlation.  The printed sign of the
    Laplacian term is +1/2; the kinetic operator is read as -1/2 Laplacian.
  * Algorithm 1: H_1 <- DFT(rho(P_1)); matrix elements <psi_i|H|psi_j> over the
    active space (Sec. Algorithm, active-space matrices).
  * Sec. Theory, density matrix P = sum_i f_i |psi_i><psi_i|: with real Gamma-point
    orbitals the density is rho(r) = sum_ij Re(P_ij) psi_i(r) psi_j(r).
  * Hartree by FFT (spectral Poisson, zero G = 0 component: neutralising
    background) and Slater LDA exchange stand in for RMG's multigrid Poisson and
    PBE; both are fixed choices of this synthetic workload.
  * Sec. Algorithm, time-dependent field: the constant field is a sawtooth
    potential with a dipole correction in the vacuum (Bengtsson, Phys. Rev. B
    59, 12301 (1999)).  Reading: along every axis q selected by the system's
    dipole_correction bit mask, the electrons' dipole d_q = h^3 sum rho s_q
    (s_q the sawtooth coordinate, jump in the vacuum) minus that of the ions
    taken as point charges adds the potential (4 pi / Omega) d_q s_q and the
    energy (2 pi / Omega) d_q^2, Omega the cell volume.  This cancels the
    spurious uniform field that the periodic images of the dipole set up across
    the cell (exact for a charge that varies along q only), and H[P] stays the
    derivative of E[P].  The synthetic ionic wells are not Coulombic, so their
    point charges are an input of the system (default: the electron count
    shared equally, a neutral cell).
"""

import numpy as np

from .grid import fd_coefficients_float, laplacian, dipole_coordinate
from .system import v_ion, projectors, apply_vnl

CX = (3.0 / np.pi) ** (1.0 / 3.0)


def density(Pr: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """rho(r) = sum_ij Pr_ij psi_i(r) psi_j(r) for a real symmetric Pr = Re(P)."""
    return np.sum((Pr @ psi) * psi, axis=0)


def g_squared(sys) -> np.ndarray:
    """|G|^2 on the FFT grid [nz, ny, nx], G = 2 pi m / L, m from the FFT
    frequency order (the Nyquist row of an even grid keeps its squared value)."""
    nx, ny, nz = sys.n
    h = sys.h
    gx = 2 * np.pi * np.fft.fftfreq(nx, d=h)
    gy = 2 * np.pi * np.fft.fftfreq(ny, d=h)
    gz = 2 * np.pi * np.fft.fftfreq(nz, d=h)
    return gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2


def hartree(rho: np.ndarray, sys) -> np.ndarray:
    """Periodic Hartree potential: V_H(G) = 4 pi rho(G) / |G|^2, V_H(G=0) = 0."""
    nx, ny, nz = sys.n
    g2 = g_squared(sys)
    rg = np.fft.fftn(rho.reshape(nz, ny, nx))
    with np.errstate(divide="ignore", invalid="ignore"):
        vg = np.where(g2 > 0, 4.0 * np.pi * rg / np.where(g2 > 0, g2, 1.0), 0.0)
    return np.fft.ifftn(vg).real.ravel()


def ion_charges(sys) -> np.ndarray:
    """Point charges of the ions for the dipole correction: sys.ion_charge, or
    the electron count sum_i f_i shared equally between the atoms (a neutral
    cell)."""
    q = getattr(sys, "ion_charge", None)
    if q is not None:
        return np.asarray(q, dtype=np.float64)
    if sys.n_atoms == 0:
        return np.zeros(0)
    return np.full(sys.n_atoms, float(np.sum(sys.occupations())) / sys.n_atoms)


def sawtooth_at(x: np.ndarray, sys, axis: int) -> np.ndarray:
    """The sawtooth coordinate at arbitrary positions x along the axis: the
    continuous form of the grid's (((x/h - j0) mod n) - (n-1)/2) h."""
    h = sys.h
    n = sys.n[axis]
    j0 = int(getattr(sys, "saw_jump", (0, 0, 0))[axis])
    return (np.mod(np.asarray(x) / h - j0, n) - 0.5 * (n - 1)) * h


def dipole_correction(rho: np.ndarray, sys):
    """Vacuum dipole correction of a density: (v_dc on the grid, E_dc).

    For each axis q in the bit mask sys.dipole_correction the dipole of the
    cell's charge, written for electrons as d_q = h^3 sum_r rho(r) s_q(r) -
    sum_a Z_a s_q(R_a) (electrons minus ion point charges), gives
    v_dc += (4 pi / Omega) d_q s_q and E_dc += (2 pi / Omega) d_q^2, so that
    dE_dc / d rho(r) = h^3 v_dc(r).  No mask: (0, 0)."""
    mask = int(getattr(sys, "dipole_correction", 0))
    if not mask:
        return 0.0, 0.0
    omega = float(np.prod(sys.cell))
    dv = sys.h ** 3
    z = ion_charges(sys)
    v = np.zeros(sys.ng)
    e = 0.0
    for q in range(3):
        if (mask >> q) & 1:
            s = dipole_coordinate(sys, q).ravel()
            d = dv * float(np.sum(rho * s))
            if sys.n_atoms:
                d -= float(np.sum(z * sawtooth_at(sys.pos[:, q], sys, q)))
            v += (4.0 * np.pi / omega) * d * s
            e += (2.0 * np.pi / omega) * d * d
    return v, e


def electrostatic(rho: np.ndarray, sys):
    """Electron-electron electrostatic potential and energy: periodic Hartree
    plus the vacuum dipole correction, (V_H + v_dc, E_H + E_dc)."""
    vh = hartree(rho, sys)
    vdc, edc = dipole_correction(rho, sys)
    dv = sys.h ** 3
    e = 0.5 * dv * float(np.sum(rho * vh)) + edc
    return vh + vdc, e


def lda_x(rho: np.ndarray):
    """Slater exchange of the spin-unpolarised gas: v_x = -(3 rho / pi)^(1/3),
    energy density e_x = -(3/4) (3/pi)^(1/3) rho^(4/3); rho clipped at 0."""
    rc = np.maximum(rho, 0.0)
    c = np.cbrt(rc)
    vx = -CX * c
    ex = -0.75 * CX * rc * c
    return vx, ex


class Model:
    """The fixed ingredients of one trajectory: orbitals Psi[N, Ng] (real,
    h^3-orthonormal), ionic terms, dipole matrices M_q and the constant part
    H_core = h^3 Psi^T (T + V_ion + V_nl) Psi."""

    def __init__(self, sys, psi: np.ndarray, frozen_rho: np.ndarray = None, fd_mix_M: float = 0.0):
        self.sys = sys
        self.h = sys.h
        self.dv = sys.h ** 3
        n_orb = psi.shape[0]
        self.N = n_orb
        self.psi = np.ascontiguousarray(psi.reshape(n_orb, sys.ng), dtype=np.float64)
        self.coeffs = fd_coefficients_float(4, fd_mix_M)
        self.vion = v_ion(sys).ravel()
        self.projs = projectors(sys)
        self.occ = sys.occupations()[:n_orb] if n_orb == sys.n_orb else None
        self.qs = [dipole_coordinate(sys, ax).ravel() for ax in range(3)]
        self.M = np.stack([self.project_local(q) for q in self.qs])
        self.frozen_rho = frozen_rho
        tpsi = self.apply_h(self.psi, self.vion)
        self.hcore = self.project(tpsi)

    # --- grid operators -------------------------------------------------
    def apply_h(self, psi: np.ndarray, vloc: np.ndarray) -> np.ndarray:
        """(H psi_j) = -1/2 L_FD psi_j + v_loc psi_j + V_nl psi_j for every row of psi."""
        sys = self.sys
        nx, ny, nz = sys.n
        out = np.empty_like(psi)
        for j in range(psi.shape[0]):
            f = psi[j].reshape(nz, ny, nx)
            out[j] = (-0.5 * laplacian(f, self.h, self.coeffs)).ravel() + vloc * psi[j]
        if self.projs:
            out += apply_vnl(psi, self.projs, self.h)
        return out

    def project(self, hpsi: np.ndarray) -> np.ndarray:
        """Active-space matrix h^3 Psi (H Psi)^T, symmetrised (A + A^T)/2."""
        a = self.dv * (self.psi @ hpsi.T)
        return 0.5 * (a + a.T)

    def project_local(self, v: np.ndarray) -> np.ndarray:
        """h^3 Psi diag(v) Psi^T (dipole matrices, local potentials)."""
        a = self.dv * ((self.psi * v[None, :]) @ self.psi.T)
        return 0.5 * (a + a.T)

    # --- density functional ---------------------------------------------
    def potentials(self, rho: np.ndarray):
        """Electrostatic (Hartree plus dipole correction) and exchange
        potentials and energies of a density.  With a frozen density (test
        mode) the potentials are those of the frozen density, so H[P] is
        constant."""
        src = rho if self.frozen_rho is None else self.frozen_rho
        vh, e_h = electrostatic(src, self.sys)
        vx, ex = lda_x(src)
        e_x = self.dv * float(np.sum(ex))
        return vh, vx, e_h, e_x

    def h_of_p(self, P: np.ndarray):
        """H[P] = h^3 Psi^T [T + V_ion + V_nl + V_H(rho) + v_x(rho)] Psi with
        rho = rho(P), the Hamiltonian applied in full to every orbital."""
        rho = density(P.real, self.psi)
        vh, vx, e_h, e_x = self.potentials(rho)
        hpsi = self.apply_h(self.psi, self.vion + vh + vx)
        H = self.project(hpsi)
        return H, dict(rho=rho, vh=vh, vx=vx, e_h=e_h, e_x=e_x, H=H)

    # --- observables -----------------------------------------------------
    def dipole(self, P: np.ndarray) -> np.ndarray:
        """mu_q = Tr(P M_q), mu_0 = 0 (Algorithm 1, analysis block)."""
        return np.array([np.real(np.trace(P @ self.M[q])) for q in range(3)])

    def energy(self, P: np.ndarray, aux) -> float:
        """E = Tr(Re P H_core) + E_H + E_x, whose derivative with respect to P is
        H[P] (the paper plots E but does not define it).  With a frozen density
        H is constant and the conserved energy is Tr(Re P H)."""
        if self.frozen_rho is not None:
            return float(np.sum(P.real * aux["H"]))
        return float(np.sum(P.real * self.hcore)) + aux["e_h"] + aux["e_x"]
