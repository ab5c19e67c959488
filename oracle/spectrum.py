"""Photoabsorption spectrum from the dipole history (oracle; test
infrastructure only).

Sec. Numerical Results: the spectrum is the sum of Fourier transforms of
mu_x(t), mu_y(t), mu_z(t) from three runs kicked along x, y, z.  The paper
does not state the damping, window or normalisation.  The printed dipole
mu = mu_0 + Tr(P M) (Algorithm 1) is the electrons' position expectation; their
charge dipole is its negative, so the reading used here is

  S_q(w) = -(2 w / (pi kappa)) Im sum_j dt c_j [mu_q(t_j) - mu_q(0-)] e^{(i w - gamma) t_j}

with trapezoid weights c_j and damping gamma: S >= 0 at the resonances, and
its integral over w approaches the Thomas-Reiche-Kuhn sum of the active space,
Tr(P_0 [M, [H, M]]), as gamma -> 0.
"""

import numpy as np


def spectrum(mu_q: np.ndarray, mu_ref: float, dt: float, kappa: float, omegas: np.ndarray,
             gamma: float = 0.01) -> np.ndarray:
    """Dipole strength S_q(w) for one kick direction q (mu_q: history along q)."""
    t = dt * np.arange(len(mu_q))
    c = np.ones(len(mu_q))
    c[0] = c[-1] = 0.5
    d = (mu_q - mu_ref) * c * dt * np.exp(-gamma * t)
    ft = np.exp(1j * np.outer(omegas, t)) @ d
    return -2.0 * omegas / (np.pi * kappa) * np.imag(ft)
