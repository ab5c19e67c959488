"""Grid, finite-difference Laplacian and quadrature (oracle; test infrastructure only).

Paper passages: Sec. "Overview of RMG" -- the 2n+1-point central difference
formula whose coefficients make the second derivative exact for polynomials of
degree up to 2n, used with n = 4; the grid expectation value (quadrature weight
h per point in 1-D, h^3 per point on the 3-D grid).
"""

from fractions import Fraction

import numpy as np
from scipy.ndimage import correlate1d


def fd_coefficients(n_half: int = 4):
    """Exact rational coefficients a_0..a_n of the symmetric 2n+1-point second
    derivative on unit spacing (Sec. Overview of RMG, central difference formula).

    Conditions: applied to x^(2m) at x = 0 the stencil must return the exact
    second derivative, i.e. 2 for m = 1 and 0 for every other m = 0..n (odd
    powers cancel by symmetry).  Solved by exact Gaussian elimination.
    """
    n = n_half
    # Unknowns a_0..a_n.  Row m: a_0 * [m == 0] + sum_k 2 a_k k^(2m) = rhs_m.
    rows = []
    for m in range(n + 1):
        row = [Fraction(1 if m == 0 else 0)]
        for k in range(1, n + 1):
            row.append(Fraction(2 * k ** (2 * m)))
        rhs = Fraction(2 if m == 1 else 0)
        rows.append(row + [rhs])
    # Gauss-Jordan in exact arithmetic.
    size = n + 1
    for c in range(size):
        piv = next(r for r in range(c, size) if rows[r][c] != 0)
        rows[c], rows[piv] = rows[piv], rows[c]
        p = rows[c][c]
        rows[c] = [v / p for v in rows[c]]
        for r in range(size):
            if r != c and rows[r][c] != 0:
                f = rows[r][c]
                rows[r] = [a - f * b for a, b in zip(rows[r], rows[c])]
    return [rows[i][size] for i in range(size)]


def fd_coefficients_float(n_half: int = 4, mix_M: float = 0.0) -> np.ndarray:
    """Float coefficients; with mix_M > 0 the adaptive blend (1+M) L_n - M L_(n-1)
    of Sec. Overview of RMG (M fixed, not fitted)."""
    a = np.array([float(v) for v in fd_coefficients(n_half)])
    if mix_M:
        b = np.array([float(v) for v in fd_coefficients(n_half - 1)] + [0.0])
        a = (1.0 + mix_M) * a - mix_M * b
    return a


def laplacian(f: np.ndarray, h: float, coeffs: np.ndarray) -> np.ndarray:
    """Periodic FD Laplacian of f[..., nz, ny, nx]: along each axis
    a_0 f_i + sum_k a_k (f_(i+k) + f_(i-k)), divided by h^2 (wrap-around).
    Each axis is one periodic 1-D correlation with the symmetric weights."""
    w = np.concatenate([coeffs[:0:-1], coeffs])  # a_n..a_1, a_0, a_1..a_n
    out = np.zeros_like(f)
    for ax in (-1, -2, -3):
        out += correlate1d(f, w, axis=ax, mode="wrap")
    return out / (h * h)


def fd_dispersion(kvec, h: float, coeffs: np.ndarray) -> float:
    """Eigenvalue of the periodic FD Laplacian on exp(i k.r): the closed form
    h^-2 sum_axes [a_0 + 2 sum_k a_k cos(k k_q h)]."""
    lam = 0.0
    for kq in kvec:
        lam += coeffs[0] + 2.0 * sum(coeffs[k] * np.cos(k * kq * h) for k in range(1, len(coeffs)))
    return lam / (h * h)


def axis_coords(n: int, h: float) -> np.ndarray:
    """Grid point positions i h along one axis."""
    return np.arange(n) * h


def dipole_coordinate(sys, axis: int) -> np.ndarray:
    """Sawtooth position operator on the periodic cell (Sec. Algorithm: the
    field is a sawtooth-like potential whose jump lies in the vacuum).

    Along the axis the coordinate rises by h per grid plane and drops by n h
    once, between planes j0 - 1 and j0 (j0 = sys.saw_jump[axis], 0 = the cell
    faces), centred so that it sums to zero over the cell:
    q_i = (((i - j0) mod n) - (n-1)/2) h.  Returned on the [nz, ny, nx] grid."""
    nx, ny, nz = sys.n
    h = sys.h
    n_ax = sys.n[axis]
    j0 = int(getattr(sys, "saw_jump", (0, 0, 0))[axis])
    q = (((np.arange(n_ax) - j0) % n_ax) - 0.5 * (n_ax - 1)) * h
    shape = [1, 1, 1]
    shape[2 - axis] = n_ax
    return np.broadcast_to(q.reshape(shape), (nz, ny, nx)).copy()


def inner(f: np.ndarray, g: np.ndarray, h: float) -> float:
    """Grid quadrature <f, g> = h^3 sum f g (Sec. Overview of RMG, expectation
    value; weight h^3 per point in three dimensions)."""
    return float(np.sum(f * g)) * h ** 3
