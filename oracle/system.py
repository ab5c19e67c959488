"""Electron-ion terms of the synthetic molecules (oracle; test infrastructure only).

The paper represents ions by norm-conserving pseudopotentials with local and
separable nonlocal parts (Sec. Overview of RMG, potential term V_eff; nonlocal
pseudopotentials).  The synthetic stand-in used throughout:

  local:    V_ion(r) = - sum_a sum_images D_a exp(-|r - R_a - nL|^2 / (2 w_a^2))
  nonlocal: V_nl = sum_a sum_p |beta_ap> D_ap <beta_ap| (h^3 quadrature in the
            bra), with beta_a1 ~ g(s), beta_a(2,3,4) ~ (s_q / sigma) g(s),
            g(s) = exp(-s^2 / (2 sigma^2)) (1 - s^2/r_c^2)^2 for s < r_c,
            each column normalised so that h^3 sum beta^2 = 1.
"""

import numpy as np


def grid_xyz(sys):
    """Coordinates (X, Y, Z) of the grid points, each shaped [nz, ny, nx]."""
    nx, ny, nz = sys.n
    h = sys.h
    z, y, x = np.meshgrid(np.arange(nz) * h, np.arange(ny) * h, np.arange(nx) * h, indexing="ij")
    return x, y, z


def v_ion(sys) -> np.ndarray:
    """Local ionic potential on the grid, periodic images -n_images..n_images per axis."""
    x, y, z = grid_xyz(sys)
    L = sys.cell
    v = np.zeros_like(x)
    r = range(-sys.n_images, sys.n_images + 1)
    for a in range(sys.n_atoms):
        R = sys.pos[a]
        inv = 1.0 / (2.0 * sys.width[a] ** 2)
        for i in r:
            dx2 = (x - R[0] - i * L[0]) ** 2
            for j in r:
                dy2 = (y - R[1] - j * L[1]) ** 2
                for k in r:
                    dz2 = (z - R[2] - k * L[2]) ** 2
                    v -= sys.depth[a] * np.exp(-(dx2 + dy2 + dz2) * inv)
    return v


def min_image(d: np.ndarray, L: float) -> np.ndarray:
    """Minimum-image displacement on a periodic axis of length L."""
    return d - L * np.round(d / L)


def radial_profile(s2: np.ndarray, sigma: float, rcut: float) -> np.ndarray:
    """Unnormalised radial factor g(s) = exp(-s^2 / (2 sigma^2)) (1 - s^2/r_c^2)^2
    of the projectors, given s^2 (valid for s < r_c; zero value and slope at r_c)."""
    return np.exp(-s2 / (2 * sigma ** 2)) * (1.0 - s2 / rcut ** 2) ** 2


def projectors(sys):
    """Per-atom projector tables: list of (flat grid indices, beta[n_sph, rank], D[rank]).

    The sphere is every grid point whose minimum-image distance to the atom is
    below r_c.  Points are listed in increasing flat index (z, y, x order)."""
    if sys.nl_rank == 0:
        return []
    x, y, z = grid_xyz(sys)
    L = sys.cell
    out = []
    for a in range(sys.n_atoms):
        d = [min_image(c - sys.pos[a][q], L[q]) for q, c in enumerate((x, y, z))]
        s2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
        mask = s2 < sys.nl_rcut ** 2
        idx = np.flatnonzero(mask.ravel())
        s2m = s2.ravel()[idx]
        g = radial_profile(s2m, sys.nl_sigma, sys.nl_rcut)
        cols = [g]
        for q in range(3):
            cols.append(d[q].ravel()[idx] / sys.nl_sigma * g)
        beta = np.stack(cols[: sys.nl_rank], axis=1)
        beta = beta / np.sqrt(np.sum(beta * beta, axis=0) * sys.h ** 3)
        out.append((idx, beta, np.array(sys.nl_D[a], dtype=np.float64)))
    return out


def apply_vnl(psi: np.ndarray, projs, h: float) -> np.ndarray:
    """V_nl applied to orbitals psi[N, Ng]: for every atom, c = h^3 beta^T psi_sphere,
    then add beta (D c) on the sphere."""
    out = np.zeros_like(psi)
    for idx, beta, D in projs:
        c = h ** 3 * (psi[:, idx] @ beta)  # [N, rank]
        out[:, idx] += (c * D[None, :]) @ beta.T
    return out
