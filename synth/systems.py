"""Synthetic molecules and run parameters.

Workload shapes follow the paper's finite-system runs: a uniform periodic grid
with spacing 0.3-0.35 bohr (Sec. Numerical Results: benzene and C60 grids,
chlorophyll h = 0.3, Ag nanorods h = 1/3), an occupied-plus-virtual active space
(Algorithm 1, active-space selection) and delta kicks along x, y, z (Sec.
Numerical Results, kick perturbation).  Atoms are Gaussian local wells with
optional rank-4 separable projectors standing in for norm-conserving
pseudopotentials, which the paper uses but does not print.

Draw order for one molecule from ``numpy.random.default_rng(seed)`` (PCG64):
positions (rejection sampled), depths, widths, then projector strengths.
"""

from __future__ import annotations

import dataclasses
import hashlib
import json
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class System:
    """One synthetic molecule on a periodic grid.

    Grid point (i, j, k) sits at (i h, j h, k h) in a cell of side n h; arrays
    on the grid are stored C-order as [nz][ny][nx] (x fastest).
    """

    n: tuple  # (nx, ny, nz)
    h: float
    pos: np.ndarray  # (n_atoms, 3) bohr, in the frame of the grid points
    depth: np.ndarray  # (n_atoms,) Ha, well depth D_a
    width: np.ndarray  # (n_atoms,) bohr, Gaussian width w_a
    n_occ: int
    n_virt: int
    nl_rank: int = 0  # 0 (no nonlocal part) or 4 (s + three p-like projectors)
    nl_rcut: float = 2.0
    nl_sigma: float = 0.6
    nl_D: Optional[np.ndarray] = None  # (n_atoms, nl_rank) Ha
    n_images: int = 2  # periodic images summed per axis for the local wells
    seed: int = 0
    # sawtooth jump plane per axis (grid index of the first plane after the jump; 0 = cell faces)
    saw_jump: tuple = (0, 0, 0)
    # bit q set: vacuum dipole correction along axis q
    dipole_correction: int = 0
    # ion point charges for the dipole correction (None: electrons shared equally)
    ion_charge: Optional[np.ndarray] = None

    @property
    def n_orb(self) -> int:
        return self.n_occ + self.n_virt

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def ng(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def cell(self) -> np.ndarray:
        return np.array([self.n[0] * self.h, self.n[1] * self.h, self.n[2] * self.h])

    def occupations(self) -> np.ndarray:
        """Closed shell: two electrons per occupied orbital, none per virtual."""
        f = np.zeros(self.n_orb)
        f[: self.n_occ] = 2.0
        return f

    def to_json(self) -> str:
        d = {
            "n": list(self.n),
            "h": float(self.h).hex(),
            "pos": [[float(v).hex() for v in p] for p in self.pos],
            "depth": [float(v).hex() for v in self.depth],
            "width": [float(v).hex() for v in self.width],
            "n_occ": self.n_occ,
            "n_virt": self.n_virt,
            "nl_rank": self.nl_rank,
            "nl_rcut": float(self.nl_rcut).hex(),
            "nl_sigma": float(self.nl_sigma).hex(),
            "nl_D": None if self.nl_D is None else [[float(v).hex() for v in r] for r in self.nl_D],
            "n_images": self.n_images,
            "seed": self.seed,
        }
        if tuple(self.saw_jump) != (0, 0, 0):
            d["saw_jump"] = [int(v) for v in self.saw_jump]
        if self.dipole_correction:
            d["dipole_correction"] = int(self.dipole_correction)
        if self.ion_charge is not None:
            d["ion_charge"] = [float(v).hex() for v in self.ion_charge]
        return json.dumps(d, sort_keys=True)

    def digest(self) -> str:
        return hashlib.sha256(self.to_json().encode()).hexdigest()[:16]


@dataclasses.dataclass
class RunParams:
    """Time-loop parameters (Algorithm 1, parameter block)."""

    dt: float = 0.05
    n_steps: int = 200
    kappa: float = 1e-3  # delta-kick strength (a.u. of field x time)
    axis: int = 0  # 0 = x, 1 = y, 2 = z
    h_thrs: float = 1e-12  # Hamiltonian self-consistency threshold
    dp_thrs: float = 1e-15  # commutator-series threshold
    max_scf: int = 50
    max_terms: int = 200


def _positions(rng, n_atoms, lo, hi, min_dist):
    pos = np.zeros((0, 3))
    tries = 0
    while pos.shape[0] < n_atoms:
        p = lo + (hi - lo) * rng.random(3)
        tries += 1
        if tries > 100000:
            raise RuntimeError("cannot place atoms with the requested spacing")
        if pos.shape[0] and np.min(np.linalg.norm(pos - p, axis=1)) < min_dist:
            continue
        pos = np.vstack([pos, p])
    return pos


def make_system(n, h, n_atoms, n_occ, n_virt, seed, region=(0.25, 0.75), nl_rank=0,
                nl_rcut=2.0, nl_sigma=0.6, min_dist=2.0, depth_range=(1.0, 3.0),
                width_range=(0.8, 1.5), d_range=(0.5, 2.0)) -> System:
    """Gaussian-well molecule: positions uniform in region*L per axis with pair
    distance >= min_dist, depths U[depth_range] Ha, widths U[width_range] bohr,
    projector strengths U[d_range] Ha."""
    if isinstance(n, int):
        n = (n, n, n)
    rng = np.random.default_rng(seed)
    cell = np.array(n, dtype=float) * h
    pos = _positions(rng, n_atoms, region[0] * cell, region[1] * cell, min_dist)
    depth = rng.uniform(depth_range[0], depth_range[1], n_atoms)
    width = rng.uniform(width_range[0], width_range[1], n_atoms)
    nl_D = rng.uniform(d_range[0], d_range[1], (n_atoms, nl_rank)) if nl_rank else None
    return System(n=tuple(int(v) for v in n), h=float(h), pos=pos, depth=depth, width=width,
                  n_occ=n_occ, n_virt=n_virt, nl_rank=nl_rank, nl_rcut=nl_rcut,
                  nl_sigma=nl_sigma, nl_D=nl_D, seed=seed)


def make_fcc_cluster(n, h, n_sites, a_lat, n_occ, n_virt, seed, jitter=0.1) -> System:
    """The n_sites fcc lattice sites (constant a_lat) nearest the cell centre,
    each displaced by N(0, jitter) bohr; local wells only."""
    if isinstance(n, int):
        n = (n, n, n)
    rng = np.random.default_rng(seed)
    cell = np.array(n, dtype=float) * h
    centre = 0.5 * cell
    m = int(np.ceil(3 * (n_sites ** (1 / 3)))) + 2
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    idx = np.arange(-m, m + 1)
    g = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1).reshape(-1, 3)
    sites = (g[:, None, :] + base[None]).reshape(-1, 3) * a_lat
    r = np.linalg.norm(sites, axis=1)
    order = np.lexsort((sites[:, 2], sites[:, 1], sites[:, 0], np.round(r, 9)))
    sites = sites[order[:n_sites]]
    pos = centre + sites + rng.normal(0.0, jitter, sites.shape)
    depth = rng.uniform(1.0, 3.0, n_sites)
    width = rng.uniform(0.8, 1.5, n_sites)
    return System(n=tuple(int(v) for v in n), h=float(h), pos=pos, depth=depth, width=width,
                  n_occ=n_occ, n_virt=n_virt, nl_rank=0, seed=seed, n_images=1)


def make_molecule(seed, n_choices=(32, 36, 40, 48, 54, 60, 64), h=0.35):
    """One small molecule of the ragged batch: grid edge from n_choices,
    N ~ U{8..64} even with half occupied, atoms ~ U{2..20}."""
    rng = np.random.default_rng(seed)
    n = int(rng.choice(n_choices))
    n_orb = 2 * int(rng.integers(4, 33))
    n_atoms = int(rng.integers(2, 21))
    return n, n_orb, n_atoms


# Five workloads: a small parity case, a plain-vs-mixed case, a ragged batch,
# the learned-predictor case and a large nanoparticle-shaped case.
CONFIGS = {
    # seed 3: the first seed >= 1 whose self-consistent ground state has an
    # occupied gap > 1e-3 Ha and an active-space edge gap > 1e-6 Ha (seeds 1
    # and 2 have a degenerate highest occupied level).
    "c1_parity_32": dict(n=32, h=0.35, n_atoms=4, n_occ=8, n_virt=8, seed=3,
                         region=(0.25, 0.75), nl_rank=0, dt=0.05, n_steps=200),
    # seed 14: the first seed >= 2 whose self-consistent ground state (GPU solver,
    # start block of N + 30 smooth random vectors of the same seed) converges with a
    # HOMO-LUMO gap > 1e-3 Ha (1.03e-3; active-space edge gap 1.1e-3 Ha); the
    # density loops of seeds 2-13 end with gaps of 2e-5 - 8.8e-4 Ha.
    "c2_mixed_96": dict(n=96, h=0.3, n_atoms=40, n_occ=160, n_virt=80, seed=14,
                        region=(0.2, 0.8), nl_rank=4, dt=0.05, n_steps=2000,
                        gs=dict(n_guard=30, degree=24, max_scf=150, max_passes=20, tol_rho=1e-10, tol_res=1e-9,
                                mix=0.15)),
    "c5_cluster_192": dict(n=192, h=0.3, n_atoms=600, n_occ=2400, n_virt=600, seed=5,
                           dt=0.05, n_steps=500),
}


def config_system(name: str) -> System:
    c = CONFIGS[name]
    if name.startswith("c5"):
        return make_fcc_cluster(c["n"], c["h"], c["n_atoms"], 7.58, c["n_occ"], c["n_virt"], c["seed"])
    return make_system(c["n"], c["h"], c["n_atoms"], c["n_occ"], c["n_virt"], c["seed"],
                       region=c["region"], nl_rank=c["nl_rank"])


def config_run(name: str, **over) -> RunParams:
    c = CONFIGS[name]
    rp = RunParams(dt=c["dt"], n_steps=c["n_steps"])
    for k, v in over.items():
        setattr(rp, k, v)
    return rp


def ground_state_start(name: str) -> np.ndarray:
    """Start block of the GPU ground-state solve of a configuration: N + n_guard
    smooth random vectors of the configuration's seed."""
    s = config_system(name)
    return lowpass_orbitals(s.n, s.h, s.n_orb + CONFIGS[name]["gs"]["n_guard"], seed=s.seed)


def batch_systems(n_mol=16, seed0=300, h=0.35) -> List[System]:
    """The ragged batch: 16 molecules of uneven grid and active-space size;
    the smallest and largest grid edges appear at least once."""
    out = []
    for i in range(n_mol):
        s = seed0 + i
        n, n_orb, n_atoms = make_molecule(s, h=h)
        if i == 0:
            n = 32
        if i == 1:
            n = 64
        out.append(make_system(n, h, n_atoms, n_orb // 2, n_orb // 2, s, region=(0.25, 0.75)))
    return out


def lowpass_orbitals(n, h, n_orb, seed, g_cut=1.5, dtype=np.float64) -> np.ndarray:
    """Smooth random functions for throughput runs: white noise filtered by
    exp(-|G|^2 / (2 g_cut^2)) in Fourier space.  Not orthonormal; the library's
    reorthonormalisation step makes them an orthonormal active space."""
    if isinstance(n, int):
        n = (n, n, n)
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    gx = 2 * np.pi * np.fft.fftfreq(nx, d=h)
    gy = 2 * np.pi * np.fft.fftfreq(ny, d=h)
    gz = 2 * np.pi * np.fft.fftfreq(nz, d=h)
    g2 = gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2
    filt = np.exp(-g2 / (2 * g_cut ** 2))
    out = np.empty((n_orb, nz, ny, nx), dtype=dtype)
    for i in range(n_orb):
        w = rng.standard_normal((nz, ny, nx))
        f = np.fft.ifftn(np.fft.fftn(w) * filt).real
        f /= np.sqrt(np.sum(f * f) * h ** 3)
        out[i] = f
    return out


def basis_mixing(n: int, seed: int, strength: float = 0.3, lower: bool = False) -> np.ndarray:
    """Random well-conditioned N x N matrix A = I + strength * G / sqrt(N), G standard
    normal (strictly lower triangular when lower=True, so A is unit lower
    triangular).  A non-orthogonal basis for tests is Phi = A Psi."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    if lower:
        G = np.tril(G, -1)
    return np.eye(n) + strength * G / np.sqrt(n)
