"""Helpers shared by the GPU tests: build binding arguments from a synthetic
system and run the library on cuda:0."""

import numpy as np

from paper_2410_09189_amd import rt


def system_args(s, psi, orthonormalize=False, device_psi=None, nonorthogonal=False):
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    return rt.SystemArgs(n=s.n, h=s.h, pos=s.pos, depth=s.depth, width=s.width, n_occ=s.n_occ,
                         n_virt=s.n_virt, psi0=psi if device_psi is None else device_psi,
                         nl_rank=s.nl_rank, nl_rcut=s.nl_rcut, nl_sigma=s.nl_sigma, nl_D=s.nl_D,
                         n_images=s.n_images, orthonormalize=orthonormalize, nonorthogonal=nonorthogonal,
                         saw_jump=tuple(getattr(s, "saw_jump", (0, 0, 0))),
                         dipole_correction=int(getattr(s, "dipole_correction", 0)),
                         ion_charge=getattr(s, "ion_charge", None))


def run_args(rp, n_traj_axes=(0,), sys_index=None, kappas=None, **kw):
    n = len(n_traj_axes)
    return rt.RunArgs(dt=rp.dt, n_steps_max=rp.n_steps, h_thrs=rp.h_thrs, dp_thrs=rp.dp_thrs,
                      max_scf=rp.max_scf, max_terms=rp.max_terms,
                      traj_sys=sys_index if sys_index is not None else [0] * n,
                      traj_kappa=kappas if kappas is not None else [rp.kappa] * n,
                      traj_axis=list(n_traj_axes), **kw)


def orthonormalize_np(s, psi):
    """Oracle-side reading of the basis transform: S = h^3 Psi Psi^T = L L^T, Psi <- L^-1 Psi."""
    import scipy.linalg

    P = psi.reshape(psi.shape[0], -1)
    S = s.h ** 3 * P @ P.T
    L = np.linalg.cholesky(S)
    return scipy.linalg.solve_triangular(L, P, lower=True).reshape(psi.shape)
