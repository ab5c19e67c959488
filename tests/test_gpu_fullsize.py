"""Parity at the benchmark's full size and launch configuration: the 96^3 molecule
with 40 wells and rank-4 projectors, 160 + 80 orbitals, the x/y/z kicks stepped
together as three trajectories (dt 0.05, H_thrs 1e-7, dP_thrs 1e-10, graph
capture on), after two time steps.  The oracle cannot run this trajectory in
seconds, so it checks what it can compute directly at this size:

* the dipole matrices M_q = h^3 Psi diag(q) Psi^T (full);
* sampled columns of the ground-state Hamiltonian H_gs (H applied by the
  oracle to those orbitals);
* for every trajectory, the Hamiltonian the step holds for its density matrix,
  through the identity H[P] - H_gs = h^3 Psi diag(V_Hx[rho(P)] - V_Hx[rho_gs]) Psi^T
  (full; in mixed precision within the error model of the perturbation);
* the density of trajectory 0, the dipole Tr(P M_q), and the invariants of P
  (Hermiticity, trace 2 N_occ, idempotency P^2 = 2P) that the unitary step keeps.
"""

import functools

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle.grid import dipole_coordinate, fd_coefficients_float, laplacian
from oracle.hamiltonian import density, hartree, lda_x
from oracle.system import apply_vnl, projectors, v_ion
from rt_helpers import system_args

pytestmark = pytest.mark.gpu

MIXED_REL = 1e-4  # error model of the BF16x3 perturbation products (test_gpu_parity)
NAME = "c2_mixed_96"
AXES = (0, 1, 2)


def _say(msg):
    print(f"[case] {msg}", flush=True)


@functools.lru_cache(maxsize=None)
def _inputs():
    s = synth.config_system(NAME)
    psi = synth.lowpass_orbitals(s.n, s.h, s.n_orb, seed=s.seed)
    return s, psi


@functools.lru_cache(maxsize=None)
def _oracle_static():
    """Orthonormal orbitals (the basis transform the library applies at init),
    dipole matrices and the ground-state Hartree-exchange potential."""
    s, psi = _inputs()
    N = s.n_orb
    P = psi.reshape(N, -1)
    L = np.linalg.cholesky(s.h ** 3 * P @ P.T)
    X = scipy.linalg.solve_triangular(L, P, lower=True)
    M = []
    for q in range(3):
        a = s.h ** 3 * (X * dipole_coordinate(s, q).ravel()[None, :]) @ X.T
        M.append(0.5 * (a + a.T))
    rho_gs = density(np.diag(s.occupations()), X)
    vhx_gs = hartree(rho_gs, s) + lda_x(rho_gs)[0]
    return X, np.stack(M), rho_gs, vhx_gs


def _delta_h(s, X, Sre, vhx_gs):
    rho = density(Sre, X)
    dv = hartree(rho, s) + lda_x(rho)[0] - vhx_gs
    a = s.h ** 3 * (X * dv[None, :]) @ X.T
    return 0.5 * (a + a.T), rho


@functools.lru_cache(maxsize=None)
def _gpu_run(precision):
    import torch

    from paper_2410_09189_amd import rt

    assert torch.cuda.is_available(), "GPU test without a GPU"
    s, psi = _inputs()
    hup = rt.RT_HUPDATE_LOCAL if precision == rt.RT_MIXED else rt.RT_HUPDATE_FULL
    ra = rt.RunArgs(dt=0.05, n_steps_max=2, h_thrs=1e-7, dp_thrs=1e-10, max_scf=50, max_terms=200,
                    traj_sys=[0] * 3, traj_kappa=[1e-3] * 3, traj_axis=list(AXES), hupdate=hup,
                    precision=precision)
    ses = rt.Session([system_args(s, psi, orthonormalize=True)], ra)
    stats = rt.rt_step(ses.ctx, 2, n_traj=3, stats=True)
    N = s.n_orb
    out = dict(stats=stats, M=np.stack([rt.rt_get_matrix(ses.ctx, 0, 5 + q, N) for q in range(3)]),
               Hgs=rt.rt_get_matrix(ses.ctx, 0, 8, N), rho0=rt.rt_get_grid(ses.ctx, 0, 0, s.ng))
    for t in range(3):
        out[t] = dict(S=rt.rt_get_matrix(ses.ctx, t, 2, N), A=rt.rt_get_matrix(ses.ctx, t, 3, N),
                      H0=rt.rt_get_matrix(ses.ctx, t, 0, N), mu=rt.rt_dipole(ses.ctx, t, 0, 3)[0])
    ses.close()
    return out


@pytest.mark.parametrize("mode", ["mixed", "fp64"])
def test_full_size_step_matches_oracle(mode):
    from paper_2410_09189_amd import rt

    _say(f"96^3 N=240 three kicks, two steps, {mode}")
    s, _ = _inputs()
    N, ng = s.n_orb, s.ng
    g = _gpu_run(rt.RT_MIXED if mode == "mixed" else rt.RT_FP64)
    print("step stats (updates, terms, residual):", g["stats"], flush=True)
    X, M, rho_gs, vhx_gs = _oracle_static()
    # dipole matrices (FP64 projection at init)
    assert np.max(np.abs(g["M"] - M)) < 1e-11 * np.max(np.abs(M))
    # sampled columns of H_gs: the oracle applies H to those orbitals
    Hgs = g["Hgs"]
    vloc = v_ion(s).ravel() + vhx_gs
    projs = projectors(s)
    coeffs = fd_coefficients_float(4)
    nx, ny, nz = s.n
    for j in (0, 101, 159, 160, 239):
        hx = (-0.5 * laplacian(X[j].reshape(nz, ny, nx), s.h, coeffs)).ravel() + vloc * X[j]
        hx = hx + apply_vnl(X[j:j + 1], projs, s.h)[0]
        col = s.h ** 3 * X @ hx
        assert np.max(np.abs(Hgs[:, j] - col)) < 1e-11 * np.max(np.abs(Hgs)), j
    for t in range(1 if mode == "fp64" else 3):
        tr = g[t]
        Sre, Aim = tr["S"], tr["A"]
        P = Sre + 1j * Aim
        # invariants the unitary propagation keeps
        assert np.max(np.abs(Sre - Sre.T)) < 1e-12 and np.max(np.abs(Aim + Aim.T)) < 1e-12
        assert abs(np.trace(Sre) - 2 * s.n_occ) < 1e-9
        assert np.max(np.abs(P @ P - 2 * P)) < 1e-8
        # dipole = Tr(P M_q)
        mu_ref = np.array([np.trace(Sre @ M[q]) for q in range(3)])
        assert np.max(np.abs(tr["mu"][2] - mu_ref)) < 1e-11 * np.max(np.abs(mu_ref)), t
        # the Hamiltonian held for P: H[P] - H_gs from the oracle's potentials
        dH, rho = _delta_h(s, X, Sre, vhx_gs)
        got = tr["H0"] - Hgs
        err = np.max(np.abs(got - dH))
        scale = np.max(np.abs(dH))
        print(f"traj {t}: max|dH| {scale:.3e}  max err {err:.3e}", flush=True)
        if mode == "mixed":
            assert err < MIXED_REL * scale + 1e-12 * np.max(np.abs(Hgs))
        else:
            assert err < 1e-9 * scale + 1e-11 * np.max(np.abs(Hgs))
        if t == 0:
            drho = np.max(np.abs(rho - rho_gs))
            rerr = np.max(np.abs(g["rho0"] - rho))
            print(f"traj 0: max|rho - rho_gs| {drho:.3e}  max rho err {rerr:.3e}", flush=True)
            assert rerr < (MIXED_REL if mode == "mixed" else 1e-9) * drho + 1e-13 * np.max(rho_gs)
    assert g["stats"][0][0] >= 1 and all(st[0] <= 50 for st in g["stats"])
    assert ng == 96 ** 3 and N == 240


def test_nanoparticle_shape_fp32_apply_sampled_against_oracle():
    """The 192^3 x 3000-orbital FP32 apply the benchmark times (85 GB in, 85 GB out,
    the chunking over the context's 64-orbital block included): three sampled
    orbitals against the oracle's FD8 stencil + V_loc in FP64, and the two-strip
    tiling against the built-in one bit for bit."""
    import torch

    from paper_2410_09189_amd import rt

    _say("192^3 x 3000 orbitals FP32 apply, sampled")
    s = synth.config_system("c5_cluster_192")
    ng = s.ng
    gen = torch.Generator(device="cuda")
    gen.manual_seed(s.seed)
    psi0 = torch.randn((64, ng), dtype=torch.float64, device="cuda", generator=gen)
    sa = rt.SystemArgs(n=s.n, h=s.h, pos=s.pos, depth=s.depth, width=s.width, n_occ=32, n_virt=32, psi0=psi0,
                       n_images=s.n_images, orthonormalize=True)
    ra = rt.RunArgs(dt=0.05, n_steps_max=1, h_thrs=1e-7, dp_thrs=1e-10, max_scf=50, max_terms=200, traj_sys=[],
                    traj_kappa=[], traj_axis=[], hupdate=rt.RT_HUPDATE_LOCAL)
    ses = rt.Session([sa], ra)
    del psi0
    n_orb = 3000
    x = torch.randn((n_orb, ng), dtype=torch.float32, device="cuda", generator=gen)
    y = torch.empty_like(x)
    rt.rt_apply_h(ses.ctx, 0, x.data_ptr(), y.data_ptr(), n_orb, 1)
    torch.cuda.synchronize()
    vloc = rt.rt_get_grid(ses.ctx, 0, 4, ng)
    # the tiling the autotuner takes at this shape (16-row tiles, two strips a
    # thread) gives the built-in tiling's result bit for bit (first 200 orbitals)
    rt.rt_tune_set(ses.ctx, 0, rt.RT_TUNE_STENCIL_FP32, 16, 1, 3)
    y2 = torch.empty((200, ng), dtype=torch.float32, device="cuda")
    rt.rt_apply_h(ses.ctx, 0, x.data_ptr(), y2.data_ptr(), 200, 1)
    torch.cuda.synchronize()
    assert torch.equal(y2, y[:200])
    del y2
    ses.close()
    coeffs = fd_coefficients_float(4)
    nx, ny, nz = s.n
    for j in (0, 1777, 2999):
        xj = x[j].double().cpu().numpy()
        ref = (-0.5 * laplacian(xj.reshape(nz, ny, nx), s.h, coeffs)).ravel() + vloc * xj
        got = y[j].double().cpu().numpy()
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"orbital {j}: rel err {err:.2e}", flush=True)
        assert err < 1e-5
