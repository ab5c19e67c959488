"""Sawtooth jump planes and the vacuum dipole correction (Sec. Algorithm,
time-dependent field; Bengtsson's correction) on the HIP path, through the C
ABI, against the FP64 oracle on the same seeded inputs.  Tolerances as in the
other parity tests: FP64 stages within 1e-11 relative, FP64 trajectories within
1e-10 a.u., mixed trajectories within 1e-5 of the dipole change."""

import dataclasses
import functools

import numpy as np
import pytest

import oracle
import synth
from conftest import c1_ground_state, c1_system
from oracle import hamiltonian
from oracle.ground_state import ground_state as oracle_ground_state
from rt_helpers import orthonormalize_np, run_args, system_args

pytestmark = pytest.mark.gpu

# jump planes in the vacuum of each cell (molecules occupy the middle 40-50 %)
RAGGED_JUMP = (3, 37, 30)  # 36 x 40 x 32
C1_JUMP = (4, 28, 3)  # 32^3
STEPS = 100


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _rt():
    import torch

    from paper_2410_09189_amd import rt

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return rt


def _ragged_dc(mask=7, seed=10):
    s = synth.make_system((36, 40, 32), 0.3, 6, 10, 10, seed=seed, nl_rank=4, region=(0.3, 0.7))
    psi = synth.lowpass_orbitals(s.n, 0.3, 20, seed)
    return dataclasses.replace(s, saw_jump=RAGGED_JUMP, dipole_correction=mask), psi


def test_dipole_matrices_and_ground_hamiltonian_with_jump_planes():
    _say("M_q and H_gs with jump planes (3, 37, 30) and the correction on all axes, 36x40x32 N=20")
    rt = _rt()
    s, psi = _ragged_dc()
    rp = synth.RunParams(dt=0.05, n_steps=2)
    ses = rt.Session([system_args(s, psi, orthonormalize=True)], run_args(rp))
    m = oracle.Model(s, orthonormalize_np(s, psi))
    N = m.N
    for q in range(3):
        Mq = rt.rt_get_matrix(ses.ctx, 0, 5 + q, N)
        assert np.max(np.abs(Mq - m.M[q])) < 1e-11 * np.max(np.abs(m.M[q]))
    Hgs = rt.rt_get_matrix(ses.ctx, 0, 8, N)
    P0 = np.diag(s.occupations()).astype(complex)
    ref, _ = m.h_of_p(P0)
    assert np.max(np.abs(Hgs - ref)) < 1e-11 * np.max(np.abs(ref))
    # the correction is far above the tolerance here
    m0 = oracle.Model(dataclasses.replace(s, dipole_correction=0), m.psi)
    assert np.max(np.abs(ref - m0.h_of_p(P0)[0])) > 1e-6 * np.max(np.abs(ref))
    ses.close()


@pytest.mark.parametrize("hupdate", [0, 1])
def test_eval_h_with_dipole_correction_matches_oracle(hupdate):
    _say(f"eval_h with the dipole correction hupdate={hupdate} 36x40x32 N=20")
    rt = _rt()
    import torch

    s, psi = _ragged_dc(seed=11)
    rp = synth.RunParams(dt=0.05, n_steps=2)
    ses = rt.Session([system_args(s, psi, orthonormalize=True)], run_args(rp, hupdate=hupdate))
    m = oracle.Model(s, orthonormalize_np(s, psi))
    N = m.N
    rng = np.random.default_rng(4)
    A = rng.standard_normal((N, N))
    S = np.diag(s.occupations()) + 0.1 * (A + A.T)
    Sd = torch.from_numpy(S).cuda()
    Hd = torch.empty_like(Sd)
    rt.rt_eval_h(ses.ctx, 0, Sd.data_ptr(), Hd.data_ptr())
    torch.cuda.synchronize()
    ref, aux = m.h_of_p(S.astype(complex))
    got = Hd.cpu().numpy()
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))
    rho = rt.rt_get_grid(ses.ctx, 0, 0, s.ng)
    assert np.max(np.abs(rho - aux["rho"])) < 1e-12 * np.max(np.abs(aux["rho"]))
    # V_H alone, and V_loc = V_ion + V_H + v_dc + v_x
    vh = rt.rt_get_grid(ses.ctx, 0, 1, s.ng)
    vh_ref = hamiltonian.hartree(aux["rho"], s)
    assert np.max(np.abs(vh - vh_ref)) < 1e-12 * np.max(np.abs(vh_ref))
    vloc = rt.rt_get_grid(ses.ctx, 0, 4, s.ng)
    vloc_ref = m.vion + aux["vh"] + aux["vx"]
    assert np.max(np.abs(vloc - vloc_ref)) < 1e-12 * np.max(np.abs(vloc_ref))
    ses.close()


@functools.lru_cache(maxsize=None)
def _nonpolar_charges():
    """Ion charges of the C1 molecule (sum = 16 electrons) whose dipole about the
    sawtooth equals that of the oracle's ground-state electrons, so that the
    corrected Hamiltonian keeps that ground state stationary and only the
    response to the kick feels the correction (least change from equal shares)."""
    s = dataclasses.replace(c1_system(), saw_jump=C1_JUMP, dipole_correction=7)
    psi, _ = c1_ground_state()
    m = oracle.Model(s, psi)
    rho = hamiltonian.density(np.diag(s.occupations()), m.psi)
    d_el = [s.h ** 3 * float(np.sum(rho * m.qs[q])) for q in range(3)]
    A = np.vstack([np.ones(s.n_atoms)] + [hamiltonian.sawtooth_at(s.pos[:, q], s, q) for q in range(3)])
    b = np.array([float(np.sum(s.occupations()))] + d_el)
    z0 = np.full(s.n_atoms, b[0] / s.n_atoms)
    return tuple(z0 + np.linalg.lstsq(A, b - A @ z0, rcond=None)[0])


def _c1_dc_system(mask, charges):
    z = None if charges == "equal" else np.array(_nonpolar_charges())
    return dataclasses.replace(c1_system(), saw_jump=C1_JUMP, dipole_correction=mask, ion_charge=z)


@functools.lru_cache(maxsize=None)
def _c1_dc_oracle(mask, charges):
    psi, _ = c1_ground_state()
    rp = synth.config_run("c1_parity_32", n_steps=STEPS)
    return oracle.run(oracle.Model(_c1_dc_system(mask, charges), psi), rp)


# "nonpolar": stationary start, the correction acts on the response (its depolarising
# field changes the dipole by about half here); "equal": the ground state without the
# correction meets a strong static correction field (FP64 only: the mixed path resolves
# changes relative to the ground-state density, and this start is far from it)
@pytest.mark.parametrize("precision,hupdate,charges", [(0, 0, "nonpolar"), (0, 1, "nonpolar"),
                                                       (1, 1, "nonpolar"), (0, 0, "equal")])
def test_c1_kick_with_dipole_correction_matches_oracle(precision, hupdate, charges):
    _say(f"C1 32^3 {STEPS} steps, jumps {C1_JUMP}, correction on x,y,z, {charges} ion charges, "
         f"precision={precision} hupdate={hupdate}")
    rt = _rt()
    ref = _c1_dc_oracle(7, charges)
    s = _c1_dc_system(7, charges)
    psi, _ = c1_ground_state()
    rp = synth.config_run("c1_parity_32", n_steps=STEPS, h_thrs=1e-9 if precision else 1e-12)
    ses = rt.Session([system_args(s, psi)], run_args(rp, hupdate=hupdate, precision=precision))
    rt.rt_step(ses.ctx, STEPS, n_traj=1)
    mu, E, tr = rt.rt_dipole(ses.ctx, 0, 0, STEPS + 1)
    ses.close()
    dref = ref["mu"] - ref["mu"][0]
    scale = np.max(np.abs(dref))
    err = np.max(np.abs((mu - mu[0]) - dref))
    print(f"max|dmu| {scale:.3e}  err {err:.3e}  E err {np.max(np.abs(E - ref['E'])):.3e}", flush=True)
    assert scale > 1e-5
    if precision == 0:
        assert np.max(np.abs(mu - ref["mu"])) < 1e-10
        assert np.max(np.abs(E - ref["E"])) < 1e-10
    else:
        assert err < 1e-5 * scale
        # the energy changes by the kick only: its change agrees to the mixed path's resolution
        assert np.max(np.abs((E - E[0]) - (ref["E"] - ref["E"][0]))) < 1e-7
    assert np.max(np.abs(tr - 16.0)) < 1e-12


def test_c1_correction_changes_the_response():
    """Corrected and uncorrected oracle responses differ far beyond the parity
    tolerance, so the parity above checks the correction itself; the nonpolar
    charges keep the ground state stationary."""
    a = _c1_dc_oracle(7, "nonpolar")["mu"]
    b = _c1_dc_oracle(0, "nonpolar")["mu"]
    da, db = a - a[0], b - b[0]
    assert np.max(np.abs(da - db)) > 0.1 * np.max(np.abs(da))


def test_ground_state_with_dipole_correction_matches_oracle():
    _say("ground state 16^3 rank-4 projectors N=4, jumps (2, 14, 1), correction on x,y,z")
    rt = _rt()
    s = synth.make_system(16, 0.4, 2, 2, 2, seed=1, nl_rank=4, region=(0.3, 0.7))
    s = dataclasses.replace(s, saw_jump=(2, 14, 1), dipole_correction=7)
    ref = oracle_ground_state(s, tol_rho=1e-11, tol_res=1e-10)
    x0 = synth.lowpass_orbitals(s.n, s.h, s.n_orb + 6, seed=3)
    psi, eps, rho, st = rt.ground_state(system_args(s, x0), rt.gs_params(n_guard=6, degree=8))
    print("stats", st, "max |eps - eps_oracle|", np.max(np.abs(eps[:4] - ref["eps"][:4])), flush=True)
    assert np.max(np.abs(eps[:4] - ref["eps"][:4])) < 1e-9
    s0 = dataclasses.replace(s, dipole_correction=0)
    ref0 = oracle_ground_state(s0, tol_rho=1e-11, tol_res=1e-10)
    assert np.max(np.abs(ref0["eps"][:4] - ref["eps"][:4])) > 1e-7
    P = psi.cpu().numpy().reshape(4, -1)
    Q = ref["psi"].reshape(4, -1)
    O = s.h ** 3 * P @ Q.T
    assert np.min(np.abs(np.diag(O))) > 1 - 1e-9


def test_corrected_ground_state_is_stationary_under_propagation():
    """The GPU ground state with the correction, propagated without a kick: the
    time step's Hamiltonian carries the same correction, so nothing moves."""
    _say("C1 ground state with the correction (GPU), then 100 steps without a kick")
    rt = _rt()
    import torch

    s = dataclasses.replace(c1_system(), saw_jump=C1_JUMP, dipole_correction=7)
    x0 = synth.lowpass_orbitals(s.n, s.h, s.n_orb + 8, seed=21)
    psi, eps, rho, st = rt.ground_state(system_args(s, x0), rt.gs_params(n_guard=8, degree=10))
    print("stats", st, flush=True)
    assert st["residual"] <= 1e-10
    rp = synth.config_run("c1_parity_32", n_steps=STEPS)
    rp.kappa = 0.0
    ses = rt.Session([system_args(s, psi.cpu().numpy(), device_psi=psi)], run_args(rp))
    rt.rt_step(ses.ctx, STEPS, n_traj=1)
    mu, E, tr = rt.rt_dipole(ses.ctx, 0, 0, STEPS + 1)
    ses.close()
    torch.cuda.synchronize()
    print(f"no kick: max|mu - mu0| {np.max(np.abs(mu - mu[0])):.3e}  max|E - E0| {np.max(np.abs(E - E[0])):.3e}",
          flush=True)
    assert np.max(np.abs(mu - mu[0])) < 1e-8
    assert np.max(np.abs(E - E[0])) < 1e-10
