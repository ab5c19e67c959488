"""Initialisation by orbital blocks (rt_run.h_block): the FP64 grid Hamiltonian
is applied hb orbitals at a time, so that the buffer beside Psi holds hb
orbitals (what lets a 192^3 x 3000-orbital system fit one device).  Through the
C ABI, against the same context built with every orbital at once: H_core and
H_gs within FP64 rounding and exactly symmetric, trajectories (FP64 and mixed
precision, both with the local update) within the FP64 parity bound."""

import numpy as np
import pytest

import synth
from rt_helpers import run_args, system_args

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _system():
    s = synth.make_system((36, 40, 32), 0.3, 6, 10, 10, seed=12, nl_rank=4, region=(0.3, 0.7))
    psi = synth.lowpass_orbitals(s.n, 0.3, 20, 12)
    # orthonormal in the grid inner product (h_block excludes the library's own step)
    q, _ = np.linalg.qr(psi.reshape(20, -1).T)
    return s, np.ascontiguousarray((q.T / np.sqrt(s.h ** 3)).reshape(psi.shape))


@pytest.mark.parametrize("precision", [0, 1])
def test_blocked_initialisation_matches_all_at_once(precision):
    _say(f"h_block 0 vs 3 (20 orbitals: blocks 3,...,3,2), precision={precision}, 36x40x32, 40 steps x/y/z")
    from paper_2410_09189_amd import rt

    s, psi = _system()
    N = 20
    rp = synth.RunParams(dt=0.05, n_steps=40, kappa=1e-3, h_thrs=1e-10 if precision == 0 else 1e-9)
    out = []
    for hb in (0, 3):
        ses = rt.Session([system_args(s, psi)], run_args(rp, n_traj_axes=(0, 1, 2), precision=precision,
                                                         hupdate=rt.RT_HUPDATE_LOCAL, h_block=hb))
        mats = {k: rt.rt_get_matrix(ses.ctx, 0, k, N) for k in (4, 8)}  # H_core, H_gs
        rt.rt_step(ses.ctx, 40, n_traj=3)
        mus = np.stack([rt.rt_dipole(ses.ctx, t, 0, 41)[0][:, t] for t in range(3)])
        es = np.stack([rt.rt_dipole(ses.ctx, t, 0, 41)[1] for t in range(3)])
        out.append((mats, mus, es))
        ses.close()
    (m0, mu0, e0), (m1, mu1, e1) = out
    for k in (4, 8):
        scale = np.max(np.abs(m0[k]))
        err = np.max(np.abs(m1[k] - m0[k]))
        print(f"matrix {k}: max diff {err:.3e} of {scale:.3e}", flush=True)
        assert err < 1e-12 * scale
        assert np.array_equal(m1[k], m1[k].T)
    d0 = mu0 - mu0[:, :1]
    err = np.max(np.abs(mu1 - mu0))
    print(f"dipole: max diff {err:.3e} of max|dmu| {np.max(np.abs(d0)):.3e}", flush=True)
    assert np.max(np.abs(d0)) > 1e-5
    assert err < 1e-10
    assert np.max(np.abs(e1 - e0)) < 1e-10
