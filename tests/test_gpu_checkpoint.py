"""Checkpoint and resume through the C ABI: 100 steps, a checkpoint, a fresh
context loaded from it and 100 more steps equal 200 steps in one context bit for
bit -- the dipole, energy and electron-count histories and the final density
matrix -- in FP64 with the paper's linear first guess, in mixed precision with
the quadratic guess (which reads H_-2) and with the learned guess (which reads the
feature rings and the fallback statistics).  Corrupted or mismatched checkpoints
are refused with nothing changed."""

import numpy as np
import pytest

import synth
from conftest import c1_ground_state, c1_system
from rt_helpers import run_args, system_args

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _args(mode):
    from paper_2410_09189_amd import predictor, rt

    s = c1_system()
    psi, _ = c1_ground_state()
    rp = synth.config_run("c1_parity_32", n_steps=200, h_thrs=1e-9, dp_thrs=1e-13)
    kw = {}
    if mode == "mixed_quadratic":
        kw = dict(precision=rt.RT_MIXED, hupdate=rt.RT_HUPDATE_LOCAL, predictor=rt.RT_PRED_QUADRATIC)
    elif mode == "fp64_learned":
        dims = rt.rt_mlp_dims()
        p = predictor.init_params(dims, seed=3)
        p[2 * dims[0] + dims[2]:2 * dims[0] + 2 * dims[2]] = 1e6  # outputs of ~1e-6 Ha
        kw = dict(predictor=rt.RT_PRED_MLP, mlp_params=p)
    return system_args(s, psi), run_args(rp, n_traj_axes=(0, 1), kappas=[1e-3, 2e-3], **kw)


def _observe(rt, ctx):
    out = []
    for t in range(2):
        mu, E, tr = rt.rt_dipole(ctx, t, 0, 201)
        out += [mu, E, tr] + [rt.rt_get_matrix(ctx, t, w, 16) for w in range(4)]  # H_0, H_-1, Re P, Im P
    return out


@pytest.mark.parametrize("mode", ["fp64_linear", "mixed_quadratic", "fp64_learned"])
def test_resume_from_checkpoint_equals_uninterrupted_run_bitwise(mode):
    _say(f"checkpoint 100 + 100 vs 200 steps, {mode}")
    from paper_2410_09189_amd import rt

    sa, ra = _args(mode)
    ses = rt.Session([sa], ra)
    rt.rt_step(ses.ctx, 200, n_traj=2)
    ref = _observe(rt, ses.ctx)
    ses.close()

    sa, ra = _args(mode)
    ses = rt.Session([sa], ra)
    rt.rt_step(ses.ctx, 100, n_traj=2)
    blob = rt.rt_checkpoint_save(ses.ctx)
    ses.close()

    sa, ra = _args(mode)
    ses = rt.Session([sa], ra)
    rt.rt_checkpoint_load(ses.ctx, blob)
    rt.rt_step(ses.ctx, 100, n_traj=2)
    got = _observe(rt, ses.ctx)
    ses.close()
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_bad_checkpoints_are_refused_and_change_nothing():
    _say("checkpoint validation")
    from paper_2410_09189_amd import rt

    sa, ra = _args("fp64_linear")
    ses = rt.Session([sa], ra)
    rt.rt_step(ses.ctx, 5, n_traj=2)
    blob = rt.rt_checkpoint_save(ses.ctx)
    before = rt.rt_checkpoint_save(ses.ctx)
    bad = [blob[:-8], np.concatenate([blob, np.zeros(8, np.uint8)]), blob.copy()]
    bad[2][0] ^= 0xFF  # magic
    for b in bad:
        with pytest.raises(rt.RTError) as e:
            rt.rt_checkpoint_load(ses.ctx, b)
        assert e.value.status == rt.RT_EINVAL
    assert np.array_equal(rt.rt_checkpoint_save(ses.ctx), before)
    ses.close()
    # a context of another shape (one trajectory) refuses it
    s = c1_system()
    psi, _ = c1_ground_state()
    ses = rt.Session([system_args(s, psi)], run_args(synth.config_run("c1_parity_32", n_steps=10)))
    with pytest.raises(rt.RTError) as e:
        rt.rt_checkpoint_load(ses.ctx, blob)
    assert e.value.status == rt.RT_EINVAL
    ses.close()
