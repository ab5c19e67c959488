"""The autotuner of launch shapes, through the C ABI.  Every stencil tiling it
may pick (y-tile rows x z chunks x halo look-ahead) gives the same H apply bit
for bit in FP64 and
FP32; tuned runs (stencil tiles and projection splits chosen by timing) agree
with runs at the built-in shapes within rounding -- the FP64 parity bound and the
mixed-precision bound; a second context reads every choice from the cache."""

import numpy as np
import pytest

import synth
from conftest import c1_ground_state, c1_system
from rt_helpers import run_args, system_args

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _ragged():
    s = synth.make_system((36, 40, 32), 0.3, 6, 10, 10, seed=7, nl_rank=4, region=(0.3, 0.7))
    return s, synth.lowpass_orbitals((36, 40, 32), 0.3, 20, 7)


def test_every_stencil_tiling_gives_the_same_apply_bitwise():
    _say("stencil tilings, 36x40x32 N=20, fp64 and fp32")
    import torch

    from paper_2410_09189_amd import rt

    s, psi = _ragged()
    ses = rt.Session([system_args(s, psi, orthonormalize=True)], run_args(synth.RunParams(dt=0.05, n_steps=2)))
    x64 = torch.from_numpy(psi.reshape(20, -1)).cuda()
    for dtype, kern, x in ((0, rt.RT_TUNE_STENCIL_FP64, x64), (1, rt.RT_TUNE_STENCIL_FP32, x64.float())):
        y = torch.empty_like(x)
        rt.rt_apply_h(ses.ctx, 0, x.data_ptr(), y.data_ptr(), 20, dtype)
        ref = y.cpu().numpy()
        spr = 36 // (2 if dtype == 0 else 4)
        n = 0
        tys = [t for t in range(1, 41) if 40 % t == 0 and t * spr <= 1024]  # (two strips a thread past 512)
        # every tiling at the built-in halo look-ahead, then every look-ahead on a few
        # tilings (z chunks of 2 planes have fewer planes than the look-ahead)
        shapes = [(ty, nzc, 0) for ty in tys for nzc in (1, 2, 4, 8, 16)]
        shapes += [(ty, nzc, hq) for ty in (tys[0], tys[-1]) for nzc in (1, 4, 16) for hq in (3, 4, 5, 6, 8)]
        for ty, nzc, hq in shapes:
            rt.rt_tune_set(ses.ctx, 0, kern, ty, nzc, hq)
            y.zero_()
            rt.rt_apply_h(ses.ctx, 0, x.data_ptr(), y.data_ptr(), 20, dtype)
            assert np.array_equal(y.cpu().numpy(), ref), (dtype, ty, nzc, hq)
            n += 1
        assert n >= 55
        with pytest.raises(rt.RTError):
            rt.rt_tune_set(ses.ctx, 0, kern, 3, 1)  # 3 does not divide ny = 40
        with pytest.raises(rt.RTError):
            rt.rt_tune_set(ses.ctx, 0, kern, 0, 0, 2)  # not a look-ahead candidate
        rt.rt_tune_set(ses.ctx, 0, kern, 0, 0)
    ses.close()


def test_two_strip_tilings_give_the_same_apply_bitwise():
    """Tiles of more than 512 strips run with two strips a thread (and one or two
    halo strips): on a 96-point x edge (48 FP64 / 24 FP32 strips a row) they give the
    built-in tiling's apply bit for bit."""
    _say("two-strip stencil tilings, 96x24x16 N=20, fp64 and fp32")
    import torch

    from paper_2410_09189_amd import rt

    n = (96, 24, 16)
    s = synth.make_system(n, 0.3, 4, 10, 10, seed=9, nl_rank=0, region=(0.3, 0.7))
    psi = synth.lowpass_orbitals(n, 0.3, 20, 9)
    ses = rt.Session([system_args(s, psi, orthonormalize=True)], run_args(synth.RunParams(dt=0.05, n_steps=2)))
    x64 = torch.from_numpy(psi.reshape(20, -1)).cuda()
    for dtype, kern, x, spr in ((0, rt.RT_TUNE_STENCIL_FP64, x64, 48), (1, rt.RT_TUNE_STENCIL_FP32, x64.float(), 24)):
        y = torch.empty_like(x)
        rt.rt_apply_h(ses.ctx, 0, x.data_ptr(), y.data_ptr(), 20, dtype)
        ref = y.cpu().numpy()
        two = [t for t in range(1, 25) if 24 % t == 0 and 512 < t * spr <= 1024]
        assert two
        for ty in two:
            for nzc, hq in ((1, 0), (2, 0), (1, 3), (1, 8)):
                rt.rt_tune_set(ses.ctx, 0, kern, ty, nzc, hq)
                y.zero_()
                rt.rt_apply_h(ses.ctx, 0, x.data_ptr(), y.data_ptr(), 20, dtype)
                assert np.array_equal(y.cpu().numpy(), ref), (dtype, ty, nzc, hq)
    ses.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_tuned_run_matches_built_in_shapes(precision, tmp_path):
    _say(f"autotuned vs built-in launch shapes, C1 three kicks, precision={precision}")
    from paper_2410_09189_amd import rt

    s = c1_system()
    psi, _ = c1_ground_state()
    rp = synth.config_run("c1_parity_32", n_steps=40, h_thrs=1e-10 if precision == 0 else 1e-9, dp_thrs=1e-14)
    kw = dict(precision=precision, hupdate=rt.RT_HUPDATE_FULL if precision == 0 else rt.RT_HUPDATE_LOCAL)
    cache = tmp_path / "tune.txt"
    mus = []
    for tuned in (False, True):
        ses = rt.Session([system_args(s, psi)], run_args(rp, n_traj_axes=(0, 1, 2), **kw))
        if tuned:
            rep = rt.rt_autotune(ses.ctx, cache)
            print(rep, flush=True)
            assert "(cached)" not in rep
        rt.rt_step(ses.ctx, 40, n_traj=3)
        mus.append(np.stack([rt.rt_dipole(ses.ctx, t, 0, 41)[0][:, t] for t in range(3)]))
        ses.close()
    d0 = mus[0] - mus[0][:, :1]
    err = np.max(np.abs(mus[1] - mus[0]))
    print(f"tuned vs built-in: max|dmu| {err:.3e} of max|dmu(t)| {np.max(np.abs(d0)):.3e}", flush=True)
    if precision == 0:
        assert err < 1e-12
    else:
        assert err < 1e-5 * np.max(np.abs(d0))
    # a second context takes every choice from the cache
    ses = rt.Session([system_args(s, psi)], run_args(rp, n_traj_axes=(0, 1, 2), **kw))
    rep = rt.rt_autotune(ses.ctx, cache)
    lines = [ln for ln in rep.splitlines() if ln.startswith("system")]
    assert lines and all("(cached)" in ln for ln in lines), rep
    ses.close()
