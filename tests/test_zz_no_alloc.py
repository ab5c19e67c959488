"""The allocation-free eigensolver entry point (rt_eigh_noalloc, static per-GPU
work array) against the workspace entry point rt_eigh, through the C ABI: the
same kernels run in the same order, so results agree bit for bit, and both
agree with LAPACK.  Calls in a row reuse the array: the largest size first,
then smaller ones (odd n takes the padded order)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _sym(n, seed):
    a = np.random.default_rng(seed).standard_normal((n, n))
    return 0.5 * (a + a.T)


def test_eigh_noalloc_equals_workspace_eigh_on_calls_in_a_row():
    import torch

    from paper_2410_09189_amd import rt

    assert torch.cuda.is_available(), "GPU test without a GPU"
    stream = torch.cuda.current_stream().cuda_stream
    for n in (rt.RT_EIGH_NOALLOC_MAX_N, 130, 37):
        _say(f"rt_eigh_noalloc n={n}")
        a = _sym(n, 900 + n)
        A = torch.from_numpy(a).cuda()
        ev = torch.empty(n, dtype=torch.float64, device="cuda")
        V = torch.empty((n, n), dtype=torch.float64, device="cuda")
        sw = rt.rt_eigh_noalloc(stream, n, A.data_ptr(), ev.data_ptr(), V.data_ptr())
        ev_na, V_na = ev.cpu().numpy(), V.cpu().numpy()
        ev_ws, V_ws, sw_ws = rt.eigh(a)
        assert sw == sw_ws
        assert np.array_equal(ev_na, ev_ws) and np.array_equal(V_na, V_ws)
        nrm = np.linalg.norm(a, 2)
        assert np.max(np.abs(ev_na - np.linalg.eigvalsh(a))) <= 2e-13 * nrm
        resid = np.linalg.norm(a @ V_na.T - V_na.T * ev_na[None, :], axis=0)
        assert np.max(resid) <= 2e-13 * nrm * np.sqrt(n)
        assert np.max(np.abs(V_na @ V_na.T - np.eye(n))) <= 2e-13 * np.sqrt(n)
