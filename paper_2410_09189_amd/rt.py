"""ctypes binding of include/rt_tddft.h (argument marshalling only).

Every numerical step runs in the HIP library librt_tddft.so; this module only
lays out the C structs, keeps host arrays alive for the duration of a call and
turns status codes into exceptions.  PyTorch, when used, supplies the device
workspace and the stream.  Importing this module loads the library and fails
loudly if it has not been built.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt_tddft.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_ENOCONV, RT_ESTATE = 0, -1, -2, -3, -4, -5
RT_FP64, RT_MIXED = 0, 1
RT_PRED_LINEAR, RT_PRED_MLP, RT_PRED_QUADRATIC = 0, 1, 2
RT_HUPDATE_FULL, RT_HUPDATE_LOCAL = 0, 1

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class rt_system(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
        ("n_atoms", ctypes.c_int), ("pos", _dp), ("depth", _dp), ("width", _dp),
        ("n_images", ctypes.c_int), ("nl_rank", ctypes.c_int), ("nl_rcut", ctypes.c_double),
        ("nl_sigma", ctypes.c_double), ("nl_D", _dp), ("n_occ", ctypes.c_int),
        ("n_virt", ctypes.c_int), ("occ", _dp), ("psi0", ctypes.c_void_p),
        ("psi0_on_device", ctypes.c_int), ("orthonormalize", ctypes.c_int),
        ("nonorthogonal", ctypes.c_int), ("saw_jump", ctypes.c_int * 3),
        ("dipole_correction", ctypes.c_int), ("ion_charge", _dp),
    ]


class rt_run(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double), ("n_steps_max", ctypes.c_int), ("h_thrs", ctypes.c_double),
        ("dp_thrs", ctypes.c_double), ("max_scf", ctypes.c_int), ("max_terms", ctypes.c_int),
        ("precision", ctypes.c_int), ("predictor", ctypes.c_int), ("hupdate", ctypes.c_int),
        ("frozen_hxc", ctypes.c_int), ("n_traj", ctypes.c_int), ("traj_sys", _ip),
        ("traj_kappa", _dp), ("traj_axis", _ip), ("mlp_params", ctypes.POINTER(ctypes.c_float)),
        ("traj_field", _dp), ("magnus_order", ctypes.c_int), ("graph_capture", ctypes.c_int),
        ("h_block", ctypes.c_int),
    ]


class rt_step_stats(ctypes.Structure):
    _fields_ = [("scf_iters", ctypes.c_int32), ("series_terms", ctypes.c_int32),
                ("residual", ctypes.c_double)]


class rt_gs_params(ctypes.Structure):
    _fields_ = [("n_guard", ctypes.c_int), ("degree", ctypes.c_int), ("max_scf", ctypes.c_int),
                ("max_passes", ctypes.c_int), ("tol_rho", ctypes.c_double), ("tol_res", ctypes.c_double),
                ("mix", ctypes.c_double), ("pulay_depth", ctypes.c_int)]


class rt_gs_stats(ctypes.Structure):
    _fields_ = [("scf_iters", ctypes.c_int32), ("filter_passes", ctypes.c_int32), ("h_applies", ctypes.c_int64),
                ("eigensolves", ctypes.c_int64), ("jacobi_sweeps", ctypes.c_int64), ("rho_err", ctypes.c_double),
                ("residual", ctypes.c_double)]


class RTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2410_09189_amd/build.py")
    # One HIP runtime per process: PyTorch brings its own libamdhip64, and the
    # library must bind to that one (same soname) rather than load a second
    # runtime, which could not open the device.  So torch is loaded first.
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    sig = {
        "rt_workspace_size": ([ctypes.POINTER(rt_system), ctypes.c_int, ctypes.POINTER(rt_run),
                               ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "rt_init": ([ctypes.POINTER(rt_system), ctypes.c_int, ctypes.POINTER(rt_run), vp, ctypes.c_size_t,
                     vp, ctypes.POINTER(vp)], ctypes.c_int),
        "rt_apply_h": ([vp, ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "rt_step": ([vp, ctypes.c_int, ctypes.POINTER(rt_step_stats)], ctypes.c_int),
        "rt_dipole": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp], ctypes.c_int),
        "rt_get_matrix": ([vp, ctypes.c_int, ctypes.c_int, _dp], ctypes.c_int),
        "rt_set_state": ([vp, ctypes.c_int, _dp, _dp, _dp, _dp], ctypes.c_int),
        "rt_autotune": ([vp, ctypes.c_char_p], ctypes.c_int),
        "rt_tune_set": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "rt_tune_get": ([vp, ctypes.c_int, ctypes.c_int, _ip, _ip, _ip], ctypes.c_int),
        "rt_tune_report": ([vp], ctypes.c_char_p),
        "rt_checkpoint_size": ([vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "rt_checkpoint_save": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "rt_checkpoint_load": ([vp, vp, ctypes.c_size_t], ctypes.c_int),
        "rt_eval_h": ([vp, ctypes.c_int, vp, vp], ctypes.c_int),
        "rt_propagate": ([vp, ctypes.c_int, vp, ctypes.c_double, vp, vp, _ip], ctypes.c_int),
        "rt_get_grid": ([vp, ctypes.c_int, ctypes.c_int, _dp], ctypes.c_int),
        "rt_profile": ([vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "rt_profile_read": ([vp, ctypes.c_int, _dp, ctypes.POINTER(ctypes.c_long),
                             ctypes.POINTER(ctypes.c_char_p)], ctypes.c_int),
        "rt_mlp_dims": ([_ip, _ip, _ip], None),
        "rt_mlp_n_params": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int64),
        "rt_mlp_work_floats": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int64),
        "rt_mlp_forward": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.c_int, vp], ctypes.c_int),
        "rt_mlp_loss_grad": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.c_int, vp, vp, vp],
                             ctypes.c_int),
        "rt_mlp_adam": ([vp, vp, vp, vp, vp, ctypes.c_int64, ctypes.c_int, ctypes.c_float], ctypes.c_int),
        "rt_mlp_colstats": ([vp, vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_float], ctypes.c_int),
        "rt_record": ([vp, vp, vp, ctypes.c_int], ctypes.c_int),
        "rt_record_count": ([vp, _ip], ctypes.c_int),
        "rt_ground_state_workspace_size": ([ctypes.POINTER(rt_system), ctypes.POINTER(rt_gs_params),
                                            ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "rt_ground_state": ([ctypes.POINTER(rt_system), ctypes.POINTER(rt_gs_params), vp, ctypes.c_size_t, vp, vp,
                             _dp, vp, ctypes.POINTER(rt_gs_stats)], ctypes.c_int),
        "rt_eigh_workspace_size": ([ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "rt_eigh": ([vp, ctypes.c_int, vp, vp, vp, vp, ctypes.c_size_t, _ip], ctypes.c_int),
        "rt_eigh_noalloc": ([vp, ctypes.c_int, vp, vp, vp, _ip], ctypes.c_int),
        "rt_free": ([vp], None),
        "rt_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _ptr(a, ctype=ctypes.c_double):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctype))


def _check(status, ctx=None):
    if status != RT_OK:
        msg = lib.rt_last_error(ctx)
        raise RTError(status, msg.decode() if msg else "")


class SystemArgs:
    """Holds the host arrays referenced by one rt_system struct."""

    def __init__(self, n, h, pos, depth, width, n_occ, n_virt, psi0, nl_rank=0, nl_rcut=2.0,
                 nl_sigma=0.6, nl_D=None, n_images=2, occ=None, orthonormalize=False,
                 nonorthogonal=False, saw_jump=(0, 0, 0), dipole_correction=0, ion_charge=None):
        self.pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        self.depth = np.ascontiguousarray(depth, dtype=np.float64)
        self.width = np.ascontiguousarray(width, dtype=np.float64)
        self.nl_D = None if nl_D is None else np.ascontiguousarray(nl_D, dtype=np.float64)
        self.occ = None if occ is None else np.ascontiguousarray(occ, dtype=np.float64)
        self.ion_charge = None if ion_charge is None else np.ascontiguousarray(ion_charge, dtype=np.float64)
        if self.ion_charge is not None and self.ion_charge.shape != (self.pos.shape[0],):
            raise ValueError("ion_charge needs one value per atom")
        self.psi0 = psi0  # numpy float64 array (host) or torch CUDA tensor (device)
        s = rt_system()
        s.n[:] = list(n)
        s.h = h
        s.n_atoms = self.pos.shape[0]
        s.pos, s.depth, s.width = _ptr(self.pos), _ptr(self.depth), _ptr(self.width)
        s.n_images = n_images
        s.nl_rank, s.nl_rcut, s.nl_sigma = nl_rank, nl_rcut, nl_sigma
        s.nl_D = _ptr(self.nl_D)
        s.n_occ, s.n_virt = n_occ, n_virt
        s.occ = _ptr(self.occ)
        if isinstance(psi0, np.ndarray):
            assert psi0.dtype == np.float64 and psi0.flags.c_contiguous
            s.psi0 = psi0.ctypes.data
            s.psi0_on_device = 0
        else:
            s.psi0 = psi0.data_ptr()
            s.psi0_on_device = 1
        s.orthonormalize = int(orthonormalize)
        s.nonorthogonal = int(nonorthogonal)
        s.saw_jump[:] = [int(v) for v in saw_jump]
        s.dipole_correction = int(dipole_correction)
        s.ion_charge = _ptr(self.ion_charge)
        self.struct = s


class RunArgs:
    def __init__(self, dt, n_steps_max, h_thrs, dp_thrs, max_scf, max_terms, traj_sys, traj_kappa,
                 traj_axis, precision=RT_FP64, predictor=RT_PRED_LINEAR, hupdate=RT_HUPDATE_FULL,
                 frozen_hxc=False, mlp_params=None, traj_field=None, magnus_order=0, graph_capture=True,
                 h_block=0):
        self.traj_sys = np.ascontiguousarray(traj_sys, dtype=np.int32)
        self.traj_kappa = np.ascontiguousarray(traj_kappa, dtype=np.float64)
        self.traj_axis = np.ascontiguousarray(traj_axis, dtype=np.int32)
        r = rt_run()
        r.dt, r.n_steps_max, r.h_thrs, r.dp_thrs = dt, n_steps_max, h_thrs, dp_thrs
        r.max_scf, r.max_terms = max_scf, max_terms
        r.precision, r.predictor, r.hupdate, r.frozen_hxc = precision, predictor, hupdate, int(frozen_hxc)
        r.graph_capture = int(graph_capture)
        r.h_block = int(h_block)
        r.n_traj = len(self.traj_sys)
        r.traj_sys = _ptr(self.traj_sys, ctypes.c_int)
        r.traj_kappa = _ptr(self.traj_kappa)
        r.traj_axis = _ptr(self.traj_axis, ctypes.c_int)
        self.mlp_params = None if mlp_params is None else np.ascontiguousarray(mlp_params, dtype=np.float32)
        r.mlp_params = _ptr(self.mlp_params, ctypes.c_float)
        # traj_field: per trajectory (a, omega, tau, phase, d_x, d_y, d_z) of a sin^2 pulse
        self.traj_field = (None if traj_field is None else
                           np.ascontiguousarray(np.reshape(traj_field, (r.n_traj, 7)), dtype=np.float64))
        r.traj_field = _ptr(self.traj_field)
        r.magnus_order = int(magnus_order)
        self.struct = r


def _check_psi_rows(system, rows):
    """The library copies rows * ng doubles from psi0; a shorter array would be read
    past its end (on the device that is a memory fault), so refuse it here."""
    s = system.struct
    need = rows * s.n[0] * s.n[1] * s.n[2]
    a = system.psi0
    have = a.size if isinstance(a, np.ndarray) else a.numel()
    dtype_ok = a.dtype == np.float64 if isinstance(a, np.ndarray) else str(a.dtype) == "torch.float64"
    if have != need or not dtype_ok:
        raise ValueError(f"psi0 must hold {rows} x {need // max(rows, 1)} float64 values, got {have} ({a.dtype})")
    if not isinstance(a, np.ndarray) and not a.is_contiguous():
        raise ValueError("psi0 must be contiguous")


def rt_workspace_size(systems, run) -> int:
    arr = (rt_system * len(systems))(*[s.struct for s in systems])
    out = ctypes.c_size_t(0)
    _check(lib.rt_workspace_size(arr, len(systems), ctypes.byref(run.struct), ctypes.byref(out)))
    return out.value


def rt_init(systems, run, workspace_ptr: int, ws_bytes: int, stream_ptr: int):
    for sy in systems:
        _check_psi_rows(sy, sy.struct.n_occ + sy.struct.n_virt)
    arr = (rt_system * len(systems))(*[s.struct for s in systems])
    ctx = ctypes.c_void_p(None)
    _check(lib.rt_init(arr, len(systems), ctypes.byref(run.struct), ctypes.c_void_p(workspace_ptr),
                       ws_bytes, ctypes.c_void_p(stream_ptr), ctypes.byref(ctx)))
    return ctx


def rt_apply_h(ctx, sys_index, psi_ptr, hpsi_ptr, n_orb, dtype):
    _check(lib.rt_apply_h(ctx, sys_index, ctypes.c_void_p(psi_ptr), ctypes.c_void_p(hpsi_ptr), n_orb, dtype), ctx)


def rt_step(ctx, n_steps, n_traj=None, stats=False):
    buf = (rt_step_stats * (n_steps * n_traj))() if stats else None
    _check(lib.rt_step(ctx, n_steps, buf), ctx)
    if stats:
        return [(b.scf_iters, b.series_terms, b.residual) for b in buf]
    return None


def rt_dipole(ctx, traj, first_step, count):
    mu = np.zeros((count, 3))
    e = np.zeros(count)
    tr = np.zeros(count)
    _check(lib.rt_dipole(ctx, traj, first_step, count, _ptr(mu), _ptr(e), _ptr(tr)), ctx)
    return mu, e, tr


def rt_get_matrix(ctx, traj, which, n):
    out = np.zeros((n, n))
    _check(lib.rt_get_matrix(ctx, traj, which, _ptr(out)), ctx)
    return out


def rt_set_state(ctx, traj, p_re=None, p_im=None, h0=None, hm1=None):
    args = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (p_re, p_im, h0, hm1)]
    _check(lib.rt_set_state(ctx, traj, *[_ptr(a) for a in args]), ctx)


def rt_eval_h(ctx, sys_index, p_re_ptr, h_out_ptr):
    _check(lib.rt_eval_h(ctx, sys_index, ctypes.c_void_p(p_re_ptr), ctypes.c_void_p(h_out_ptr)), ctx)


def rt_propagate(ctx, sys_index, hbar_ptr, dt, p_re_ptr, p_im_ptr):
    terms = ctypes.c_int(0)
    _check(lib.rt_propagate(ctx, sys_index, ctypes.c_void_p(hbar_ptr), dt, ctypes.c_void_p(p_re_ptr),
                            ctypes.c_void_p(p_im_ptr), ctypes.byref(terms)), ctx)
    return terms.value


def rt_get_grid(ctx, sys_index, which, shape):
    out = np.zeros(shape)
    _check(lib.rt_get_grid(ctx, sys_index, which, _ptr(out)), ctx)
    return out


def rt_profile(ctx, enable=True, reset=True):
    _check(lib.rt_profile(ctx, int(enable), int(reset)), ctx)


def rt_profile_read(ctx):
    """{phase name: (total ms, launches)} for every phase."""
    out = {}
    for ph in range(10):
        ms = ctypes.c_double(0)
        n = ctypes.c_long(0)
        name = ctypes.c_char_p()
        _check(lib.rt_profile_read(ctx, ph, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(name)), ctx)
        out[name.value.decode()] = (ms.value, n.value)
    return out


def rt_mlp_dims():
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib.rt_mlp_dims(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def rt_mlp_n_params(n_in, n_h, n_out):
    return int(lib.rt_mlp_n_params(n_in, n_h, n_out))


def rt_mlp_work_floats(n_in, n_h, n_out, batch):
    return int(lib.rt_mlp_work_floats(n_in, n_h, n_out, batch))


def rt_mlp_forward(stream, dims, params_ptr, x_ptr, y_ptr, batch, work_ptr):
    _check(lib.rt_mlp_forward(ctypes.c_void_p(stream), *dims, ctypes.c_void_p(params_ptr), ctypes.c_void_p(x_ptr),
                              ctypes.c_void_p(y_ptr), batch, ctypes.c_void_p(work_ptr)))


def rt_mlp_loss_grad(stream, dims, params_ptr, x_ptr, t_ptr, batch, grads_ptr, work_ptr, loss_ptr):
    _check(lib.rt_mlp_loss_grad(ctypes.c_void_p(stream), *dims, ctypes.c_void_p(params_ptr), ctypes.c_void_p(x_ptr),
                                ctypes.c_void_p(t_ptr), batch, ctypes.c_void_p(grads_ptr), ctypes.c_void_p(work_ptr),
                                ctypes.c_void_p(loss_ptr)))


def rt_mlp_adam(stream, p_ptr, g_ptr, m_ptr, v_ptr, n, t, lr):
    _check(lib.rt_mlp_adam(ctypes.c_void_p(stream), ctypes.c_void_p(p_ptr), ctypes.c_void_p(g_ptr),
                           ctypes.c_void_p(m_ptr), ctypes.c_void_p(v_ptr), n, t, lr))


def rt_mlp_colstats(stream, x_ptr, rows, cols, mean_ptr, scale_ptr, floor_std):
    _check(lib.rt_mlp_colstats(ctypes.c_void_p(stream), ctypes.c_void_p(x_ptr), rows, cols,
                               ctypes.c_void_p(mean_ptr), ctypes.c_void_p(scale_ptr), floor_std))


def rt_record(ctx, x_ptr, y_ptr, capacity):
    _check(lib.rt_record(ctx, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr), capacity), ctx)


def rt_record_count(ctx):
    n = ctypes.c_int(0)
    _check(lib.rt_record_count(ctx, ctypes.byref(n)), ctx)
    return n.value


def gs_params(n_guard=8, degree=24, max_scf=100, max_passes=30, tol_rho=1e-11, tol_res=1e-10, mix=0.3,
              pulay_depth=8):
    p = rt_gs_params()
    p.n_guard, p.degree, p.max_scf, p.max_passes = n_guard, degree, max_scf, max_passes
    p.tol_rho, p.tol_res, p.mix, p.pulay_depth = tol_rho, tol_res, mix, pulay_depth
    return p


def rt_ground_state_workspace_size(system, params) -> int:
    out = ctypes.c_size_t(0)
    _check(lib.rt_ground_state_workspace_size(ctypes.byref(system.struct), ctypes.byref(params),
                                              ctypes.byref(out)))
    return out.value


def rt_ground_state(system, params, workspace_ptr, ws_bytes, stream_ptr, psi_out_ptr, rho_out_ptr=None):
    """Runs the solve; returns (Ritz values [N + n_guard], stats dict).  On a
    failure the RTError carries .eps and .stats of the last iterate."""
    n = system.struct.n_occ + system.struct.n_virt + params.n_guard
    rt_ground_state_workspace_size(system, params)  # parameter errors first (RT_EINVAL)
    _check_psi_rows(system, n)
    eps = np.zeros(n)
    st = rt_gs_stats()
    status = lib.rt_ground_state(ctypes.byref(system.struct), ctypes.byref(params), ctypes.c_void_p(workspace_ptr),
                                 ws_bytes, ctypes.c_void_p(stream_ptr), ctypes.c_void_p(psi_out_ptr), _ptr(eps),
                                 ctypes.c_void_p(rho_out_ptr), ctypes.byref(st))
    stats = {f: getattr(st, f) for f, _ in rt_gs_stats._fields_}
    if status != RT_OK:
        err = RTError(status, rt_last_error(None))
        err.eps, err.stats = eps, stats
        raise err
    return eps, stats


RT_TUNE_STENCIL_FP64, RT_TUNE_STENCIL_FP32, RT_TUNE_PROJ_FP64, RT_TUNE_PROJ_MIXED = 0, 1, 2, 3


def rt_autotune(ctx, cache_path=None) -> str:
    """Times the launch-shape candidates of the context's kernels and keeps the
    fastest (cache_path: text cache of earlier choices).  Returns the report."""
    _check(lib.rt_autotune(ctx, None if cache_path is None else str(cache_path).encode()), ctx)
    return lib.rt_tune_report(ctx).decode()


def rt_tune_set(ctx, sys_index, kernel, p1, p2=0, p3=0):
    _check(lib.rt_tune_set(ctx, sys_index, kernel, p1, p2, p3), ctx)


def rt_tune_get(ctx, sys_index, kernel):
    a, b, c = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
    _check(lib.rt_tune_get(ctx, sys_index, kernel, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), ctx)
    return a.value, b.value, c.value


def rt_checkpoint_save(ctx) -> np.ndarray:
    """The context's checkpoint as a host byte array."""
    n = ctypes.c_size_t(0)
    _check(lib.rt_checkpoint_size(ctx, ctypes.byref(n)), ctx)
    buf = np.empty(n.value, dtype=np.uint8)
    _check(lib.rt_checkpoint_save(ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.size), ctx)
    return buf


def rt_checkpoint_load(ctx, buf):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(lib.rt_checkpoint_load(ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.size), ctx)


def rt_eigh_workspace_size(n) -> int:
    out = ctypes.c_size_t(0)
    _check(lib.rt_eigh_workspace_size(n, ctypes.byref(out)))
    return out.value


def rt_eigh(stream_ptr, n, a_ptr, evals_ptr, vecs_ptr, workspace_ptr, ws_bytes):
    """Returns the number of Jacobi sweeps."""
    sw = ctypes.c_int(0)
    _check(lib.rt_eigh(ctypes.c_void_p(stream_ptr), n, ctypes.c_void_p(a_ptr), ctypes.c_void_p(evals_ptr),
                       ctypes.c_void_p(vecs_ptr), ctypes.c_void_p(workspace_ptr), ws_bytes, ctypes.byref(sw)))
    return sw.value


RT_EIGH_NOALLOC_MAX_N = 512


def rt_eigh_noalloc(stream_ptr, n, a_ptr, evals_ptr, vecs_ptr):
    """rt_eigh without a workspace (the library's static per-GPU array, n <= 512).
    Returns the number of Jacobi sweeps."""
    sw = ctypes.c_int(0)
    _check(lib.rt_eigh_noalloc(ctypes.c_void_p(stream_ptr), n, ctypes.c_void_p(a_ptr), ctypes.c_void_p(evals_ptr),
                               ctypes.c_void_p(vecs_ptr), ctypes.byref(sw)))
    return sw.value


def ground_state(system, params, device="cuda"):
    """Device workspace from torch, then rt_ground_state on torch's current stream.
    Returns (psi [N][ng] torch tensor on the device, Ritz values, rho tensor, stats).
    When the density loop stops at max_scf the RTError also carries .psi and .rho
    of the last iterate."""
    import torch

    s = system.struct
    ng = s.n[0] * s.n[1] * s.n[2]
    N = s.n_occ + s.n_virt
    ws_bytes = rt_ground_state_workspace_size(system, params)
    _check_psi_rows(system, N + params.n_guard)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
    psi = torch.empty((N, ng), dtype=torch.float64, device=device)
    rho = torch.empty(ng, dtype=torch.float64, device=device)
    stream = torch.cuda.current_stream(device).cuda_stream
    try:
        eps, stats = rt_ground_state(system, params, ws.data_ptr(), ws_bytes, stream, psi.data_ptr(), rho.data_ptr())
    except RTError as e:
        if e.status == RT_ENOCONV and e.stats.get("scf_iters", 0) >= params.max_scf:
            e.psi, e.rho = psi, rho  # the last iterate of the density loop
        raise
    del ws
    return psi, eps, rho, stats


def eigh(a, device="cuda"):
    """Eigen-decomposition of the symmetric part of a (numpy [n][n]) by rt_eigh.
    Returns (eigenvalues ascending, eigenvectors as rows, sweeps)."""
    import torch

    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    ws_bytes = rt_eigh_workspace_size(n)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
    A = torch.from_numpy(a).to(device)
    ev = torch.empty(n, dtype=torch.float64, device=device)
    V = torch.empty((n, n), dtype=torch.float64, device=device)
    stream = torch.cuda.current_stream(device).cuda_stream
    sw = rt_eigh(stream, n, A.data_ptr(), ev.data_ptr(), V.data_ptr(), ws.data_ptr(), ws_bytes)
    return ev.cpu().numpy(), V.cpu().numpy(), sw


def rt_free(ctx):
    lib.rt_free(ctx)


def rt_last_error(ctx=None) -> str:
    m = lib.rt_last_error(ctx)
    return m.decode() if m else ""


class Session:
    """Device workspace (a torch uint8 tensor) + context on torch's current stream."""

    def __init__(self, systems, run, device="cuda"):
        import torch

        self.systems, self.run = systems, run
        self.ws_bytes = rt_workspace_size(systems, run)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(device).cuda_stream
        self.ctx = rt_init(systems, run, self.ws.data_ptr(), self.ws_bytes, self.stream)

    def close(self):
        """Frees the context and lets torch reuse the workspace (after the stream's
        work on it has finished)."""
        if getattr(self, "ctx", None) is not None:  # (absent when rt_init raised)
            rt_free(self.ctx)
            self.ctx = None
        if getattr(self, "ws", None) is not None:
            import torch

            torch.cuda.synchronize(self.ws.device)
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
