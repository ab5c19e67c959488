"""Throughput of the RT-TDDFT time step on one MI355X.

Workload (default): the plain-vs-mixed molecule -- 96^3 periodic grid, h = 0.3
bohr, 40 Gaussian wells with rank-4 separable projectors (r_c = 2 bohr),
160 occupied + 80 virtual orbitals, delta kick 1e-3 along x, dt = 0.05 a.u.,
self-consistency and series thresholds of the paper (1e-7, 1e-10).  Inputs are
seeded synthetic; the orbitals are the molecule's stationary ground state,
solved on the GPU by the library's ground-state solver before the timed legs
(reported, not part of the step).

One "step" = one time step of Algorithm 1 for the three delta-kick
trajectories (x, y, z) a photoabsorption spectrum needs, stepped together:
first guess of H(t + dt) (the paper's linear extrapolation for the plain FP64
leg; the headline mixed leg uses the quadratic extrapolation when its dipole
error stays at the plain leg's level), Hamiltonian self-consistency loop (commutator-series
propagation, density, FFT Hartree, LDA exchange, Hamiltonian update and
projection), observables.  All inputs are resident in HBM before the timed
region.

Equal dipole error: the plain FP64 step (linear guess, full H apply) and the mixed
step (linear or quadratic guess) each run over a sweep of self-consistency
thresholds; every leg's dipole history is compared with a tightly converged FP64
run.  `value` is the fastest mixed sweep point whose dipole error is within 3x of
the plain FP64 step's at the paper's threshold; `pareto_vs_plain` gives, for every
mixed point, the speedup over the fastest plain point with no larger error
(within 10 %).
Sweep legs run without phase timers; the phase breakdown and roofline come from
separate runs at the paper's threshold.

Also reported (not part of `value`): the 16-molecule ragged batch stepped in one
context, the non-orthogonal / fourth-order Magnus / pulse variants and the
learned first guess on this molecule, the FP32 H apply at the
192^3 x 3000-orbital nanoparticle shape, and the GPU ground-state solve of the
16 batch molecules.

Prints one JSON line.  `--gpus N` with N > 1 exits: the benchmark runs on one GPU.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RT-TDDFT steps/sec & orbital-gridpoint H-applies/sec vs plain FP64, equal dipole err"
PEAK_HBM = 8.0e12  # B/s
PEAK_FP64 = 78.6e12  # flop/s (MFMA and vector)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PEAK_BF16 = 2.5e15  # flop/s dense MFMA


def roof(phase, N, ng, mixed, T, full):
    """Algorithmic bytes and flops of one launch of a phase, and the matrix peak
    that applies.  BF16x3 contractions execute three bf16 products per FP
    product on the matrix cores.  Batched launches (T trajectories) read the
    orbitals once."""
    pairs = float(N) * (N + 1) / 2  # unique entries of a symmetric N x N result / pair products
    if phase == "project_gemm":
        if mixed:
            return 4.0 * N * ng + 4.0 * T * ng, T * 3 * 2 * pairs * ng, PEAK_BF16
        if full:  # one launch for the T trajectories: psi once, every trajectory's H psi
            return 8.0 * N * ng + 8.0 * T * N * ng, T * 2 * pairs * ng, PEAK_FP64
        return 8.0 * N * ng + 8.0 * T * ng, T * 2 * pairs * ng, PEAK_FP64
    if phase == "density":
        if mixed:
            return 4.0 * N * ng + 16.0 * T * ng, T * 3 * 2 * pairs * ng, PEAK_BF16
        return 8.0 * N * ng + 8.0 * T * ng, T * 2 * pairs * ng, PEAK_FP64
    if phase == "series_gemm":
        return T * 3 * 16.0 * N * N, T * 4.0 * N ** 3, PEAK_FP64
    if phase == "stencil_fd8":
        return 16.0 * N * ng + 8.0 * ng, 0.0, PEAK_FP64
    return None


def _oracle_sample(s, psi_host, m_mean, dt, n_traj):
    """One timed pass over the bounded sample (see cpu_baseline); returns
    (steps/s of the full workload, seconds per update, per-part timings)."""
    from oracle import grid, hamiltonian, propagate, system

    N = psi_host.shape[0]
    nx, ny, nz = s.n
    coeffs = grid.fd_coefficients_float(4)
    vloc = np.zeros(s.ng)
    projs = system.projectors(s)
    k = 16
    t0 = time.perf_counter()
    for j in range(k):
        f = psi_host[j].reshape(nz, ny, nx)
        _ = (-0.5 * grid.laplacian(f, s.h, coeffs)).ravel() + vloc * psi_host[j]
    _ = system.apply_vnl(psi_host[:k], projs, s.h)
    t_apply1 = (time.perf_counter() - t0) / k
    ns = 96
    sub = psi_host[:ns]
    rng = np.random.default_rng(0)
    A = rng.standard_normal((ns, ns))
    t0 = time.perf_counter()
    rho = hamiltonian.density(0.5 * (A + A.T), sub)
    t_dens = time.perf_counter() - t0
    t0 = time.perf_counter()
    _ = s.h ** 3 * (sub @ sub.T)
    t_proj = time.perf_counter() - t0
    t0 = time.perf_counter()
    _ = hamiltonian.hartree(rho, s)
    _ = hamiltonian.lda_x(rho)
    t_pot = time.perf_counter() - t0
    H = rng.standard_normal((N, N))
    P = np.diag(s.occupations()).astype(np.complex128)
    t0 = time.perf_counter()
    _ = propagate.propagate_exact(0.5 * (H + H.T), P, dt)
    t_exp = time.perf_counter() - t0
    scale2 = (N / ns) ** 2
    t_update = N * t_apply1 + scale2 * (t_dens + t_proj) + t_pot + t_exp
    parts = {"h_apply_ms_per_orbital": t_apply1 * 1e3, "density_s_at_96": t_dens, "projection_s_at_96": t_proj,
             "potentials_s": t_pot, "exponential_s": t_exp}
    return 1.0 / (t_update * m_mean * n_traj), t_update, parts, s.ng / t_apply1


def _oracle_c1_step(n_steps=10):
    """Whole time steps of the 32^3 parity molecule by the oracle (exact
    propagator, self-consistent midpoint at the paper's H_thrs 1e-7): steps/s."""
    import oracle
    import synth

    sysm = synth.config_system("c1_parity_32")
    d = np.load(os.path.join(ROOT, "tests", "golden", "c1_ground_state.npz"))
    m = oracle.Model(sysm, d["psi"])
    rp = synth.config_run("c1_parity_32", n_steps=n_steps, h_thrs=1e-7, dp_thrs=1e-10)
    t0 = time.perf_counter()
    oracle.run(m, rp)
    return n_steps / (time.perf_counter() - t0)


def cpu_baseline(s, psi_host, m_mean, dt, n_traj):
    """The oracle's own functions on the host's cores, timed on a bounded sample
    of the same workload and scaled to one step of the same batch:
    per-orbital H apply (FD8 Laplacian + local + nonlocal) on 16 orbitals,
    density and projection contractions at N_s = 96 scaled by (N / N_s)^2,
    Hartree + LDA on the full grid, exact exponential propagation at full N.
    One update = N applies + density + projection + potentials + propagation;
    one step = mean updates per step (from the GPU run) x trajectories.  Timed
    with all the host's BLAS threads and again with one; also whole oracle
    steps of the 32^3 parity molecule (small enough to run outright)."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits

        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threadpool_limits = None
        cores = os.cpu_count()
    N = psi_host.shape[0]
    nx, ny, nz = s.n
    v_all, t_update, parts, h_rate = _oracle_sample(s, psi_host, m_mean, dt, n_traj)
    log(f"cpu baseline ({cores} threads): one update {t_update:.1f} s")
    v_one = c1_all = c1_one = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            v_one, t_update1, _, _ = _oracle_sample(s, psi_host, m_mean, dt, n_traj)
            log(f"cpu baseline (1 thread): one update {t_update1:.1f} s")
            c1_one = _oracle_c1_step()
    c1_all = _oracle_c1_step()
    log(f"cpu baseline: 32^3 oracle steps/s {c1_all:.2f} ({cores} threads), {c1_one} (1 thread)")
    return {
        "value": v_all, "unit": "steps/s", "cores": int(cores), "kind": "oracle",
        "value_1_core": v_one,
        "sample": (f"oracle functions on the {nx}^3 N={N} workload: H apply of 16 orbitals "
                   f"({parts['h_apply_ms_per_orbital']:.0f} ms each), density+projection at N=96 scaled by "
                   f"(N/96)^2, Hartree+LDA, exact exponential; one update = {t_update:.1f} s, x {m_mean:.2f} "
                   f"updates per trajectory-step x {n_traj} trajectories per step"),
        "h_applies_per_s": h_rate,
        "c1_parity_32_steps_per_s": {"all_cores": c1_all, "one_core": c1_one,
                                     "note": "10 whole oracle steps, exact propagator, H_thrs 1e-7"},
        "parts": parts,
    }


AXES = (0, 1, 2)  # x, y, z kicks: the three runs a photoabsorption spectrum needs


def run_leg(rt, torch, sa, s, args, precision, hupdate, h_thrs, dp_thrs, profile, predictor=0):
    total = args.warmup + args.steps
    T = len(AXES)
    ra = rt.RunArgs(dt=0.05, n_steps_max=total, h_thrs=h_thrs, dp_thrs=dp_thrs, max_scf=50, max_terms=200,
                    traj_sys=[0] * T, traj_kappa=[1e-3] * T, traj_axis=list(AXES), hupdate=hupdate,
                    precision=precision, predictor=predictor)
    ses = rt.Session([sa], ra)
    ctx = ses.ctx
    if not args.no_tune:
        # launch shapes from the library's autotuner (timed once per shape, then cached)
        rt.rt_autotune(ctx, TUNE_CACHE)
    rt.rt_step(ctx, args.warmup, n_traj=T, stats=False)
    torch.cuda.synchronize()
    if profile:
        rt.rt_profile(ctx, enable=True, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = rt.rt_step(ctx, args.steps, n_traj=T, stats=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = rt.rt_profile_read(ctx) if profile else None
    dip = [rt.rt_dipole(ctx, t, 0, total + 1) for t in range(T)]
    mu = np.stack([dip[t][0][:, t] for t in range(T)], axis=1)  # mu_q of the q-kicked run
    E = np.stack([d[1] for d in dip], axis=1)
    tr = np.stack([d[2] for d in dip], axis=1)
    leg = dict(elapsed=elapsed, stats=stats, prof=prof, mu=mu, E=E, tr=tr, ses=ses)
    return leg


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
# autotuner cache of this run (a fresh file per run: the choices are timed on this GPU)
TUNE_CACHE = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"rt_tune_cache_{os.getpid()}.txt")


def measured_traffic(key, nbytes, tiling=None):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel's source file
    has changed since the counters were taken, when the counted launches had other
    algorithmic bytes than this one (another launch shape), or, for the stencil, when
    they ran another tiling (tile rows and z chunks set which halo rows and planes are
    read again; the look-ahead only sets which plane's halo is in flight)."""
    import hashlib

    try:
        rec = json.load(open(TRAFFIC_FILE))["kernels"][key]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    if abs(rec["algorithmic_bytes_per_launch"] - nbytes) > 0.5:
        return None
    if tiling is not None and list(rec.get("tiling", [0, 0]))[:2] != list(tiling)[:2]:
        return None
    return rec["traffic_bytes_per_launch"]


def roofline_of(prof, N, ng, mixed, full):
    T = len(AXES)
    cands = [k for k in prof if prof[k][1] and roof(k, N, ng, mixed, T, full)]
    dom = max(cands, key=lambda k: prof[k][0])
    nbytes, flops, pk = roof(dom, N, ng, mixed, T, full)
    ms, launches = prof[dom]
    avg = ms / 1e3 / launches
    t_hbm, t_mfma = nbytes / PEAK_HBM, (flops / pk if flops else 0.0)
    traffic = measured_traffic(dom if mixed else dom + "_fp64", nbytes)
    if t_hbm >= t_mfma:
        return {"bound": "hbm", "kernel": dom, "achieved": nbytes / avg / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": nbytes / avg / PEAK_HBM, "traffic": traffic, "avg_launch_us": avg * 1e6,
                "algorithmic_bytes_per_launch": nbytes}
    return {"bound": "mfma", "kernel": dom, "achieved": flops / avg / 1e12, "peak": pk / 1e12,
            "unit": "TFLOP/s", "frac": flops / avg / pk, "traffic": traffic, "avg_launch_us": avg * 1e6,
            "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes}


def batched_molecules(rt, torch, steps, warmup, tune=True):
    """Ragged batch: 16 synthetic molecules (grids 32^3..64^3, 10..60 orbitals) x the
    three kicks, mixed precision, stepped in one context (each molecule on its own
    stream, all advancing through the self-consistency rounds together), against the
    same 16 molecules in 16 contexts stepped one after another."""
    import synth

    mols = synth.batch_systems()
    psis = [synth.lowpass_orbitals(m.n, m.h, m.n_orb, seed=m.seed) for m in mols]

    def sa(m, p):
        return rt.SystemArgs(n=m.n, h=m.h, pos=m.pos, depth=m.depth, width=m.width, n_occ=m.n_occ,
                             n_virt=m.n_virt, psi0=p, nl_rank=m.nl_rank, nl_rcut=m.nl_rcut, nl_sigma=m.nl_sigma,
                             nl_D=m.nl_D, n_images=m.n_images, orthonormalize=True)

    def ra(n_mol):
        return rt.RunArgs(dt=0.05, n_steps_max=steps + warmup, h_thrs=1e-7, dp_thrs=1e-10, max_scf=50,
                          max_terms=200, traj_sys=[i for i in range(n_mol) for _ in AXES],
                          traj_kappa=[1e-3] * (len(AXES) * n_mol), traj_axis=list(AXES) * n_mol,
                          precision=rt.RT_MIXED, hupdate=rt.RT_HUPDATE_LOCAL)

    nm, nt = len(mols), len(AXES) * len(mols)
    ses = rt.Session([sa(m, p) for m, p in zip(mols, psis)], ra(nm))
    if tune:
        rt.rt_autotune(ses.ctx, TUNE_CACHE)
    rt.rt_step(ses.ctx, warmup, n_traj=nt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rt.rt_step(ses.ctx, steps, n_traj=nt)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    ses.close()
    sess = [rt.Session([sa(m, p)], ra(1)) for m, p in zip(mols, psis)]
    if tune:
        for x in sess:
            rt.rt_autotune(x.ctx, TUNE_CACHE)
    for x in sess:
        rt.rt_step(x.ctx, warmup, n_traj=len(AXES))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for x in sess:
            rt.rt_step(x.ctx, 1, n_traj=len(AXES))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for x in sess:
        x.close()
    return {"workload": "16 molecules (grid edges " + ",".join(str(m.n[0]) for m in mols) + "; orbitals "
                        + ",".join(str(m.n_orb) for m in mols) + ") x 3 kicks, mixed, dt 0.05, H_thrs 1e-7",
            "steps_per_s": steps / t_one, "trajectory_steps_per_s": nt * steps / t_one,
            "sequential_contexts_steps_per_s": steps / t_seq, "speedup_vs_sequential_contexts": t_seq / t_one}


def ground_states(rt, torch):
    """Ground state of each of the 16 batch molecules by the GPU solver
    (Chebyshev-filtered subspace iteration, Jacobi Rayleigh-Ritz, Pulay mixing)
    from a smooth random start block of N + n_guard vectors.  Molecules whose
    HOMO-LUMO gap is below 1e-3 Ha have no well-defined closed-shell aufbau
    ground state; the solver stops on its density-iteration cap for them."""
    import synth

    mols = synth.batch_systems()
    rows = []
    for i, m in enumerate(mols):
        N = m.n_orb
        ng_ = max(8, (N // 8 + 1) // 2 * 2)
        ng_ += (N + ng_) % 2
        x0 = synth.lowpass_orbitals(m.n, m.h, N + ng_, seed=m.seed)
        sa = rt.SystemArgs(n=m.n, h=m.h, pos=m.pos, depth=m.depth, width=m.width, n_occ=m.n_occ,
                           n_virt=m.n_virt, psi0=x0, nl_rank=m.nl_rank, nl_rcut=m.nl_rcut, nl_sigma=m.nl_sigma,
                           nl_D=m.nl_D, n_images=m.n_images)
        p = rt.gs_params(n_guard=ng_, degree=24, max_scf=80, max_passes=20, tol_rho=1e-10, tol_res=1e-9)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            _, eps, _, st = rt.ground_state(sa, p)
            ok = True
        except rt.RTError as e:
            if e.status != rt.RT_ENOCONV:
                raise
            eps, st, ok = e.eps, e.stats, False
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rows.append(dict(mol=i, grid=m.n[0], N=N, converged=ok, seconds=round(dt, 3), scf_iters=st["scf_iters"],
                         filter_passes=st["filter_passes"], homo_lumo_gap=float(eps[m.n_occ] - eps[m.n_occ - 1]),
                         rho_err=st["rho_err"], residual=st["residual"]))
    conv = [r for r in rows if r["converged"]]
    return {"workload": "the 16 batch molecules, start block N + n_guard smooth random vectors, degree 24, "
                        "tol_rho 1e-10, tol_res 1e-9, max_scf 80",
            "converged": len(conv), "seconds_total": sum(r["seconds"] for r in rows),
            "seconds_converged": sum(r["seconds"] for r in conv),
            "min_gap_converged": min((r["homo_lumo_gap"] for r in conv), default=None),
            "max_gap_not_converged": max((r["homo_lumo_gap"] for r in rows if not r["converged"]), default=None),
            "molecules": rows}


def no_kick_control(rt, torch, sa, n=100):
    """The stationary input without a kick (FP64 and mixed, local update, 100
    steps): how far the dipole and the energy move on their own."""
    out = {}
    for prec, name in ((rt.RT_FP64, "fp64"), (rt.RT_MIXED, "mixed")):
        ra = rt.RunArgs(dt=0.05, n_steps_max=n, h_thrs=1e-10, dp_thrs=1e-10, max_scf=50, max_terms=200,
                        traj_sys=[0], traj_kappa=[0.0], traj_axis=[0], hupdate=rt.RT_HUPDATE_LOCAL, precision=prec)
        ses = rt.Session([sa], ra)
        rt.rt_step(ses.ctx, n, n_traj=1)
        mu, E, _ = rt.rt_dipole(ses.ctx, 0, 0, n + 1)
        ses.close()
        out[name] = {"max_abs_dmu": float(np.max(np.abs(mu - mu[0]))), "max_abs_dE": float(np.max(np.abs(E - E[0])))}
    out["steps"] = n
    return out


def variants(rt, torch, s, psi, args):
    """The ranked extensions on the 96^3 workload, mixed precision, three
    trajectories, H_thrs 1e-7, timed like the main legs: the non-orthogonal
    basis (the ground-state orbitals mixed by a unit lower-triangular matrix,
    Phi = A Psi, overlap S = A A^T != I, the same occupied space),
    fourth-order Magnus (Omega_2 in every series term), and sin^2 pulses along
    x, y, z instead of kicks (a 1e-3, omega 0.4, tau 10).  Each against the
    plain mixed step on the same workload."""
    T = len(AXES)
    total = args.warmup + args.steps
    out = {}
    cases = (("mixed_kick", False, {}, [1e-3] * T, None),
             ("nonorthogonal_basis", True, {}, [1e-3] * T, None),
             ("magnus_order_4", False, {"magnus_order": 4}, [1e-3] * T, None),
             ("pulse_fields", False, {}, [0.0] * T,
              [[1e-3, 0.4, 10.0, 0.0] + [1.0 if q == a else 0.0 for q in range(3)] for a in AXES]))
    import synth

    phi = torch.from_numpy(synth.basis_mixing(s.n_orb, 1, lower=True)).cuda() @ psi
    for name, nonorth, extra, kappas, field in cases:
        sa = rt.SystemArgs(n=s.n, h=s.h, pos=s.pos, depth=s.depth, width=s.width, n_occ=s.n_occ,
                           n_virt=s.n_virt, psi0=phi if nonorth else psi, nl_rank=s.nl_rank, nl_rcut=s.nl_rcut,
                           nl_sigma=s.nl_sigma, nl_D=s.nl_D, n_images=s.n_images, nonorthogonal=nonorth)
        ra = rt.RunArgs(dt=0.05, n_steps_max=total, h_thrs=args.h_thrs, dp_thrs=args.dp_thrs, max_scf=50,
                        max_terms=200, traj_sys=[0] * T, traj_kappa=kappas, traj_axis=list(AXES),
                        precision=rt.RT_MIXED, hupdate=rt.RT_HUPDATE_LOCAL, traj_field=field, **extra)
        ses = rt.Session([sa], ra)
        rt.rt_step(ses.ctx, args.warmup, n_traj=T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = rt.rt_step(ses.ctx, args.steps, n_traj=T, stats=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ses.close()
        out[name] = {"steps_per_s": args.steps / el, "ms_per_step": 1e3 * el / args.steps,
                     "mean_scf_updates_per_step": float(np.mean([x[0] for x in st])),
                     "mean_series_terms_per_update": float(sum(x[1] for x in st) / max(1, sum(x[0] for x in st)))}
    base = out["mixed_kick"]["steps_per_s"]
    for v in out.values():
        v["relative_to_mixed_kick"] = v["steps_per_s"] / base
    return out


def apply_h_192(rt, torch, n_orb=3000, reps=3, tune=True):
    """Stencil roofline at the nanoparticle shape: the grid Hamiltonian (FD8 +
    V_loc; this molecule has local wells only) applied in FP32 to 3000 orbitals
    of the 192^3 grid, 85 GB in and 85 GB out, through rt_apply_h of a context
    built on 64 random orthonormalised orbitals of that molecule.  Inputs are
    seeded device-side random numbers (the time of an apply does not depend on
    the values)."""
    import synth

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
    if tune:
        # stencil tiles for this grid from the library's autotuner (timed on the
        # context's 64 orbitals; the tiling does not depend on the orbital count)
        rt.rt_autotune(ses.ctx, TUNE_CACHE)
    tiling = rt.rt_tune_get(ses.ctx, 0, rt.RT_TUNE_STENCIL_FP32)
    x = torch.randn((n_orb, ng), dtype=torch.float32, device="cuda", generator=gen)
    y = torch.empty_like(x)
    rt.rt_apply_h(ses.ctx, 0, x.data_ptr(), y.data_ptr(), n_orb, 1)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        rt.rt_apply_h(ses.ctx, 0, x.data_ptr(), y.data_ptr(), n_orb, 1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ses.close()
    del x, y
    nbytes = 8.0 * n_orb * ng + 4.0 * ng * ((n_orb + 63) // 64)
    return {"workload": f"192^3 grid (h 0.3), 600-well fcc cluster, FP32 H apply of {n_orb} orbitals "
                        "(stencil + V_loc) through rt_apply_h",
            "ms_per_apply": ms, "orbital_gridpoints_per_s": n_orb * ng / (ms * 1e-3), "stencil_tiling": tiling,
            "hbm_GBps_algorithmic": nbytes / (ms * 1e-3) / 1e9, "hbm_frac": nbytes / (ms * 1e-3) / 8e12,
            "algorithmic_bytes": nbytes}


def plane_wave_orbitals(torch, n, h, n_orb, chunk=96, device="cuda"):
    """n_orb orthonormal orbitals of the periodic n^3 grid (h^3 inner product):
    the constant and cos / sin(G . r) pairs of the lowest |G| (integer triplets m,
    one of each +-m), exactly orthogonal under the grid sum.  Generated on the
    device chunk by chunk and staged in a host array [n_orb][n^3] (float64)."""
    omega = (n * h) ** 3
    ms = []
    r = 1
    while len(ms) < n_orb:
        ms = []
        rng_ = range(-r, r + 1)
        cand = sorted(((a * a + b * b + c * c, (a, b, c)) for a in rng_ for b in rng_ for c in rng_))
        for _, m in cand:
            first = next((v for v in m if v != 0), 0)
            if m == (0, 0, 0):
                ms.append((m, "c"))
            elif first > 0:
                ms.extend([(m, "c"), (m, "s")])
        r += 1
    ms = ms[:n_orb]
    host = np.empty((n_orb, n ** 3), dtype=np.float64)
    ax = torch.arange(n, dtype=torch.float64, device=device) * (2.0 * np.pi / n)
    for j0 in range(0, n_orb, chunk):
        blk = torch.empty((min(chunk, n_orb - j0), n, n, n), dtype=torch.float64, device=device)
        for k, (m, kind) in enumerate(ms[j0:j0 + blk.shape[0]]):
            ph = (m[2] * ax)[:, None, None] + (m[1] * ax)[None, :, None] + (m[0] * ax)[None, None, :]
            if m == (0, 0, 0):
                blk[k].fill_(1.0 / np.sqrt(omega))
            else:
                (torch.cos(ph, out=blk[k]) if kind == "c" else torch.sin(ph, out=blk[k])).mul_(np.sqrt(2.0 / omega))
        torch.from_numpy(host[j0:j0 + blk.shape[0]]).copy_(blk.reshape(blk.shape[0], -1))
        del blk
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return host


def c5_time_step(rt, torch, steps=4, warmup=1, h_block=128):
    """A whole time step at the nanoparticle shape: 192^3 grid, the 600-well fcc
    cluster, 2400 occupied + 600 virtual orbitals, one x kick, mixed precision
    with the local update and the quadratic first guess.  The FP64 orbitals
    (170 GB) and their bf16 hi/lo pair (85 GB) are resident; the initial grid
    Hamiltonian is applied 128 orbitals at a time (rt_run.h_block).  The orbitals
    are orthonormal plane waves (the step's cost does not depend on their values;
    they are not the cluster's ground state, so the state evolves from the start).
    Reports steps/s, Hamiltonian updates per step and the phase times."""
    import synth

    s = synth.config_system("c5_cluster_192")
    N, ng = s.n_orb, s.ng
    t0 = time.perf_counter()
    psi = plane_wave_orbitals(torch, s.n[0], s.h, N)
    t_gen = time.perf_counter() - t0
    sa = rt.SystemArgs(n=s.n, h=s.h, pos=s.pos, depth=s.depth, width=s.width, n_occ=s.n_occ, n_virt=s.n_virt,
                       psi0=psi, n_images=s.n_images)
    n_steps = warmup + steps + 2
    ra = rt.RunArgs(dt=0.05, n_steps_max=n_steps, h_thrs=1e-7, dp_thrs=1e-10, max_scf=30, max_terms=400,
                    traj_sys=[0], traj_kappa=[1e-3], traj_axis=[0], precision=rt.RT_MIXED,
                    hupdate=rt.RT_HUPDATE_LOCAL, predictor=rt.RT_PRED_QUADRATIC, h_block=h_block)
    ws = rt.rt_workspace_size([sa], ra)
    log(f"c5: orbitals generated in {t_gen:.1f} s; workspace {ws / 2**30:.1f} GiB")
    t0 = time.perf_counter()
    ses = rt.Session([sa], ra)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    del psi, sa
    log(f"c5: rt_init {t_init:.1f} s")
    rt.rt_step(ses.ctx, warmup, n_traj=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = rt.rt_step(ses.ctx, steps, n_traj=1, stats=True)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    rt.rt_profile(ses.ctx, enable=True, reset=True)
    rt.rt_step(ses.ctx, 1, n_traj=1)
    torch.cuda.synchronize()
    ph = rt.rt_profile_read(ses.ctx)
    rt.rt_profile(ses.ctx, enable=False, reset=True)
    mu, E, tr = rt.rt_dipole(ses.ctx, 0, 0, warmup + steps + 2)
    ses.close()
    del ses
    torch.cuda.empty_cache()
    upd = [x[0] for x in st]
    return {"workload": "c5_cluster_192: 192^3 h=0.3, 600-well fcc cluster (radius 25 bohr), N=3000 (2400 occ + "
                        "600 virt), one x kick, mixed BF16x3 + local update + quadratic first guess, dt=0.05, "
                        "H_thrs=1e-07; orthonormal plane-wave orbitals",
            "steps_per_s": steps / t_run, "ms_per_step": 1e3 * t_run / steps,
            "updates_per_step": float(np.mean(upd)), "workspace_GiB": ws / 2 ** 30,
            "init_s": t_init, "orbital_generation_s": t_gen,
            "phases_ms_one_step": {k: v[0] for k, v in ph.items() if v[1]},
            "phase_launches_one_step": {k: v[1] for k, v in ph.items() if v[1]},
            "trace_electrons": float(tr[-1]), "dipole_x_change": float(mu[-1][0] - mu[0][0])}


def learned_predictor(rt, torch, sa, s):
    """The learned first guess on the 96^3 molecule (mixed precision): training
    samples recorded by the step itself on x and y kicks of two strengths, the
    network trained on the GPU with the library's kernels, then a held-out z kick
    stepped with the linear and with the learned guess at dt 0.2 (where the
    linear guess often needs a third update).  Reports Hamiltonian updates per
    step after the 8 warm-up steps the features need, the time per step, and the
    dipole difference between the two runs (same fixed point)."""
    from paper_2410_09189_amd import predictor

    dt, n_rec, n_eval, h_thrs = 0.2, 150, 100, 1e-9

    def ra(axes, kappas, n, pred=0, params=None):
        return rt.RunArgs(dt=dt, n_steps_max=n, h_thrs=h_thrs, dp_thrs=1e-13, max_scf=50, max_terms=200,
                          traj_sys=[0] * len(axes), traj_kappa=list(kappas), traj_axis=list(axes),
                          precision=rt.RT_MIXED, hupdate=rt.RT_HUPDATE_LOCAL, predictor=pred, mlp_params=params)

    t0 = time.perf_counter()
    X, Y = predictor.record(lambda: rt.Session([sa], ra((0, 1, 0, 1), (1e-3, 1e-3, 2e-3, 2e-3), n_rec)),
                            n_rec, capacity=4 * n_rec)
    t_rec = time.perf_counter() - t0
    t0 = time.perf_counter()
    params, hist = predictor.train(X, Y, epochs=30, batch=64, lr=1e-3, seed=0)
    t_train = time.perf_counter() - t0
    res = {}
    for pred in (rt.RT_PRED_LINEAR, rt.RT_PRED_MLP):
        ses = rt.Session([sa], ra((2,), (1.5e-3,), n_eval, pred=pred,
                                  params=params if pred == rt.RT_PRED_MLP else None))
        rt.rt_step(ses.ctx, 8, n_traj=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = rt.rt_step(ses.ctx, n_eval - 8, n_traj=1, stats=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        mu = rt.rt_dipole(ses.ctx, 0, 0, n_eval + 1)[0]
        ses.close()
        res[pred] = (mu, float(np.mean([x[0] for x in st])), 1e3 * el / (n_eval - 8))
    mu_l, m_l, ms_l = res[rt.RT_PRED_LINEAR]
    mu_m, m_m, ms_m = res[rt.RT_PRED_MLP]
    return {"workload": f"96^3 N=240 mixed, dt {dt}, H_thrs {h_thrs:g}; trained on x/y kicks (kappa 1e-3, 2e-3), "
                        f"{n_rec} recorded steps each; evaluated on a held-out z kick (kappa 1.5e-3), {n_eval} steps",
            "samples": int(X.shape[0]), "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
            "record_s": round(t_rec, 2), "train_s": round(t_train, 2),
            "updates_per_step_linear": m_l, "updates_per_step_learned": m_m,
            "ms_per_step_linear": ms_l, "ms_per_step_learned": ms_m,
            "dipole_max_diff_learned_vs_linear": float(np.max(np.abs(mu_m - mu_l))),
            "dipole_max_abs": float(np.max(np.abs(mu_l - mu_l[0])))}


def learned_predictor_c4(rt, torch, dts=(0.05, 0.2, 0.5, 1.0), train_seeds=(400, 404, 406, 410),
                         test_seeds=(411, 413, 14), n_rec=60, n_eval=60, h_thrs=1e-7):
    """The learned first guess across molecules: 96^3 molecules of the N=240 mixed
    workload's generator (40 wells + rank-4 projectors, 160 + 80 orbitals), ground
    states on the GPU (a density loop stopped at 40 iterations is kept when
    self-consistent to 1e-5; others are left out), samples recorded on x/y/z kicks
    of the training seeds,
    one network per time step trained on the GPU, then the held-out seeds stepped
    with a z kick under the linear, quadratic and learned guesses.  Reports
    Hamiltonian updates per step (after the 8 warm-up steps the features need),
    time per step, the network's own time per step, and the dipole difference
    to the linear run (same fixed point).  The seeds are generator seeds whose
    density loop settles within 40 iterations (of seeds 400-415 and 500-503 on the
    box: 400, 404, 406, 410, 411, 413; the rest slosh at rho_err 1e-5 - 1e-3
    between near-degenerate levels) plus the N=240 workload's own molecule (14);
    training and test molecules are disjoint."""
    import synth
    from paper_2410_09189_amd import predictor

    c = synth.CONFIGS["c2_mixed_96"]
    gsp = dict(n_guard=30, degree=24, max_scf=40, max_passes=20, tol_rho=1e-9, tol_res=1e-8, mix=0.15)

    def molecule(seed):
        s = synth.make_system(c["n"], c["h"], c["n_atoms"], c["n_occ"], c["n_virt"], seed, region=c["region"],
                              nl_rank=c["nl_rank"])
        x0 = synth.lowpass_orbitals(s.n, s.h, s.n_orb + gsp["n_guard"], seed)
        kw = dict(n=s.n, h=s.h, pos=s.pos, depth=s.depth, width=s.width, n_occ=s.n_occ, n_virt=s.n_virt,
                  nl_rank=s.nl_rank, nl_rcut=s.nl_rcut, nl_sigma=s.nl_sigma, nl_D=s.nl_D, n_images=s.n_images)
        t0 = time.perf_counter()
        try:
            psi, eps, _, st = rt.ground_state(rt.SystemArgs(psi0=x0, **kw), rt.gs_params(**gsp))
        except rt.RTError as e:
            # most molecules of this generator have HOMO-LUMO gaps of 1e-5 - 1e-3 Ha and
            # converge slowly; an iterate self-consistent to rho_err <= 1e-5 is kept
            if not hasattr(e, "psi") or not (e.stats["rho_err"] <= 1e-5):
                return None, time.perf_counter() - t0, e.stats.get("rho_err")
            psi, eps, st = e.psi, e.eps, e.stats
        return rt.SystemArgs(psi0=psi, **kw), time.perf_counter() - t0, st["rho_err"]

    def ra(dt, axes, kappas, n, pred=0, params=None):
        return rt.RunArgs(dt=dt, n_steps_max=n, h_thrs=h_thrs, dp_thrs=1e-12, max_scf=60, max_terms=400,
                          traj_sys=[0] * len(axes), traj_kappa=list(kappas), traj_axis=list(axes),
                          precision=rt.RT_MIXED, hupdate=rt.RT_HUPDATE_LOCAL, predictor=pred, mlp_params=params)

    t_gs = 0.0
    train, test, dropped = [], [], []
    for seeds, dst in ((train_seeds, train), (test_seeds, test)):
        for seed in seeds:
            sa, t, rerr = molecule(seed)
            t_gs += t
            (dst.append((seed, sa)) if sa is not None else dropped.append(seed))
            log(f"learned c4: molecule {seed} {'kept' if sa is not None else 'left out'} ({t:.1f} s, "
                f"rho_err {rerr:.1e})")
    # the network's forward pass alone, at the run's batch size (one trajectory)
    n_in, n_h, n_out = rt.rt_mlp_dims()
    out = {"workload": "96^3 molecules of the N=240 mixed workload's generator, mixed precision, local update, "
                       f"H_thrs {h_thrs:g}; train seeds {list(train_seeds)} (x/y/z kicks 1e-3, {n_rec} recorded "
                       f"steps), held-out seeds {list(test_seeds)} (z kick 1.5e-3, {n_eval} steps)",
           "train_molecules": [x[0] for x in train], "test_molecules": [x[0] for x in test],
           "left_out": dropped, "ground_state_s": round(t_gs, 1), "per_dt": {}}
    if not train or not test:
        out["note"] = "too few molecules with a usable ground state"
        return out
    for dt in dts:
        Xs, Ys = [], []
        for _, sa in train:
            X, Y = predictor.record(lambda: rt.Session([sa], ra(dt, (0, 1, 2), (1e-3,) * 3, n_rec)), n_rec,
                                    capacity=3 * n_rec)
            Xs.append(X)
            Ys.append(Y)
        X, Y = torch.cat(Xs), torch.cat(Ys)
        n_samples = X.shape[0]
        params, hist = predictor.train(X, Y, epochs=30, batch=64, lr=1e-3, seed=0)
        del Xs, Ys, X, Y
        row = {"samples": int(n_samples), "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]}
        agg = {}
        for name, pred in (("linear", rt.RT_PRED_LINEAR), ("quadratic", rt.RT_PRED_QUADRATIC),
                           ("learned", rt.RT_PRED_MLP)):
            ups, mss, dmu = [], [], []
            for seed, sa in test:
                ses = rt.Session([sa], ra(dt, (2,), (1.5e-3,), n_eval, pred=pred,
                                          params=params if pred == rt.RT_PRED_MLP else None))
                rt.rt_step(ses.ctx, 8, n_traj=1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = rt.rt_step(ses.ctx, n_eval - 8, n_traj=1, stats=True)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                mu = rt.rt_dipole(ses.ctx, 0, 0, n_eval + 1)[0][:, 2]
                ses.close()
                ups.append(float(np.mean([x[0] for x in st])))
                mss.append(1e3 * el / (n_eval - 8))
                dmu.append(mu)
            agg[name] = {"updates_per_step": float(np.mean(ups)), "ms_per_step": float(np.mean(mss)),
                         "updates_per_step_each": ups, "mu": dmu}
        for name in ("quadratic", "learned"):
            agg[name]["dipole_max_diff_vs_linear"] = float(max(np.max(np.abs(a - b)) for a, b in
                                                               zip(agg[name]["mu"], agg["linear"]["mu"])))
        scale = float(max(np.max(np.abs(m - m[0])) for m in agg["linear"]["mu"]))
        for v in agg.values():
            del v["mu"]
        row.update(agg)
        row["dipole_change_scale"] = scale
        # the network's forward pass alone (one trajectory), to separate it from the step
        x = torch.zeros((1, n_in), dtype=torch.float32, device="cuda")
        y = torch.empty((1, n_out), dtype=torch.float32, device="cuda")
        pd = torch.from_numpy(params).cuda()
        wk = torch.empty(rt.rt_mlp_work_floats(n_in, n_h, n_out, 1), dtype=torch.float32, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        for _ in range(3):
            rt.rt_mlp_forward(stream, (n_in, n_h, n_out), pd.data_ptr(), x.data_ptr(), y.data_ptr(), 1, wk.data_ptr())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            rt.rt_mlp_forward(stream, (n_in, n_h, n_out), pd.data_ptr(), x.data_ptr(), y.data_ptr(), 1, wk.data_ptr())
        e1.record()
        torch.cuda.synchronize()
        row["network_forward_ms"] = e0.elapsed_time(e1) / 20
        row["learned_ms_per_step_net_of_inference"] = row["learned"]["ms_per_step"] - row["network_forward_ms"]
        out["per_dt"][str(dt)] = row
        log(f"learned c4 dt {dt}: updates linear {agg['linear']['updates_per_step']:.2f}, quadratic "
            f"{agg['quadratic']['updates_per_step']:.2f}, learned {agg['learned']['updates_per_step']:.2f}")
    return out


def ground_state_input(rt, torch, s, name):
    """The input of the time loop: the molecule's stationary ground state, solved on
    the GPU from a block of smooth random vectors (not part of the timed step)."""
    import synth

    N = s.n_orb
    log(f"ground state of the {s.n[0]}^3 molecule on the GPU")
    x0 = synth.ground_state_start(name)
    gsp = synth.CONFIGS[name]["gs"]
    sa0 = rt.SystemArgs(n=s.n, h=s.h, pos=s.pos, depth=s.depth, width=s.width, n_occ=s.n_occ,
                        n_virt=s.n_virt, psi0=x0, nl_rank=s.nl_rank, nl_rcut=s.nl_rcut,
                        nl_sigma=s.nl_sigma, nl_D=s.nl_D, n_images=s.n_images)
    torch.cuda.synchronize()
    t_gs = time.perf_counter()
    psi, eps_gs, _, st_gs = rt.ground_state(sa0, rt.gs_params(**gsp))
    torch.cuda.synchronize()
    t_gs = time.perf_counter() - t_gs
    gs_info = {"seconds": round(t_gs, 2), "density_iterations": st_gs["scf_iters"],
               "homo_lumo_gap": float(eps_gs[s.n_occ] - eps_gs[s.n_occ - 1]),
               "active_space_edge_gap": float(eps_gs[N] - eps_gs[N - 1]), "rho_err": st_gs["rho_err"],
               "residual": st_gs["residual"], "params": gsp}
    log(f"ground state: {t_gs:.1f} s, gap {gs_info['homo_lumo_gap']:.3e}")
    sa = rt.SystemArgs(n=s.n, h=s.h, pos=s.pos, depth=s.depth, width=s.width, n_occ=s.n_occ,
                       n_virt=s.n_virt, psi0=psi, nl_rank=s.nl_rank, nl_rcut=s.nl_rcut,
                       nl_sigma=s.nl_sigma, nl_D=s.nl_D, n_images=s.n_images)
    return psi, sa, gs_info


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--h-thrs", type=float, default=1e-7)
    ap.add_argument("--sweep", type=float, nargs="+", default=[1e-6, 1e-7, 1e-8, 1e-9],
                    help="self-consistency thresholds of the equal-dipole-error sweep (must include --h-thrs)")
    ap.add_argument("--dp-thrs", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="built-in launch shapes instead of the autotuner's")
    ap.add_argument("--roofline-only", action="store_true",
                    help="run only the profiled mixed leg and print its roofline (for profiler runs of the "
                         "launches the roofline times)")
    ap.add_argument("--random-orbitals", action="store_true",
                    help="smooth random orbitals made orthonormal at init instead of the ground state (for "
                         "profiler runs: the kernels and their traffic do not depend on the orbitals' values)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 16-molecule batch leg")
    ap.add_argument("--no-ground-state", action="store_true", help="skip the GPU ground-state leg")
    ap.add_argument("--only-ground-state", action="store_true",
                    help="run only the GPU ground-state leg (for profiling it on its own)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-predictor leg")
    ap.add_argument("--no-192", action="store_true", help="skip the 192^3 x 3000-orbital FP32 apply leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the non-orthogonal / fourth-order Magnus / pulse legs")
    ap.add_argument("--only-variants", action="store_true", help="run only those legs")
    ap.add_argument("--only-192", action="store_true", help="run only the 192^3 apply leg")
    ap.add_argument("--only-batch", action="store_true", help="run only the 16-molecule batch leg")
    ap.add_argument("--only-c5", action="store_true", help="run only the 192^3 x 3000 time-step leg")
    ap.add_argument("--only-learned-c4", action="store_true",
                    help="run only the learned guess across molecules and time steps")
    ap.add_argument("--only-learned", action="store_true", help="run only the learned-predictor leg")
    args = ap.parse_args()
    if args.h_thrs not in args.sweep:
        args.sweep = sorted(set(args.sweep) | {args.h_thrs}, reverse=True)
    if args.gpus != 1:
        print("bench.py: the benchmark runs on exactly one GPU (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2410_09189_amd import rt

    if args.only_192:
        log("FP32 H apply, 192^3 x 3000 orbitals")
        print(json.dumps({"apply_h_192": apply_h_192(rt, torch, tune=not args.no_tune)}), flush=True)
        return
    if args.only_learned_c4:
        log("learned first guess: train on 4 molecules, test on 3 held out, dt 0.05 .. 1.0")
        print(json.dumps({"learned_predictor_c4": learned_predictor_c4(rt, torch)}), flush=True)
        return
    if args.only_c5:
        log("time step, 192^3 x 3000 orbitals (mixed, blocked initialisation)")
        print(json.dumps({"c5_time_step": c5_time_step(rt, torch)}), flush=True)
        return
    if args.only_batch:
        log("batched: 16 molecules x 3 kicks in one context vs 16 contexts")
        print(json.dumps({"batched_16_molecules": batched_molecules(rt, torch, args.steps, args.warmup,
                                                                     tune=not args.no_tune)}), flush=True)
        return
    if args.only_ground_state:
        log("ground states of the 16 batch molecules on the GPU")
        print(json.dumps({"ground_state_16_molecules": ground_states(rt, torch)}), flush=True)
        return
    name = "c2_mixed_96"
    s = synth.config_system(name)
    N = s.n_orb
    # the input of the time loop: the molecule's stationary ground state, solved on
    # the GPU from a block of smooth random vectors (not part of the timed step)
    if args.random_orbitals:
        log("smooth random orbitals (profiling run)")
        x = synth.lowpass_orbitals(s.n, s.h, N, seed=s.seed)
        psi = torch.from_numpy(x.reshape(N, -1)).cuda()
        del x
        sa = rt.SystemArgs(n=s.n, h=s.h, pos=s.pos, depth=s.depth, width=s.width, n_occ=s.n_occ,
                           n_virt=s.n_virt, psi0=psi, nl_rank=s.nl_rank, nl_rcut=s.nl_rcut,
                           nl_sigma=s.nl_sigma, nl_D=s.nl_D, n_images=s.n_images, orthonormalize=True)
        gs_info = {"skipped": "random orbitals"}
    else:
        psi, sa, gs_info = ground_state_input(rt, torch, s, name)
    if args.only_variants:
        log("variants: non-orthogonal basis, fourth-order Magnus, pulses")
        print(json.dumps({"variants_96": variants(rt, torch, s, psi, args)}), flush=True)
        return
    if args.only_learned:
        log("learned predictor: record, train, evaluate")
        print(json.dumps({"learned_predictor_96": learned_predictor(rt, torch, sa, s)}), flush=True)
        return
    if args.roofline_only:
        log("profiled mixed leg only (quadratic first guess, paper threshold)")
        prof = run_leg(rt, torch, sa, s, args, rt.RT_MIXED, rt.RT_HUPDATE_LOCAL, args.h_thrs, args.dp_thrs, True,
                       predictor=rt.RT_PRED_QUADRATIC)
        prof["ses"].close()
        print(json.dumps({"roofline": roofline_of(prof["prof"], N, s.ng, True, False),
                          "updates_per_step": sum(x[0] for x in prof["stats"]) / len(prof["stats"]),
                          "phases_ms": {k: round(v[0], 3) for k, v in prof["prof"].items() if v[1]},
                          "phases_launches": {k: v[1] for k, v in prof["prof"].items() if v[1]}}), flush=True)
        return
    log("reference: FP64, tight thresholds (1e-12, 1e-15)")
    ref = run_leg(rt, torch, sa, s, args, rt.RT_FP64, rt.RT_HUPDATE_FULL, 1e-12, 1e-15, False)
    ref["ses"].close()
    log(f"reference done: {1e3 * ref['elapsed'] / args.steps:.2f} ms/step")
    # Equal-dipole-error comparison: each method over a sweep of self-consistency
    # thresholds (the paper's 1e-7 among them), timed without phase timers.
    # plain_fp64: the paper's step (full H apply + projection per update);
    # fp64_local: the same FP64 arithmetic with the Hamiltonian update
    # H[P] = H_gs + h^3 Psi^T dV Psi (exact, no grid apply in the loop), so that the
    # mixed step's gain splits into the update shortcut and the precision
    methods = (("plain_fp64", rt.RT_FP64, rt.RT_HUPDATE_FULL, rt.RT_PRED_LINEAR),
               ("fp64_local", rt.RT_FP64, rt.RT_HUPDATE_LOCAL, rt.RT_PRED_LINEAR),
               ("mixed_linear", rt.RT_MIXED, rt.RT_HUPDATE_LOCAL, rt.RT_PRED_LINEAR),
               ("mixed_quadratic", rt.RT_MIXED, rt.RT_HUPDATE_LOCAL, rt.RT_PRED_QUADRATIC))
    legs = {}
    for mname, prec, hup, pred in methods:
        for th in args.sweep:
            log(f"leg {mname} H_thrs={th:g}")
            leg = run_leg(rt, torch, sa, s, args, prec, hup, th, args.dp_thrs, False, predictor=pred)
            leg["ses"].close()
            legs[(mname, th)] = leg
            log(f"leg {mname} H_thrs={th:g} done: {1e3 * leg['elapsed'] / args.steps:.2f} ms/step")
    plain = legs[("plain_fp64", args.h_thrs)]
    fp64_local = legs[("fp64_local", args.h_thrs)]
    mixed_lin = legs[("mixed_linear", args.h_thrs)]
    mixed_quad = legs[("mixed_quadratic", args.h_thrs)]
    # phase timers (events around every stage) on separate runs at the paper threshold
    log("profiled runs at the paper threshold")
    prof_plain = run_leg(rt, torch, sa, s, args, rt.RT_FP64, rt.RT_HUPDATE_FULL, args.h_thrs, args.dp_thrs, True)
    prof_plain["ses"].close()
    prof_fp64_local = run_leg(rt, torch, sa, s, args, rt.RT_FP64, rt.RT_HUPDATE_LOCAL, args.h_thrs, args.dp_thrs,
                              True)
    prof_fp64_local["ses"].close()
    # the mixed profile runs the quadratic first guess: one Hamiltonian update per step
    # at the paper's threshold, so every density and projection launch carries all
    # three trajectories (the roofline's per-launch work)
    prof_mixed = run_leg(rt, torch, sa, s, args, rt.RT_MIXED, rt.RT_HUPDATE_LOCAL, args.h_thrs, args.dp_thrs, True,
                         predictor=rt.RT_PRED_QUADRATIC)
    ctx = prof_mixed["ses"].ctx
    tuned = {} if args.no_tune else {
        k: rt.rt_tune_get(ctx, 0, v) for k, v in (("stencil_fp64", rt.RT_TUNE_STENCIL_FP64),
                                                   ("stencil_fp32", rt.RT_TUNE_STENCIL_FP32),
                                                   ("projection_bf16x3", rt.RT_TUNE_PROJ_MIXED))}

    def dip_err(leg):
        d = leg["mu"] - leg["mu"][0]
        dr = ref["mu"] - ref["mu"][0]
        return float(np.max(np.abs(d - dr)) / np.max(np.abs(dr)))

    # standalone H-apply rates (FP64 and FP32 stencil + nonlocal over all orbitals)
    x64 = psi
    y64 = torch.empty_like(x64)
    x32 = x64.float()
    y32 = torch.empty_like(x32)
    rates = {}
    for dt_, (x, y) in ((0, (x64, y64)), (1, (x32, y32))):
        for _ in range(2):
            rt.rt_apply_h(ctx, 0, x.data_ptr(), y.data_ptr(), N, dt_)
        torch.cuda.synchronize()
        rt.rt_profile(ctx, enable=True, reset=True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        ev0.record()
        for _ in range(reps):
            rt.rt_apply_h(ctx, 0, x.data_ptr(), y.data_ptr(), N, dt_)
        ev1.record()
        torch.cuda.synchronize()
        ph = rt.rt_profile_read(ctx)
        rt.rt_profile(ctx, enable=False, reset=True)
        t_apply = ev0.elapsed_time(ev1) / 1e3 / reps
        b = 4 if dt_ else 8
        st_ms, st_n = ph["stencil_fd8"]
        t_st = st_ms / 1e3 / st_n  # one stencil launch covers all N orbitals
        st_bytes = 2 * b * N * s.ng + b * s.ng  # psi in, H psi out, V once
        tiling = rt.rt_tune_get(ctx, 0, rt.RT_TUNE_STENCIL_FP32 if dt_ else rt.RT_TUNE_STENCIL_FP64)
        rates["fp32" if dt_ else "fp64"] = {
            "orbital_gridpoints_per_s": N * s.ng / t_apply,
            "hbm_GBps_algorithmic": (2 * b * N * s.ng + b * s.ng) / t_apply / 1e9,
            "hbm_frac": (2 * b * N * s.ng + b * s.ng) / t_apply / PEAK_HBM,
            "stencil_only": {"avg_launch_us": t_st * 1e6, "algorithmic_bytes_per_launch": st_bytes,
                             "achieved_GBps": st_bytes / t_st / 1e9, "frac": st_bytes / t_st / PEAK_HBM,
                             # counted at one tiling; another one re-reads other halo rows
                             "traffic": measured_traffic("stencil_fd8_fp32" if dt_ else "stencil_fd8_fp64",
                                                         st_bytes, tiling),
                             "tiling": tiling},
        }
    prof_mixed["ses"].close()
    del x64, y64, x32, y32

    def summary(leg, mixed_mode, full, prof_leg):
        m_total = sum(x[0] for x in leg["stats"])
        return {
            "steps_per_s": args.steps / leg["elapsed"], "ms_per_step": 1e3 * leg["elapsed"] / args.steps,
            "trajectory_steps_per_s": len(AXES) * args.steps / leg["elapsed"],
            "mean_scf_updates_per_step": m_total / len(leg["stats"]),
            "mean_series_terms_per_update": sum(x[1] for x in leg["stats"]) / max(1, m_total),
            "hamiltonian_updates_per_s": m_total / leg["elapsed"],
            # only the full update applies the grid Hamiltonian to every orbital
            **({"h_applies_orbital_gridpoints_per_s": m_total * N * s.ng / leg["elapsed"]} if full else
               {"h_applies_orbital_gridpoints_per_s": None,
                "h_applies_note": "H[P] = H_gs + h^3 Psi^T dV Psi: no grid H apply inside the step"}),
            "dipole_rel_err_vs_fp64_tight": dip_err(leg),
            "energy_change_err_vs_fp64_tight": float(np.max(np.abs((leg["E"] - leg["E"][0]) - (ref["E"] - ref["E"][0])))),
            "roofline": roofline_of(prof_leg["prof"], N, s.ng, mixed_mode, full),
            "phases_ms": {k: round(v[0], 3) for k, v in prof_leg["prof"].items() if v[1]},
            "phases_note": "phase timers from a separate run with events around every stage",
        }

    sm_plain = summary(plain, False, True, prof_plain)
    sm_fp64_local = summary(fp64_local, False, False, prof_fp64_local)
    sm_mixed_lin = summary(mixed_lin, True, False, prof_mixed)
    sm_mixed_quad = summary(mixed_quad, True, False, prof_mixed)
    sweep = []
    for (mname, th), leg in legs.items():
        m_total = sum(x[0] for x in leg["stats"])
        sweep.append({"method": mname, "h_thrs": th, "steps_per_s": args.steps / leg["elapsed"],
                      "updates_per_step": m_total / len(leg["stats"]), "dipole_rel_err": dip_err(leg)})
    # headline: the fastest mixed configuration (either first guess, any swept threshold)
    # whose dipole error is within 3x of the plain FP64 step's at the paper's threshold
    e_ref = sm_plain["dipole_rel_err_vs_fp64_tight"]
    ok = [r for r in sweep if r["method"].startswith("mixed") and r["dipole_rel_err"] <= 3 * e_ref]
    head = max(ok, key=lambda r: r["steps_per_s"]) if ok else \
        {"method": "mixed_linear", "h_thrs": args.h_thrs, "steps_per_s": sm_mixed_lin["steps_per_s"]}
    value = head["steps_per_s"]
    # plain FP64 at matched error: the fastest plain point whose error is at most the headline's
    plain_ok = [r for r in sweep if r["method"] == "plain_fp64" and r["dipole_rel_err"] <= max(
        e_ref, head.get("dipole_rel_err", e_ref))]
    plain_match = max(plain_ok, key=lambda r: r["steps_per_s"]) if plain_ok else None
    best = sm_mixed_quad
    # Pareto view: for each mixed sweep point, the fastest plain point whose error is no
    # larger (10 % slack for equal errors), and the speedup over it
    pareto = []
    for r in sweep:
        if not r["method"].startswith("mixed"):
            continue
        pl = [q for q in sweep if q["method"] == "plain_fp64" and q["dipole_rel_err"] <= 1.1 * r["dipole_rel_err"]]
        if pl:
            q = max(pl, key=lambda q: q["steps_per_s"])
            pareto.append({"method": r["method"], "h_thrs": r["h_thrs"], "dipole_rel_err": r["dipole_rel_err"],
                           "speedup_vs_plain_at_no_larger_error": r["steps_per_s"] / q["steps_per_s"],
                           "plain_h_thrs": q["h_thrs"]})
    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 / value, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3+f64", "data": "synthetic",
        "config": {"workload": f"{name}: 96^3 h=0.3, 40 Gaussian wells + rank-4 projectors (r_c=2), "
                               f"N=240 (160 occ + 80 virt), x/y/z kick trajectories stepped together, dt=0.05, "
                               f"H_thrs={args.h_thrs:g}, dP_thrs={args.dp_thrs:g}; mixed BF16x3 "
                               f"perturbation contractions + FP64 series/Poisson/LDA/observables; headline "
                               f"{head['method']} at H_thrs={head['h_thrs']:g}",
                   "grid": list(s.n), "n_orb": N, "trajectories": len(AXES)},
        "vs_plain_fp64": value / sm_plain["steps_per_s"],
        "vs_fp64_local_update": value / sm_fp64_local["steps_per_s"],
        "vs_plain_fp64_matched_error": (value / plain_match["steps_per_s"]) if plain_match else None,
        "roofline": best["roofline"],
        "equal_dipole_err_rule": "headline: fastest mixed sweep point whose dipole error is within 3x of "
                                 "the plain FP64 step's at the paper threshold",
        "headline": head, "sweep": sweep, "pareto_vs_plain": pareto,
        "mixed": sm_mixed_lin, "mixed_quadratic": sm_mixed_quad, "plain_fp64": sm_plain,
        "fp64_local_update": sm_fp64_local,
        "fp64_tight_reference_steps_per_s": args.steps / ref["elapsed"],
        "apply_h_standalone": rates,
        "autotuned_launch_shapes": tuned,
    }
    out["ground_state"] = gs_info
    log("no-kick control")
    out["no_kick_control"] = no_kick_control(rt, torch, sa)
    if not args.no_batch:
        log("batched: 16 molecules x 3 kicks in one context vs 16 contexts")
        out["batched_16_molecules"] = batched_molecules(rt, torch, args.steps, args.warmup, tune=not args.no_tune)
    if not args.no_variants:
        log("variants: non-orthogonal basis, fourth-order Magnus, pulses")
        out["variants_96"] = variants(rt, torch, s, psi, args)
    if not args.no_192:
        log("FP32 H apply, 192^3 x 3000 orbitals")
        out["apply_h_192"] = apply_h_192(rt, torch, tune=not args.no_tune)
    if not args.no_learned:
        log("learned predictor: record, train, evaluate")
        out["learned_predictor_96"] = learned_predictor(rt, torch, sa, s)
    if not args.no_ground_state:
        log("ground states of the 16 batch molecules on the GPU")
        out["ground_state_16_molecules"] = ground_states(rt, torch)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(s, psi.cpu().numpy(), sm_plain["mean_scf_updates_per_step"], 0.05,
                                           len(AXES))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
