"""Throughput of the RT-TDDFT time step on one MI355X.

Workload (default): the plain-vs-mixed molecule -- 96^3 periodic grid, h = 0.3
bohr, 40 Gaussian wells with rank-4 separable projectors (r_c = 2 bohr),
160 occupied + 80 virtual orbitals, delta kick 1e-3 along x, dt = 0.05 a.u.,
self-consistency and series thresholds of the paper (1e-7, 1e-10).  Inputs are
seeded synthetic: smooth random orbitals made orthonormal by the library's own
basis transform at init (the ground-state solve is not part of the step).

One "step" = one time step of Algorithm 1 for the trajectory: linear
predictor, Hamiltonian self-consistency loop (commutator-series propagation,
density, FFT Hartree, LDA exchange, H applied to every orbital and projected),
observables.  All inputs are resident in HBM before the timed region.

Prints one JSON line.  `--gpus N` with N > 1 exits: this build runs on one GPU.
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


def roof(phase, N, ng, mixed):
    """Algorithmic bytes and flops of one launch of a phase, and the matrix
    peak that applies.  BF16x3 contractions execute three bf16 products per
    FP product on the matrix cores."""
    pairs = float(N) * (N + 1) / 2  # unique entries of a symmetric N x N result / pair products
    if phase == "project_gemm":
        if mixed:
            return 4.0 * N * ng + 4.0 * ng, 3 * 2 * pairs * ng, PEAK_BF16
        return 16.0 * N * ng, 2 * pairs * ng, PEAK_FP64
    if phase == "density":
        if mixed:
            return 4.0 * N * ng + 16.0 * ng, 3 * 2 * pairs * ng, PEAK_BF16
        return 8.0 * N * ng + 8.0 * ng, 2 * pairs * ng, PEAK_FP64
    if phase == "series_gemm":
        return 3 * 16.0 * N * N, 4.0 * N ** 3, PEAK_FP64
    if phase == "stencil_fd8":
        return 16.0 * N * ng + 8.0 * ng, 0.0, PEAK_FP64
    return None


def cpu_baseline(s, psi_host, m_mean, dt):
    """The oracle on the host's cores: one self-consistent Hamiltonian update
    (exact exponential of Hbar + H[P]) of the same workload, timed once."""
    import oracle
    from oracle import propagate

    try:
        from threadpoolctl import threadpool_info

        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    N = psi_host.shape[0]
    log("cpu baseline: building oracle model")
    m = oracle.Model(s, psi_host)
    P = np.diag(s.occupations()).astype(np.complex128)
    H, _ = m.h_of_p(P)
    t0 = time.perf_counter()
    P1 = propagate.propagate_exact(H, P, dt)
    H1, _ = m.h_of_p(P1)
    t_update = time.perf_counter() - t0
    t0 = time.perf_counter()
    m.apply_h(m.psi[: min(N, 16)], m.vion)
    t_apply = (time.perf_counter() - t0) / min(N, 16)
    steps_per_s = 1.0 / (t_update * m_mean)
    return {
        "value": steps_per_s, "unit": "steps/s", "cores": int(cores), "kind": "oracle",
        "sample": f"one self-consistent Hamiltonian update of the same {s.n[0]}^3 N={N} workload "
                  f"({t_update:.2f} s), scaled by the GPU run's mean {m_mean:.2f} updates per step",
        "h_applies_per_s": s.ng / t_apply,
    }


def run_leg(rt, torch, sa, s, args, precision, hupdate, h_thrs, dp_thrs, profile):
    total = args.warmup + args.steps
    ra = rt.RunArgs(dt=0.05, n_steps_max=total, h_thrs=h_thrs, dp_thrs=dp_thrs, max_scf=50, max_terms=200,
                    traj_sys=[0], traj_kappa=[1e-3], traj_axis=[0], hupdate=hupdate, precision=precision)
    ses = rt.Session([sa], ra)
    ctx = ses.ctx
    rt.rt_step(ctx, args.warmup, n_traj=1, stats=False)
    torch.cuda.synchronize()
    if profile:
        rt.rt_profile(ctx, enable=True, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = rt.rt_step(ctx, args.steps, n_traj=1, stats=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = rt.rt_profile_read(ctx) if profile else None
    mu, E, tr = rt.rt_dipole(ctx, 0, 0, total + 1)
    leg = dict(elapsed=elapsed, stats=stats, prof=prof, mu=mu, E=E, tr=tr, ses=ses)
    return leg


def roofline_of(prof, N, ng, mixed):
    cands = [k for k in prof if prof[k][1] and roof(k, N, ng, mixed)]
    dom = max(cands, key=lambda k: prof[k][0])
    nbytes, flops, pk = roof(dom, N, ng, mixed)
    ms, launches = prof[dom]
    avg = ms / 1e3 / launches
    t_hbm, t_mfma = nbytes / PEAK_HBM, (flops / pk if flops else 0.0)
    if t_hbm >= t_mfma:
        return {"bound": "hbm", "kernel": dom, "achieved": nbytes / avg / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": nbytes / avg / PEAK_HBM, "traffic": None, "avg_launch_us": avg * 1e6,
                "algorithmic_bytes_per_launch": nbytes}
    return {"bound": "mfma", "kernel": dom, "achieved": flops / avg / 1e12, "peak": pk / 1e12,
            "unit": "TFLOP/s", "frac": flops / avg / pk, "traffic": None, "avg_launch_us": avg * 1e6,
            "algorithmic_flops_per_launch": flops}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--h-thrs", type=float, default=1e-7)
    ap.add_argument("--dp-thrs", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU (no multi-GPU path); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2410_09189_amd import rt

    name = "c2_mixed_96"
    s = synth.config_system(name)
    N = s.n_orb
    log(f"generating {N} smooth random orbitals on {s.n}")
    psi = synth.lowpass_orbitals(s.n, s.h, N, seed=s.seed)
    sa = rt.SystemArgs(n=s.n, h=s.h, pos=s.pos, depth=s.depth, width=s.width, n_occ=s.n_occ,
                       n_virt=s.n_virt, psi0=psi, nl_rank=s.nl_rank, nl_rcut=s.nl_rcut,
                       nl_sigma=s.nl_sigma, nl_D=s.nl_D, n_images=s.n_images, orthonormalize=True)
    log("leg 1/3: FP64 reference, tight thresholds (1e-12, 1e-15)")
    ref = run_leg(rt, torch, sa, s, args, rt.RT_FP64, rt.RT_HUPDATE_FULL, 1e-12, 1e-15, False)
    ref["ses"].close()
    log("leg 2/3: plain FP64, full Hamiltonian apply, paper thresholds")
    plain = run_leg(rt, torch, sa, s, args, rt.RT_FP64, rt.RT_HUPDATE_FULL, args.h_thrs, args.dp_thrs, True)
    plain["ses"].close()
    log("leg 3/3: mixed BF16x3 + FP64, paper thresholds")
    mixed = run_leg(rt, torch, sa, s, args, rt.RT_MIXED, rt.RT_HUPDATE_LOCAL, args.h_thrs, args.dp_thrs, True)
    ctx = mixed["ses"].ctx

    def dip_err(leg):
        d = leg["mu"][:, 0] - leg["mu"][0, 0]
        dr = ref["mu"][:, 0] - ref["mu"][0, 0]
        return float(np.max(np.abs(d - dr)) / np.max(np.abs(dr)))

    # standalone H-apply rates (FP64 and FP32 stencil + nonlocal over all orbitals)
    x64 = torch.from_numpy(psi.reshape(N, -1)).cuda()
    y64 = torch.empty_like(x64)
    x32 = x64.float()
    y32 = torch.empty_like(x32)
    rates = {}
    for dt_, (x, y) in ((0, (x64, y64)), (1, (x32, y32))):
        for _ in range(2):
            rt.rt_apply_h(ctx, 0, x.data_ptr(), y.data_ptr(), N, dt_)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        ev0.record()
        for _ in range(reps):
            rt.rt_apply_h(ctx, 0, x.data_ptr(), y.data_ptr(), N, dt_)
        ev1.record()
        torch.cuda.synchronize()
        t_apply = ev0.elapsed_time(ev1) / 1e3 / reps
        b = 4 if dt_ else 8
        rates["fp32" if dt_ else "fp64"] = {
            "orbital_gridpoints_per_s": N * s.ng / t_apply,
            "hbm_GBps_algorithmic": (2 * b * N * s.ng + b * s.ng) / t_apply / 1e9,
            "hbm_frac": (2 * b * N * s.ng + b * s.ng) / t_apply / PEAK_HBM,
        }
    mixed["ses"].close()
    del x64, y64, x32, y32

    def summary(leg, mixed_mode):
        m_total = sum(x[0] for x in leg["stats"])
        return {
            "steps_per_s": args.steps / leg["elapsed"], "ms_per_step": 1e3 * leg["elapsed"] / args.steps,
            "mean_scf_updates_per_step": m_total / len(leg["stats"]),
            "mean_series_terms_per_update": sum(x[1] for x in leg["stats"]) / max(1, m_total),
            "h_updates_orbital_gridpoints_per_s": m_total * N * s.ng / leg["elapsed"],
            "dipole_rel_err_vs_fp64_tight": dip_err(leg),
            "energy_change_err_vs_fp64_tight": float(np.max(np.abs((leg["E"] - leg["E"][0]) - (ref["E"] - ref["E"][0])))),
            "roofline": roofline_of(leg["prof"], N, s.ng, mixed_mode),
            "phases_ms": {k: round(v[0], 3) for k, v in leg["prof"].items() if v[1]},
        }

    sm_plain = summary(plain, False)
    sm_mixed = summary(mixed, True)
    value = sm_mixed["steps_per_s"]
    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sm_mixed["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3+f64", "data": "synthetic",
        "config": {"workload": f"{name}: 96^3 h=0.3, 40 Gaussian wells + rank-4 projectors (r_c=2), "
                               f"N=240 (160 occ + 80 virt), 1 x-kick trajectory, dt=0.05, "
                               f"H_thrs={args.h_thrs:g}, dP_thrs={args.dp_thrs:g}; mixed BF16x3 "
                               f"perturbation contractions + FP64 series/Poisson/LDA/observables",
                   "grid": list(s.n), "n_orb": N, "trajectories": 1},
        "vs_plain_fp64": value / sm_plain["steps_per_s"],
        "roofline": sm_mixed["roofline"],
        "mixed": sm_mixed, "plain_fp64": sm_plain,
        "fp64_tight_reference_steps_per_s": args.steps / ref["elapsed"],
        "apply_h_standalone": rates,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        from scipy.linalg import solve_triangular

        P = psi.reshape(N, -1)
        L = np.linalg.cholesky(s.h ** 3 * (P @ P.T))
        psi_o = solve_triangular(L, P, lower=True)
        del P
        out["cpu_baseline"] = cpu_baseline(s, psi_o, sm_plain["mean_scf_updates_per_step"], 0.05)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
