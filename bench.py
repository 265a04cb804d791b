"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over the workload: assemble C and r
(node sampling, collocation, batched LU, back substitution, knot evaluation,
Monte Carlo perimeter rows, boundary rows), solve C u = r, solve
C^T lambda = dL/du and the adjoint with respect to the node samples, for the
loss sum_i (u_i - u_target_i)^2.

Default workload: the variable-coefficient configuration (32 x 32 circles of
radius 0.045 on the unit square, M = Ntheta = 64, Nr = 16, 10^4 paths per
perimeter knot, h = 1e-4), synthetic seeded inputs.  --workload selects the
uneven-resolution (assembly only; --per-circle adds the plain per-circle loop
on a reduced cover), differentiation and scale workloads.

Prints one JSON line (rank 0).  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


# HBM bytes of one LU phase (all LU launches of a step), from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE) over this script, each scaled by what the counter reads for a
# copy of known size: profiles/hbm_traffic_lu_32x32_n1024.md.  Valid for the kernels the
# counters were taken on; a changed LU kernel needs a new pass (else None).
LU_TRAFFIC_BYTES = {"config2": 1.081e11}


def lu_flops(n, nrhs):
    """Algorithmic flops of one unit (one circle) of the LU launch: factorisation
    of the n x n collocation matrix (2/3 n^3), forward elimination of its nrhs
    right-hand sides (n^2 nrhs) and their back substitution (n^2 nrhs)."""
    return 2.0 / 3.0 * n ** 3 + 2.0 * n * n * nrhs


def run_gpu(cfg, steps, warmup, with_adjoint=True, budget=0, plan="batched"):
    import numpy as np
    import torch

    import paper_2311_08946_amd.binding as pdd
    import workloads

    torch.cuda.set_device(0)
    prob = cfg["problem"]
    t0 = time.perf_counter()
    cover = pdd.Cover(prob["domain"], cfg["cover"])
    t_cover = time.perf_counter() - t0
    info = cover.info
    dev = torch.device("cuda", 0)
    xy, rc, asg, own = cover.knots()
    # loss target: the manufactured solution at the knots plus N(0, 1e-3) noise
    xy_d = torch.tensor(xy, dtype=torch.float64, device=dev)
    noise = workloads.target_noise({"noise_seed": cfg.get("noise_seed", 20),
                                    "noise_std": cfg.get("noise_std", 1e-3)}, cover.N)
    exact = pdd.eval_field(prob, "u", xy_d)
    target = exact + torch.tensor(noise, dtype=torch.float64, device=dev)

    def step():
        sysm = pdd.System(cover, prob, cfg["mc"], keep_factors=with_adjoint, hbm_budget_bytes=budget,
                          plan=plan)
        res = {"stats": sysm.stats}
        if with_adjoint:
            u, si = sysm.solve()
            g = 2.0 * (u - target)
            lam, si_t = sysm.solve(rhs=g, transpose=True)
            grads = sysm.backward(u, lam)
            res.update(iters=si.iterations, iters_t=si_t.iterations, rel=si.rel_residual,
                       rms=float(torch.sqrt(torch.mean((u - exact) ** 2))))
        return res

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return cover, results, dt, t_cover


def cpu_baseline(cfg, budget_s=20.0):
    """The oracle, single-threaded, on a bounded sample of the same workload:
    a few floating circles and a few Monte Carlo knots, extrapolated to the
    whole cover."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import geometry, montecarlo, spectral
    from oracle.geometry import ROW_MC

    prob = cfg["problem"]
    with threadpool_limits(1):
        cv = geometry.build_cover(prob["domain"], cfg["cover"])
        fl = np.nonzero(cv.floating)[0]
        mck = np.nonzero(cv.row_class == ROW_MC)[0]
        rng = np.random.default_rng(0)
        spectral.local_grid(cv.Nr[fl[0]], cv.Ntheta[fl[0]])   # grid tables are shared setup
        t0 = time.perf_counter()
        n_c = 0
        for m in rng.permutation(fl):
            spectral.floating_rows(prob, cv, m)
            n_c += 1
            if time.perf_counter() - t0 > budget_s / 2:
                break
        t_spec = (time.perf_counter() - t0) / n_c
        t0 = time.perf_counter()
        n_k = 0
        steps = 0
        for i in rng.permutation(mck):
            _, _, _, _, _, st = montecarlo.mc_rows(prob, cv, cfg["mc"], [i])
            steps += st
            n_k += 1
            if time.perf_counter() - t0 > budget_s / 2:
                break
        t_mc = (time.perf_counter() - t0) / n_k
    t_total = t_spec * len(fl) + t_mc * len(mck)
    return {
        "value": len(cv.radii) / t_total,
        "unit": "circles/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n_c} of {len(fl)} floating circles and {n_k} of {len(mck)} Monte Carlo knots "
                  f"(full paths each), extrapolated linearly; assembly only",
        "s_per_floating_circle": t_spec,
        "s_per_mc_knot": t_mc,
        "mc_path_steps_per_s": steps / (t_mc * n_k),
    }


WORKLOADS = {
    "config2": dict(adjoint=True, budget=0,
                    label="variable-coefficient operator on the unit square, 32x32 circles r=0.045, "
                          "M=Ntheta=64, Nr=16 (n=1024), 1e4 paths/perimeter knot, h=1e-4"),
    "config3": dict(adjoint=False, budget=0,
                    label="Laplace on the unit disk minus a hole, ~2e4 circles of uneven radius, "
                          "Ntheta in {32,48,64,96,128}, Nr=Ntheta/4 (n=256..4096), 1e3 paths/knot"),
    "config4": dict(adjoint=True, budget=0,
                    label="Laplace base point on a 64x64 cover, M=Ntheta=64, Nr=16 (n=1024), "
                          "1e3 paths/knot, h=8.1e-6; loss sum (u - u_target)^2"),
    "config5": dict(adjoint=True, budget=8 << 30,
                    label="Laplace on a 128x128 cover, M=64, Ntheta=48, Nr=12 (n=576), 1e5 paths/knot, "
                          "h=1e-5; LU factors recomputed in chunks under an 8 GiB budget"),
    "paper50": dict(adjoint=True, budget=0,
                    label="Section 4 test problem: Poisson with the exact solution of eq. 46 on [-50,50]^2, "
                          "10x10 circles r in [8.55, 9.43], M=Ntheta=44, Nr=22 (n=968), c^2=1.5, "
                          "5000 paths/perimeter knot, h=0.015 (plain Euler)"),
    "paper50_gm": dict(adjoint=True, budget=0,
                       label="Section 4 test problem as run in the paper: eq. 46 on [-50,50]^2, 10x10 circles, "
                             "M=Ntheta=44, Nr=22, averaged rows (eqs. 38-39), boundary-shifted Euler, "
                             "5000 paths/perimeter knot, h=0.015"),
}


def spectral_flops(cover, cfg):
    """Algorithmic LU flops of all floating circles of the cover."""
    import numpy as np
    _, off, ids = cover.nodes()
    n = np.diff(off).astype(np.float64)
    M = np.asarray(cfg["cover"]["M"], dtype=np.float64)[ids]
    return float(np.sum(2.0 / 3.0 * n ** 3 + 2.0 * n * n * (M + 1)))


def per_circle_comparison(steps):
    """The plain per-circle loop (same kernels, one launch sequence per circle)
    against the batched plan, on a reduced uneven-resolution cover (lattice
    spacing 0.055 instead of 0.0123: about 1e3 circles with the same
    resolution draw), assembly only."""
    import workloads
    cfg = workloads.config3(spacing=0.055)
    out = {}
    for plan in ("batched", "per_circle"):
        cover, results, dt, _ = run_gpu(cfg, steps, 1, with_adjoint=False, plan=plan)
        st = [r["stats"] for r in results]
        out[plan] = {"ms_assembly": sum(s.ms_total for s in st) / len(st),
                     "ms_lu": sum(s.ms_lu for s in st) / len(st),
                     "launches": int(st[-1].n_launch_spectral)}
    out["circles"] = int(cover.info.n_circles)
    out["floating"] = int(cover.info.n_float)
    out["speedup"] = out["per_circle"]["ms_assembly"] / out["batched"]["ms_assembly"]
    return out


def ras_measurement(cfg, parts, reps):
    """GMRES with the one-level RAS preconditioner (eqs. 42-45) on an assembled
    system of the workload: set-up time, iterations and time of the solve
    beside BiCGStab and plain GMRES, and the preconditioner apply against HBM
    bandwidth (its GEMV reads every stored inverse once)."""
    import numpy as np
    import torch

    import paper_2311_08946_amd.binding as pdd

    torch.cuda.set_device(0)
    prob = cfg["problem"]
    cover = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cover, prob, cfg["mc"])

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3

    R, ms_build = timed(lambda: pdd.Ras(sysm, *parts))
    sizes = np.array([len(w) for w in R.parts()], dtype=np.float64)
    out = {"parts": [int(parts[0]), int(parts[1])], "n_parts": len(sizes),
           "max_part": int(sizes.max()), "setup_ms": ms_build}
    for name, fn in (("gmres_ras", lambda: sysm.solve_gmres(R, rtol=1e-12)),
                     ("gmres", lambda: sysm.solve_gmres(None, rtol=1e-12)),
                     ("bicgstab", lambda: sysm.solve(rtol=1e-12))):
        fn()
        (u, info), ms = timed(fn)
        out[name] = {"ms": ms, "iterations": int(info.iterations), "converged": bool(info.converged)}
    x = torch.randn(cover.N, dtype=torch.float64, device="cuda")
    for _ in range(3):
        R.apply(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        R.apply(x)
    e1.record()
    torch.cuda.synchronize()
    ms_apply = e0.elapsed_time(e1) / reps
    # algorithmic bytes of one apply: the inverses (n_p^2 doubles each), the
    # gathered x and the written block results
    nbytes = float(np.sum(8.0 * sizes * sizes + 16.0 * sizes))
    achieved = nbytes / (ms_apply * 1e-3) / 1e9
    out["apply_ms"] = ms_apply
    out["apply_roofline"] = {"bound": "hbm", "kernel": "gather_x_kernel + block_gemv_kernel + combine_kernel",
                             "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "frac": achieved / PEAK_HBM_GBS, "bytes_per_apply": nbytes}
    # the same with the inverses kept in FP32
    del R
    R32, ms_b32 = timed(lambda: pdd.Ras(sysm, *parts, fp32_inverses=True))
    sysm.solve_gmres(R32, rtol=1e-12)
    (u, info), ms = timed(lambda: sysm.solve_gmres(R32, rtol=1e-12))
    out["fp32_inverses"] = {"setup_ms": ms_b32, "gmres_ras": {"ms": ms, "iterations": int(info.iterations),
                                                               "converged": bool(info.converged)}}
    for _ in range(3):
        R32.apply(x)
    e0.record()
    for _ in range(reps):
        R32.apply(x)
    e1.record()
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1) / reps
    nbytes32 = float(np.sum(4.0 * sizes * sizes + 16.0 * sizes))
    a32 = nbytes32 / (ms32 * 1e-3) / 1e9
    out["fp32_inverses"]["apply_ms"] = ms32
    out["fp32_inverses"]["apply_roofline"] = {
        "bound": "hbm", "kernel": "gather_x_kernel + block_gemv_f32_kernel + combine_kernel",
        "achieved": a32, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": a32 / PEAK_HBM_GBS,
        "bytes_per_apply": nbytes32}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="config2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--per-circle", action="store_true",
                    help="also time the plain per-circle loop on a reduced uneven cover")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer 4 times (calibrates HBM byte counters)")
    ap.add_argument("--ras", default=None, metavar="PXxPY",
                    help="instead of the step, measure GMRES with the RAS preconditioner of PXxPY parts")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 8, "launches": 4}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; the "
              "assembly would shard by spatial blocks of circles with a halo exchange in the solve.",
              file=sys.stderr)
        sys.exit(2)

    import workloads
    wl = WORKLOADS[args.workload]
    cfg = workloads.CONFIGS[args.workload]()
    if args.ras:
        px, py = (int(v) for v in args.ras.lower().split("x"))
        res = ras_measurement(cfg, (px, py), max(10, args.steps * 20))
        print(json.dumps({"metric": "GMRES+RAS solve of C u = r (ms)", "value": res["gmres_ras"]["ms"],
                          "unit": "ms", "n_gpus": 1, "higher_is_better": False, "dtype": "f64",
                          "data": "synthetic", "config": {"workload": wl["label"]}, "ras": res}),
              flush=True)
        return
    with_adj = wl["adjoint"] and not args.no_adjoint
    cover, results, dt, t_cover = run_gpu(cfg, args.steps, args.warmup, with_adjoint=with_adj,
                                          budget=wl["budget"])
    info = cover.info
    st = [r["stats"] for r in results]
    n_circles = int(info.n_circles)
    n_float = int(info.n_float)
    ms_lu = sum(s.ms_lu for s in st) / len(st)
    ms_spec = sum(s.ms_build + s.ms_lu + s.ms_solve + s.ms_eval for s in st) / len(st)
    ms_mc = sum(s.ms_mc for s in st) / len(st)
    ms_asm = sum(s.ms_total for s in st) / len(st)
    path_steps = st[-1].path_steps
    flops = spectral_flops(cover, cfg)
    achieved = flops / (ms_lu * 1e-3) / 1e12
    kernels = "lu_pupd/lu_panel/lu_urow (interchanges + L11^-1, first tile, other tiles)/lu_bdiag/lu_bupd kernels"
    if args.workload == "config2":
        kernel = ("batched LU + triangular solves of 900 circles (n=1024, 65 right-hand sides): "
                  + kernels + ", 53 launches per step on two streams")
    else:
        kernel = f"batched LU + triangular solves of {n_float} circles: " + kernels
    out = {
        "metric": "G assembly circles/s + MC path-steps/s at fixed error; fwd+adjoint seconds",
        "value": n_circles / dt,
        "unit": "circles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": wl["label"],
            "circles": n_circles, "floating": n_float, "N": int(info.N), "nnz": int(info.nnz),
            "step": "assemble + solve + transpose solve + adjoint" if with_adj else "assemble",
        },
        "assembly_ms": ms_asm,
        "assembly_circles_per_s": n_circles / (ms_asm * 1e-3),
        "spectral_circles_per_s": n_float / (ms_spec * 1e-3),
        "mc_path_steps_per_s": path_steps / (ms_mc * 1e-3) if ms_mc > 0 else None,
        "mc_paths_per_s": st[-1].paths / (ms_mc * 1e-3) if ms_mc > 0 else None,
        "fwd_adjoint_s": dt if with_adj else None,
        "phase_ms": {k: sum(getattr(s, "ms_" + k) for s in st) / len(st)
                     for k in ("sample", "build", "lu", "solve", "eval", "mc", "total")},
        "build_cover_s": t_cover,
        "factor_bytes_kept": int(st[-1].factor_bytes),
        "factors_recomputed_in_backward": bool(st[-1].recompute),
        "roofline": {
            "bound": "mfma",
            "kernel": kernel,
            "achieved": achieved, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_MFMA_TFLOPS,
            "traffic": LU_TRAFFIC_BYTES.get(args.workload),
            "traffic_unit": "HBM bytes per LU phase (one step), rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0",
        },
    }
    if with_adj:
        out["solve_iterations"] = results[-1]["iters"]
        out["solve_iterations_transpose"] = results[-1]["iters_t"]
        out["rms_error_vs_exact"] = results[-1]["rms"]
    if args.per_circle:
        out["per_circle_vs_batched"] = per_circle_comparison(max(1, min(args.steps, 2)))
    if not args.no_cpu_baseline:
        cb = cpu_baseline(cfg, args.cpu_budget)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline_detail"] = {k: cb[k] for k in ("s_per_floating_circle", "s_per_mc_knot",
                                                         "mc_path_steps_per_s")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
