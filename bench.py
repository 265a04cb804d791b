"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over the workload: assemble C and r
(node sampling, collocation, batched LU, back substitution, knot evaluation,
Monte Carlo perimeter rows, boundary rows), solve C u = r, solve
C^T lambda = dL/du and the adjoint with respect to the node samples, for the
loss sum_i (u_i - u_target_i)^2.

Workload: the variable-coefficient configuration (32 x 32 circles of radius
0.045 on the unit square, M = Ntheta = 64, Nr = 16, 10^4 paths per perimeter
knot, h = 1e-4), synthetic seeded inputs.

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


def lu_flops(n, nrhs):
    """Algorithmic flops of one unit (one circle) of the LU launch: factorisation
    of the n x n collocation matrix (2/3 n^3), forward elimination of its nrhs
    right-hand sides (n^2 nrhs) and their back substitution (n^2 nrhs)."""
    return 2.0 / 3.0 * n ** 3 + 2.0 * n * n * nrhs


def run_gpu(cfg, steps, warmup, with_adjoint=True):
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
    noise = workloads.target_noise({"noise_seed": 20, "noise_std": 1e-3}, cover.N)
    target = pdd.eval_field(prob, "u", xy_d) + torch.tensor(noise, dtype=torch.float64, device=dev)

    def step():
        sysm = pdd.System(cover, prob, cfg["mc"], keep_factors=with_adjoint)
        res = {"stats": sysm.stats}
        if with_adjoint:
            u, si = sysm.solve()
            g = 2.0 * (u - target)
            lam, si_t = sysm.solve(rhs=g, transpose=True)
            grads = sysm.backward(u, lam)
            res.update(iters=si.iterations, iters_t=si_t.iterations, rel=si.rel_residual)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the assembly would shard).", file=sys.stderr)
        sys.exit(2)

    import workloads
    cfg = workloads.config2()
    with_adj = not args.no_adjoint
    cover, results, dt, t_cover = run_gpu(cfg, args.steps, args.warmup, with_adjoint=with_adj)
    info = cover.info
    st = [r["stats"] for r in results]
    n_circles = int(info.n_circles)
    n_float = int(info.n_float)
    ms_lu = sum(s.ms_lu for s in st) / len(st)
    ms_spec = sum(s.ms_build + s.ms_lu + s.ms_solve + s.ms_eval for s in st) / len(st)
    ms_mc = sum(s.ms_mc for s in st) / len(st)
    ms_asm = sum(s.ms_total for s in st) / len(st)
    path_steps = st[-1].path_steps
    n = 16 * 64
    nrhs = 65
    flops = lu_flops(n, nrhs) * n_float
    achieved = flops / (ms_lu * 1e-3) / 1e12
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
            "workload": "variable-coefficient operator on the unit square, 32x32 circles r=0.045, "
                        "M=Ntheta=64, Nr=16 (n=1024), 1e4 paths/perimeter knot, h=1e-4",
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
        "roofline": {
            "bound": "mfma",
            "kernel": "batched LU + triangular solves of 900 circles (n=1024, 65 right-hand sides): "
                      "lu_panel/lu_urow/lu_update/lu_bdiag/lu_bupd kernels, 38 launches",
            "achieved": achieved, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_MFMA_TFLOPS, "traffic": None,
        },
    }
    if with_adj:
        out["solve_iterations"] = results[-1]["iters"]
        out["solve_iterations_transpose"] = results[-1]["iters_t"]
    if not args.no_cpu_baseline:
        cb = cpu_baseline(cfg, args.cpu_budget)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline_detail"] = {k: cb[k] for k in ("s_per_floating_circle", "s_per_mc_knot",
                                                         "mc_path_steps_per_s")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
