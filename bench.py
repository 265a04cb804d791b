"""Benchmark of the hot path on one MI355X.

One step = one pass of the whole path over the workload: assemble C and r
(node sampling, collocation, batched LU with the right-hand sides, back
substitution, knot evaluation, Monte Carlo perimeter rows, boundary rows),
solve C u = r, solve C^T lambda = dL/du and the adjoint with respect to the
node samples, for the loss sum_i (u_i - u_target_i)^2.

Default workload: the scale configuration (128 x 128 circles of radius
0.01125 on the unit square, M = 64, Ntheta = 48, Nr = 12 (n = 576), 10^5
paths per perimeter knot, h = 1e-5; Laplace with g = Re p), synthetic seeded
inputs, the autotuned schedule with graph replay.  The LU factors (48 GB)
stay resident for the adjoint; the same step with factors recomputed chunk by
chunk under an 8 GiB budget is reported beside it.  --workload selects the
other configurations.

Prints one JSON line.  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 operations of the Monte Carlo estimator (Appendix eq. 53,
# eqs. 29-30), with an elementary function counted at the operations of a
# plain range-reduction + polynomial evaluation: log 20, exp 20, sin+cos 30,
# atan2 30; sqrt, rsqrt and division 1 each, a fused multiply-add 2.
#   per Euler step: two normals by Box-Muller (log, sqrt, sin+cos, 3 mul) = 54;
#     the update X + b h + sigma sqrt(h) N (2 x 3 FMA) = 12; the circle test
#     (2 sub, 1 mul, 1 FMA, 1 cmp) = 6; the box test (4 cmp) = 4       -> 76
#     with variable coefficients add the fields at X (per SINSUM term: the
#     phase 2 pi (k . x) + phi (2 FMA = 4), sin 20, the product-sum 2 -> 26;
#     a derived source f = -(L u + c u) adds per term of u its sin and cos 30
#     and the six jet sums (6 FMA = 12) -> 46, plus the combination 7 FMA = 14),
#     the Cholesky factor of a (2 sqrt, 1 div, 1 FMA = 5), Y e^{c h} (exp +
#     mul = 21) and Z + f Y h (2 FMA = 4)
#   per exit: segment/circle crossing (about 16 FMA/mul + sqrt + div = 20),
#     exit point and weight (2 FMA = 4), the Z payoff (1 add)            -> 25
#   per exit on Gamma_m: the angle (atan2 30 + unwrap 4), then per arc knot
#     l the IMQ weight Y ((theta - theta_l)^2 + c^2)^-1/2 (1 sub, 1 FMA,
#     1 rsqrt, 1 FMA = 6)                                      -> 34 + 6 n_arc
#   per exit on the boundary: g at the exit (CPOLY_RE of degree 4: 5 complex
#     FMA = 20) times Y (1 mul) and the sum (1 add)                      -> 22
# Philox4x32-10 (about 110 integer operations per step) is not counted.
MC_OPS_STEP_CONST = 76
MC_OPS_STEP_VARIABLE_EXTRA = 5 + 21 + 4
MC_OPS_EXIT = 25
MC_OPS_GAMMA_EXIT = 34
MC_OPS_PER_ARC_KNOT = 6
MC_OPS_BOUNDARY_EXIT = 22


def lu_flops(n, nrhs):
    """Algorithmic flops of one unit (one circle) of the LU launch sequence:
    factorisation of the n x n collocation matrix (2/3 n^3), forward
    elimination of its nrhs right-hand sides (n^2 nrhs) and their back
    substitution (n^2 nrhs)."""
    return 2.0 / 3.0 * n ** 3 + 2.0 * n * n * nrhs


def spectral_flops(cover, cfg):
    """Algorithmic LU flops of all floating circles of the cover."""
    import numpy as np
    _, off, ids = cover.nodes()
    n = np.diff(off).astype(np.float64)
    M = np.asarray(cfg["cover"]["M"], dtype=np.float64)[ids]
    return float(np.sum(lu_flops(n, M + 1)))


def adjoint_bytes(cover, cfg):
    """Algorithmic HBM bytes of one adjoint pass with stored factors: per
    floating circle the LU factors once (8 n^2; both triangular solves read
    them), the solution columns W (8 n (M + 1)), pivots and row scales (12 n)
    and the seven gradient arrays written (56 n); plus u and lambda (16 N)."""
    import numpy as np
    _, off, ids = cover.nodes()
    n = np.diff(off).astype(np.float64)
    M = np.asarray(cfg["cover"]["M"], dtype=np.float64)[ids]
    return float(np.sum(8.0 * n * n + 8.0 * n * (M + 1) + 12.0 * n + 56.0 * n) + 16.0 * cover.N)


def bicgstab_bytes_per_iter(N, nnz):
    """Algorithmic HBM bytes of one BiCGStab iteration: the two products
    with C (or C^T) read every entry once (16 nnz), and each step touches
    every vector it needs once with s = r - alpha v formed on the fly:
    p = r + beta (p - omega v) reads r, p, v and writes p (32 N); v = A p
    reads p and r0, writes v (24 N); t = A s reads r and v, writes t (24 N);
    the x, r update reads r, v, x, p, t, r0 and writes x, r (64 N).
    Index arrays are not counted: the method needs the values, not a
    particular sparse format."""
    return 16.0 * nnz + (32.0 + 24.0 + 24.0 + 64.0) * N


def field_ops_per_point(prob):
    """FP64 operations of evaluating the coefficient fields of eq. 1 at one
    path point (zero for constant coefficients; see the table above)."""
    names = ("axx", "axy", "ayy", "bx", "by", "c")
    if all(prob[k]["kind"] == "const" for k in names) and prob["f"]["kind"] == "const":
        return 0
    ops = 0
    for k in names:
        if prob[k]["kind"] == "sinsum":
            ops += 26 * len(prob[k]["amp"])
    f = prob["f"]
    if f["kind"] == "sinsum":
        ops += 26 * len(f["amp"])
    elif f["kind"] == "derived_f" and f["u"]["kind"] == "sinsum":
        ops += 46 * len(f["u"]["amp"]) + 14
    return ops + MC_OPS_STEP_VARIABLE_EXTRA


def mc_ops(stats, arc_mean, field_ops):
    """Algorithmic FP64 operations of one Monte Carlo phase (see the table at
    the top of this file); field_ops from field_ops_per_point."""
    per_step = MC_OPS_STEP_CONST + field_ops
    gam = float(stats.gamma_exits)
    bnd = float(stats.paths) - gam
    return (per_step * float(stats.path_steps) + MC_OPS_EXIT * float(stats.paths)
            + (MC_OPS_GAMMA_EXIT + MC_OPS_PER_ARC_KNOT * arc_mean) * gam + MC_OPS_BOUNDARY_EXIT * bnd)


WORKLOADS = {
    "config5": dict(adjoint=True, budget=0, chunked_budget=8 << 30,
                    label="Laplace on a 128x128 cover of the unit square, r=0.01125, M=64, Ntheta=48, "
                          "Nr=12 (n=576), 1e5 paths/perimeter knot, h=1e-5; factors resident"),
    "config2": dict(adjoint=True, budget=0,
                    label="variable-coefficient operator on the unit square, 32x32 circles r=0.045, "
                          "M=Ntheta=64, Nr=16 (n=1024), 1e4 paths/perimeter knot, h=1e-4"),
    "config3": dict(adjoint=False, budget=0,
                    label="Laplace on the unit disk minus a hole, ~2e4 circles of uneven radius, "
                          "Ntheta in {32,48,64,96,128}, Nr=Ntheta/4 (n=256..4096), 1e3 paths/knot"),
    "config4": dict(adjoint=True, budget=0,
                    label="Laplace base point on a 64x64 cover, M=Ntheta=64, Nr=16 (n=1024), "
                          "1e3 paths/knot, h=8.1e-6; loss sum (u - u_target)^2"),
    "paper50": dict(adjoint=True, budget=0,
                    label="Section 4 test problem: Poisson with the exact solution of eq. 46 on [-50,50]^2, "
                          "10x10 circles r in [8.55, 9.43], M=Ntheta=44, Nr=22 (n=968), c^2=1.5, "
                          "5000 paths/perimeter knot, h=0.015 (plain Euler)"),
    "paper50_gm": dict(adjoint=True, budget=0,
                       label="Section 4 test problem as run in the paper: eq. 46 on [-50,50]^2, 10x10 circles, "
                             "M=Ntheta=44, Nr=22, averaged rows (eqs. 38-39), boundary-shifted Euler, "
                             "5000 paths/perimeter knot, h=0.015"),
}


# ------------------------------------------------------------------ GPU leg

def run_gpu(cfg, steps, warmup, with_adjoint=True, budget=0, plan="autotuned", use_graph=True):
    """Times `steps` whole steps after `warmup` untimed ones.  Each step records
    torch events around the solves and the adjoint on the stream the library
    runs them on (the current stream); assembly phases come from the library's
    own HIP events (LU on the calling stream, Monte Carlo on its side stream)."""
    import torch

    import paper_2311_08946_amd.binding as pdd
    import workloads

    torch.cuda.set_device(0)
    prob = cfg["problem"]
    t0 = time.perf_counter()
    cover = pdd.Cover(prob["domain"], cfg["cover"])
    t_cover = time.perf_counter() - t0
    dev = torch.device("cuda", 0)
    xy, rc, asg, own = cover.knots()
    # loss target: the manufactured solution at the knots plus N(0, 1e-3) noise
    xy_d = torch.tensor(xy, dtype=torch.float64, device=dev)
    noise = workloads.target_noise({"noise_seed": cfg.get("noise_seed", 20),
                                    "noise_std": cfg.get("noise_std", 1e-3)}, cover.N)
    exact = pdd.eval_field(prob, "u", xy_d)
    target = exact + torch.tensor(noise, dtype=torch.float64, device=dev)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def step():
        sysm = pdd.System(cover, prob, cfg["mc"], keep_factors=with_adjoint, hbm_budget_bytes=budget,
                          plan=plan, use_graph=use_graph)
        res = {"stats": sysm.stats}
        if with_adjoint:
            e = [ev() for _ in range(4)]
            e[0].record()
            u, si = sysm.solve()
            e[1].record()
            g = 2.0 * (u - target)
            lam, si_t = sysm.solve(rhs=g, transpose=True)
            e[2].record()
            grads = sysm.backward(u, lam)
            e[3].record()
            res.update(iters=si.iterations, iters_t=si_t.iterations, rel=si.rel_residual, events=e,
                       u=u, grads=grads)
        return res

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, marks = [], []
    for _ in range(steps):
        results.append(step())
        marks.append(time.perf_counter())      # each step ends in a host synchronisation
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / steps
    for r, a, b in zip(results, [t0] + marks[:-1], marks):
        r["wall_ms"] = (b - a) * 1e3
    for r in results:
        if "events" in r:
            e = r.pop("events")
            r["ms_solve"] = e[0].elapsed_time(e[1])
            r["ms_solve_t"] = e[1].elapsed_time(e[2])
            r["ms_backward"] = e[2].elapsed_time(e[3])
    if with_adjoint:
        r = results[-1]
        r["rms"] = float(torch.sqrt(torch.mean((r.pop("u") - exact) ** 2)))
        r.pop("grads")
    return cover, results, dt, t_cover


def per_circle_comparison(spacing=0.11):
    """The plain per-circle loop (same kernels, one launch sequence per circle)
    against the batched plan, on a reduced uneven-resolution cover (config 3's
    disk with a hole and resolution draw at lattice spacing 0.11: about 250
    circles), assembly only, one step each after one warm-up."""
    import workloads
    cfg = workloads.config3(spacing=spacing)
    out = {}
    for plan in ("autotuned", "per_circle"):
        cover, results, dt, _ = run_gpu(cfg, 1, 1, with_adjoint=False, plan=plan, use_graph=True)
        s = results[-1]["stats"]
        out[plan] = {"ms_assembly": float(s.ms_total), "ms_lu": float(s.ms_lu),
                     "launches": int(s.n_launch_spectral)}
    out["circles"] = int(cover.info.n_circles)
    out["floating"] = int(cover.info.n_float)
    out["speedup"] = out["per_circle"]["ms_assembly"] / out["autotuned"]["ms_assembly"]
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
    return out


# ------------------------------------------------------------------ CPU leg

_POOL_STATE = {}


def _pool_init():
    from threadpoolctl import threadpool_limits
    _POOL_STATE["limits"] = threadpool_limits(1)


def _spectral_task(m):
    from oracle import spectral
    t0 = time.perf_counter()
    spectral.floating_rows(_POOL_STATE["prob"], _POOL_STATE["cover"], int(m))
    return time.perf_counter() - t0


def _mc_task(i):
    from oracle import montecarlo
    t0 = time.perf_counter()
    st = montecarlo.mc_rows(_POOL_STATE["prob"], _POOL_STATE["cover"], _POOL_STATE["mc"], [int(i)])[-1]
    return time.perf_counter() - t0, st


def cpu_baseline(workload, frac=0.02, single_frac=0.0025, budget_s=30.0):
    """The oracle (plain FP64 NumPy/SciPy, untuned) on the host cores, assembly
    only: a seeded sample of `frac` of the floating circles and of the Monte
    Carlo knots (full paths each) spread over one worker process per core of
    this process's CPU share (at most 16; BLAS threads 1 per worker), timed
    by wall clock and extrapolated linearly to the whole cover; and a smaller
    sample on one core for the single-core rate.  Runs in a process that has
    not touched the GPU."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import geometry, montecarlo, spectral
    from oracle.geometry import ROW_MC

    cfg = workloads.CONFIGS[workload]()
    prob = cfg["problem"]
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    with threadpool_limits(1):
        cv = geometry.build_cover(prob["domain"], cfg["cover"])
    fl = np.nonzero(cv.floating)[0]
    mck = np.nonzero(cv.row_class == ROW_MC)[0]
    rng = np.random.default_rng(12345)
    n_fl = max(cores, int(round(frac * len(fl)))) if len(fl) else 0
    n_mc = max(cores, int(round(frac * len(mck)))) if len(mck) else 0
    s_fl = rng.choice(fl, min(n_fl, len(fl)), replace=False) if len(fl) else fl
    s_mc = rng.choice(mck, min(n_mc, len(mck)), replace=False) if len(mck) else mck
    _POOL_STATE.update(prob=prob, cover=cv, mc=cfg["mc"])
    with threadpool_limits(1):
        if len(fl):
            spectral.floating_rows(prob, cv, int(fl[0]))     # shared grid tables: set-up, not timed
    ctx = mp.get_context("fork")
    with ctx.Pool(cores, initializer=_pool_init) as pool:
        pool.map(_spectral_task, s_fl[:cores])             # each worker's grid tables
        t0 = time.perf_counter()
        pool.map(_spectral_task, s_fl, chunksize=1)
        w_fl = time.perf_counter() - t0
        t0 = time.perf_counter()
        res = pool.map(_mc_task, s_mc, chunksize=1)
        w_mc = time.perf_counter() - t0
    steps = sum(r[1] for r in res)
    t_multi = (w_fl * len(fl) / max(1, len(s_fl)) if len(s_fl) else 0.0) + \
              (w_mc * len(mck) / max(1, len(s_mc)) if len(s_mc) else 0.0)
    # one core: the first circles and knots of the same seeded sample
    n1_fl = max(2, int(round(single_frac * len(fl)))) if len(fl) else 0
    n1_mc = max(2, int(round(single_frac * len(mck)))) if len(mck) else 0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for m in s_fl[:n1_fl]:
            spectral.floating_rows(prob, cv, int(m))
            if time.perf_counter() - t0 > budget_s / 2:
                break
        k_fl = max(1, min(n1_fl, len(s_fl)))
        t_fl1 = (time.perf_counter() - t0) / k_fl if len(fl) else 0.0
        t0 = time.perf_counter()
        k_mc = 0
        for i in s_mc[:n1_mc]:
            montecarlo.mc_rows(prob, cv, cfg["mc"], [int(i)])
            k_mc += 1
            if time.perf_counter() - t0 > budget_s / 2:
                break
        t_mc1 = (time.perf_counter() - t0) / max(1, k_mc) if len(mck) else 0.0
    t_single = t_fl1 * len(fl) + t_mc1 * len(mck)
    n_circles = len(cv.radii)
    return {
        "value": n_circles / t_multi,
        "unit": "circles/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"seeded {100 * frac:g} % sample: {len(s_fl)} of {len(fl)} floating circles and "
                   f"{len(s_mc)} of {len(mck)} Monte Carlo knots (full paths), {cores} worker processes, "
                   f"wall {w_fl + w_mc:.1f} s, extrapolated linearly; assembly only"),
        "single_core": {"value": n_circles / t_single, "unit": "circles/s", "cores": 1,
                        "sample": f"{k_fl} floating circles and {k_mc} Monte Carlo knots of the same sample, "
                                  f"extrapolated linearly",
                        "s_per_floating_circle": t_fl1, "s_per_mc_knot": t_mc1},
        "mc_path_steps_per_s": steps / w_mc if w_mc > 0 else None,
    }


def cpu_baseline_subprocess(workload, frac):
    """Runs cpu_baseline in a child interpreter (no GPU state, fork-safe pool)."""
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                          "--workload", workload, "--cpu-frac", str(frac)],
                         stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=900)
    if out.returncode != 0:
        raise RuntimeError("CPU baseline failed:\n" + out.stderr[-2000:])
    return json.loads(out.stdout.strip().splitlines()[-1])


# ------------------------------------------------------------------- report

def _profile_value(name, key, sources):
    """A number recorded in profiles/<name> (a committed rocprofv3 summary),
    or None when the file is missing or the kernel sources it was taken on
    have changed since: the summary records the SHA-256 of the listed
    sources (under paper_2311_08946_amd/csrc/, concatenated in order)."""
    import hashlib
    import re
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    m_v = re.search(key + r": ([0-9.eE+-]+)", text)
    if not (m_sha and m_v):
        return None
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(here, "paper_2311_08946_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != m_sha.group(1):
        return None
    return float(m_v.group(1))


# kernel sources behind each phase's counters
PHASE_SOURCES = {"lu": ["lu.hip"], "bicgstab": ["solve.hip"], "mc": ["mc.hip", "device_common.h"]}


def measured_traffic(workload, phase):
    """HBM bytes per step of a phase, from the FETCH_SIZE / WRITE_SIZE summary
    profiles/hbm_traffic_<phase>_<workload>.md (calibrated against a copy
    kernel), or None (no summary, or the kernels changed since)."""
    if phase not in PHASE_SOURCES:
        return None
    return _profile_value(f"hbm_traffic_{phase}_{workload}.md", "bytes_per_step", PHASE_SOURCES[phase])


def measured_valu(workload):
    """VALU issue utilisation and lane instructions per path step of the paths
    kernel, from profiles/pmc_valu_paths_<workload>.md, or None."""
    util = _profile_value(f"pmc_valu_paths_{workload}.md", "valu_active_frac", PHASE_SOURCES["mc"])
    per = _profile_value(f"pmc_valu_paths_{workload}.md", "valu_insts_per_path_step", PHASE_SOURCES["mc"])
    if util is None or per is None:
        return None
    return {"valu_active_frac": util, "valu_insts_per_path_step": per}


def isolated_phases(cover, cfg, budget, plan, keep, reps=2):
    """Median LU, Monte Carlo and build times of `reps` assemblies with the
    Monte Carlo rows after the floating rows (untimed by the step): each phase
    then has the GPU to itself, while in the step the Monte Carlo kernel shares
    it with the build and the first LU panels."""
    import numpy as np
    import paper_2311_08946_amd.binding as pdd
    st = []
    for _ in range(reps):
        sysm = pdd.System(cover, cfg["problem"], cfg["mc"], keep_factors=keep, hbm_budget_bytes=budget,
                          plan=plan, mc_order="after")
        st.append(sysm.stats)
        del sysm
    return {k: float(np.median([getattr(s, "ms_" + k) for s in st])) for k in ("lu", "mc", "build", "total")}


def phase_rooflines(cover, cfg, results, with_adj):
    """One roofline entry per phase, each from times measured in this run."""
    import numpy as np
    st = [r["stats"] for r in results]
    med = lambda xs: float(np.median(xs))
    ms_lu = med([s.ms_lu for s in st])
    ms_mc = med([s.ms_mc for s in st])
    flops = spectral_flops(cover, cfg)
    info = cover.info
    out = {}
    lu_tf = flops / (ms_lu * 1e-3) / 1e12
    out["lu"] = {"bound": "mfma", "achieved": lu_tf, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                 "frac": lu_tf / PEAK_FP64_MFMA_TFLOPS, "ms": ms_lu,
                 "work": f"{flops:.4g} flops: sum over floating circles of 2/3 n^3 + 2 n^2 (M+1)"}
    if ms_mc > 0:
        # mean arc length (knots of Gamma_m) over the Monte Carlo knots' circles
        _, rc, asg, own = cover.knots()
        cnt = np.bincount(own, minlength=int(info.n_circles))
        arc_mean = float(np.mean(cnt[asg[rc == 1]]))
        ops = mc_ops(st[-1], arc_mean, field_ops_per_point(cfg["problem"]))
        tf = ops / (ms_mc * 1e-3) / 1e12
        out["mc"] = {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": tf / PEAK_FP64_VECTOR_TFLOPS, "ms": ms_mc,
                     "work": f"{ops:.4g} FP64 operations for {st[-1].path_steps} path steps, {st[-1].paths} "
                             f"paths, {st[-1].gamma_exits} exits on Gamma (mean arc {arc_mean:.1f} knots)"}
    if with_adj:
        ms_s = med([r["ms_solve"] for r in results])
        ms_t = med([r["ms_solve_t"] for r in results])
        it = results[-1]["iters"]
        it_t = results[-1]["iters_t"]
        bpi = bicgstab_bytes_per_iter(cover.N, cover.nnz)
        gbs = bpi * (it + it_t) / ((ms_s + ms_t) * 1e-3) / 1e9
        out["bicgstab"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": gbs / PEAK_HBM_GBS, "ms": ms_s + ms_t,
                           "work": f"{bpi:.4g} B per iteration x {it} + {it_t} iterations (C and C^T)"}
        if not st[-1].recompute:
            ms_b = med([r["ms_backward"] for r in results])
            nb = adjoint_bytes(cover, cfg)
            gbs = nb / (ms_b * 1e-3) / 1e9
            out["adjoint"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": gbs / PEAK_HBM_GBS, "ms": ms_b,
                              "work": f"{nb:.4g} B: factors, W, pivots, scales read, gradients written"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default=None,
                    help="default: config5 (config2 with --ras, whose dense part inverses are sized "
                         "for 32x32 circles)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the chunked-factor step and the per-circle comparison")
    ap.add_argument("--plan", default="autotuned", choices=["autotuned", "batched", "per_circle"])
    ap.add_argument("--cpu-frac", type=float, default=0.02)
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer 4 times (calibrates HBM byte counters)")
    ap.add_argument("--ras", default=None, metavar="PXxPY",
                    help="instead of the step, measure GMRES with the RAS preconditioner of PXxPY parts")
    args = ap.parse_args()
    if args.workload is None:
        args.workload = "config2" if args.ras else "config5"
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline(args.workload, args.cpu_frac)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; the "
              "assembly would shard by spatial blocks of circles with a halo exchange in the solve.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 8, "launches": 4}), flush=True)
        return

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
    # the oracle first, in a child process, before this one touches the GPU
    cb = None
    if not args.no_cpu_baseline:
        print("[bench] CPU baseline (oracle) ...", file=sys.stderr, flush=True)
        cb = cpu_baseline_subprocess(args.workload, args.cpu_frac)
    print(f"[bench] GPU: {args.workload}, {args.warmup} warm-up + {args.steps} timed steps",
          file=sys.stderr, flush=True)
    with_adj = wl["adjoint"] and not args.no_adjoint
    cover, results, dt, t_cover = run_gpu(cfg, args.steps, args.warmup, with_adjoint=with_adj,
                                          budget=wl["budget"], plan=args.plan)
    import numpy as np
    info = cover.info
    st = [r["stats"] for r in results]
    n_circles = int(info.n_circles)
    n_float = int(info.n_float)
    med = lambda xs: float(np.median(xs))
    ms_mc = med([s.ms_mc for s in st])
    ms_asm = med([s.ms_total for s in st])
    ms_spec = med([s.ms_build + s.ms_lu + s.ms_solve + s.ms_eval for s in st])
    path_steps = st[-1].path_steps
    roof = phase_rooflines(cover, cfg, results, with_adj)
    for ph in roof:
        roof[ph]["traffic"] = measured_traffic(args.workload, ph)
    if "bicgstab" in roof:
        per_it = _profile_value(f"hbm_traffic_bicgstab_{args.workload}.md", "bytes_per_iteration",
                                PHASE_SOURCES["bicgstab"])
        its = results[-1]["iters"] + results[-1]["iters_t"]     # as in the roofline's work
        roof["bicgstab"]["traffic"] = per_it * its if per_it is not None else None
    if "mc" in roof:
        roof["mc"]["counters"] = measured_valu(args.workload)
        if not st[-1].mc_after_floating:
            print("[bench] phases alone (Monte Carlo after the floating rows)", file=sys.stderr, flush=True)
            iso = isolated_phases(cover, cfg, wl["budget"], args.plan, with_adj)
            for ph in ("lu", "mc"):
                a = roof[ph]["achieved"] * roof[ph]["ms"] / iso[ph]
                roof[ph]["alone"] = {"ms": iso[ph], "achieved": a, "frac": a / roof[ph]["peak"],
                                     "assembly_ms": iso["total"]}
    # the headline roofline: the phase that takes the most time per step
    dom = max(roof, key=lambda k: roof[k]["ms"])
    kernels = {
        "lu": f"batched LU + triangular solves of {n_float} circles (lu_pupd/lu_panel/lu_urow/lu_bdiag/"
              "lu_bupd launch sequence, HIP events around it on the calling stream)",
        "mc": "paths_kernel (Euler-Maruyama paths, one per lane) on the side stream",
        "bicgstab": "BiCGStab on C and C^T (update_p/spmv_v/spmv_t/update_xr per iteration)",
        "adjoint": "adjoint_kernel over the stored factors",
    }
    roofline = dict(roof[dom])
    roofline["kernel"] = kernels[dom]
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
        "phase_ms": {k: med([getattr(s, "ms_" + k) for s in st])
                     for k in ("sample", "build", "lu", "eval", "mc", "total")},
        "build_cover_s": t_cover,
        "step_wall_ms": [round(r["wall_ms"], 1) for r in results],
        "schedule": {"plan": args.plan, "mixed_buckets": bool(st[-1].mixed_buckets),
                     "grid_cap": int(st[-1].grid_cap), "lookahead": bool(st[-1].lu_lookahead),
                     "mc_after_floating": bool(st[-1].mc_after_floating),
                     "groups": int(st[-1].n_groups),
                     "graph_replays": int(st[-1].graph_replays), "lu_launches": int(st[-1].n_launch_spectral)},
        "factor_bytes_kept": int(st[-1].factor_bytes),
        "factors_recomputed_in_backward": bool(st[-1].recompute),
        "roofline": roofline,
        "rooflines": roof,
    }
    if with_adj:
        out["phase_ms"].update(solve=med([r["ms_solve"] for r in results]),
                               solve_transpose=med([r["ms_solve_t"] for r in results]),
                               backward=med([r["ms_backward"] for r in results]))
        out["solve_iterations"] = results[-1]["iters"]
        out["solve_iterations_transpose"] = results[-1]["iters_t"]
        out["rms_error_vs_exact"] = results[-1]["rms"]
    if not args.no_extras and wl.get("chunked_budget") and with_adj:
        print("[bench] chunked-factor step", file=sys.stderr, flush=True)
        _, res_c, dt_c, _ = run_gpu(cfg, 1, 1, with_adjoint=True, budget=wl["chunked_budget"], plan=args.plan)
        r = res_c[-1]
        out["chunked_factors"] = {
            "hbm_budget_bytes": wl["chunked_budget"], "fwd_adjoint_s": dt_c,
            "ms_backward": r["ms_backward"], "recomputed": bool(r["stats"].recompute),
            "groups": int(r["stats"].n_groups), "graph_replays": int(r["stats"].graph_replays)}
    if not args.no_extras:
        print("[bench] per-circle comparison", file=sys.stderr, flush=True)
        out["per_circle_vs_batched"] = per_circle_comparison()
    if cb is not None:
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline_single_core"] = cb["single_core"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
