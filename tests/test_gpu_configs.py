"""GPU parity at the full sizes of the batching, differentiation and scale
workloads, on sampled outputs the oracle recomputes one by one.

* Uneven resolutions (unit disk minus a hole, about 2e4 circles, collocation
  sizes 256 .. 4096 in five size buckets): one floating circle per bucket and
  Monte Carlo knots against the oracle.
* Differentiation (64 x 64 cover, n = 1024): sampled rows, the adjoint of
  sampled circles against the oracle's adjoint (1e-8), and central differences
  of the assembly on 50 random coordinates.
* Scale (128 x 128 cover, n = 576, 1e5 paths per knot, h = 1e-5): sampled
  rows, BiCGStab to 1e-12, and the adjoint with the factors recomputed in
  chunks under an 8 GiB factor budget, against the oracle's adjoint.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads
from helpers_parity import (_gpu_system, _say, check_circle_gradient, gradient_terms, pick_mc_knots,
                            sampled_parity)
from oracle import geometry, spectral

pytestmark = pytest.mark.gpu

NAMES = ("axx", "axy", "ayy", "bx", "by", "c", "f")


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_08946_amd.binding as pdd
    pdd.lib()
    return pdd, torch


def test_uneven_resolution_cover_full_size_sampled():
    pdd, torch = _gpu()
    cfg = workloads.config3()
    prob = cfg["problem"]
    _say("[gpu] assemble the uneven-resolution cover (full size)")
    cv, sysm, val, b, se, se_b = _gpu_system(pdd, cfg)
    st = sysm.stats
    assert st.breakdowns == 0 and st.capped_paths == 0
    _say(f"[gpu] uneven cover: {cv.info.n_float} floating circles, LU {st.ms_lu:.0f} ms, "
         f"assembly {st.ms_total:.0f} ms")
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    assert ref_cover.N == cv.N
    rng = np.random.default_rng(303)
    fl = np.nonzero(ref_cover.floating)[0]
    sizes = ref_cover.Nr[fl] * ref_cover.Ntheta[fl]
    circles = [rng.choice(fl[sizes == s]) for s in np.unique(sizes)]
    assert sorted(set(int(s) for s in sizes)) == [256, 576, 1024, 2304, 4096]
    frac = sampled_parity(prob, ref_cover, cfg["mc"], val, b, circles, pick_mc_knots(ref_cover, rng, 32))
    _say(f"[gpu] uneven cover: MC r_i within 1e-9 on {frac:.3f} of 32 knots")
    # every entry is within 3 standard errors; r_i agrees to rounding unless one
    # of the knot's paths takes a different exit (last-ulp differences between
    # the host's and the device's libm): rare at 1e3 paths of about 16 steps
    assert frac >= 0.9


def _circle_rows(asg, m):
    return np.nonzero(asg == m)[0]


def test_differentiation_workload_full_size():
    pdd, torch = _gpu()
    from paper_2311_08946_amd import autograd as pag
    cfg = workloads.config4()
    prob = cfg["problem"]
    _say("[gpu] differentiation workload (64 x 64 cover)")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    samples = pag.node_samples(cv, prob)
    sysm = pdd.System(cv, prob, cfg["mc"], samples=samples, keep_factors=True, plan="autotuned",
                      use_graph=True)
    assert sysm.stats.breakdowns == 0 and sysm.stats.recompute == 0
    val, b, _, _ = (t.cpu().numpy() for t in sysm.copy())
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    rng = np.random.default_rng(404)
    fl = np.nonzero(ref_cover.floating)[0]
    circles = np.concatenate([fl[:1], fl[-1:], rng.choice(fl[1:-1], size=30, replace=False)])
    frac = sampled_parity(prob, ref_cover, cfg["mc"], val, b, circles, pick_mc_knots(ref_cover, rng, 16))
    _say(f"[gpu] differentiation workload: MC r_i within 1e-9 on {frac:.3f} of 16 knots")
    assert frac >= 0.9
    # loss sum_i (u_i - u_target_i)^2, u_target = exact solution + N(0, 1e-3)
    xy, rc, asg, own = cv.knots()
    xy_d = torch.tensor(xy, dtype=torch.float64, device="cuda")
    target = pdd.eval_field(prob, "u", xy_d) + torch.tensor(
        workloads.target_noise(cfg, cv.N), dtype=torch.float64, device="cuda")
    u, info = sysm.solve(rtol=1e-13)
    assert info.converged
    lam, info_t = sysm.solve(rhs=2.0 * (u - target), transpose=True, rtol=1e-13)
    assert info_t.converged
    g = {k: v.cpu().numpy() for k, v in sysm.backward(u, lam).items()}
    u_h, lam_h = u.cpu().numpy(), lam.cpu().numpy()
    n_params = 3 * len(samples["axx"])
    _say(f"[gpu] {n_params} parameters (a, c, f node samples); BiCGStab {info.iterations}/{info_t.iterations}")
    # five random floating circles: their adjoint against the oracle's, then
    # central differences of l(theta) = sum_{i in K_m} lambda_i (r_i - C_i u)
    # on ten random coordinates of each (50 in all; only the rows of the
    # coordinate's circle depend on it)
    nxy, off, ids = cv.nodes()
    pos = {int(m): f for f, m in enumerate(ids)}
    rowptr, cols = cv.pattern()
    gmax = max(np.max(np.abs(v)) for v in g.values())
    base = {k: v.clone() for k, v in samples.items()}

    def ell(s, m):
        """l over circle m's rows, and the sum of the magnitudes it adds up
        (the assembly's own rounding, about 1e-13 relative, scales with it)."""
        sy = pdd.System(cv, prob, cfg["mc"], samples=s)
        vv, bb, _, _ = (t.cpu().numpy() for t in sy.copy())
        rows = _circle_rows(asg, m)
        tot = mag = 0.0
        for i in rows:
            lo, hi = rowptr[i], rowptr[i + 1]
            cu = vv[lo:hi] * u_h[cols[lo:hi]]
            tot += lam_h[i] * (bb[i] - np.sum(cu))
            mag += abs(lam_h[i]) * (abs(bb[i]) + np.sum(np.abs(cu)))
        return tot, mag

    for m in rng.choice(fl, size=5, replace=False):
        m = int(m)
        f = pos[m]
        grid = spectral.local_grid(ref_cover.Nr[m], ref_cover.Ntheta[m])
        s_ref = spectral.node_samples(prob, grid, *ref_cover.centres[m], ref_cover.radii[m])
        ref, slack = gradient_terms(ref_cover, m, s_ref, u_h, lam_h)
        check_circle_gradient(ref, slack, {k: g[k][off[f]:off[f + 1]] for k in NAMES})
        for t in range(10):
            k = NAMES[int(rng.integers(7))]
            ql = int(rng.integers(off[f + 1] - off[f]))
            q = int(off[f]) + ql
            theta = base[k][q].item()
            eps = 1e-6 * max(1.0, abs(theta))
            sp_ = {kk: vv.clone() for kk, vv in base.items()}
            sm_ = {kk: vv.clone() for kk, vv in base.items()}
            sp_[k][q] += eps
            sm_[k][q] -= eps
            lp, mag = ell(sp_, m)
            lm, _ = ell(sm_, m)
            fd = (lp - lm) / (2 * eps)
            ga = g[k][q]
            tol = 1e-5 * abs(ga) + 1e-9 * gmax + 1e-13 * mag / eps + slack[k][ql]
            assert abs(fd - ga) <= tol, (m, k, q, fd, ga, tol)


def test_scale_workload_chunked_adjoint():
    pdd, torch = _gpu()
    cfg = workloads.config5()
    prob = cfg["problem"]
    _say("[gpu] scale workload (128 x 128 cover, 1e5 paths per knot)")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"], keep_factors=True, hbm_budget_bytes=8 << 30)
    st = sysm.stats
    assert st.breakdowns == 0 and st.capped_paths == 0 and st.recompute == 1
    _say(f"[gpu] scale: assembly {st.ms_total:.0f} ms, {st.path_steps} path steps, MC {st.ms_mc:.0f} ms")
    val, b, _, _ = (t.cpu().numpy() for t in sysm.copy())
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    rng = np.random.default_rng(505)
    fl = np.nonzero(ref_cover.floating)[0]
    circles = np.concatenate([fl[:1], fl[-1:], rng.choice(fl[1:-1], size=30, replace=False)])
    frac = sampled_parity(prob, ref_cover, cfg["mc"], val, b, circles, pick_mc_knots(ref_cover, rng, 16))
    assert frac >= 0.9
    u, info = sysm.solve(rtol=1e-12)
    assert info.converged
    rowptr, cols = cv.pattern()
    C = sp.csr_matrix((val, cols, rowptr), shape=(cv.N, cv.N))
    u_h = u.cpu().numpy()
    assert np.linalg.norm(C @ u_h - b) <= 1e-11 * np.linalg.norm(b)
    xy, rc, asg, own = cv.knots()
    xy_d = torch.tensor(xy, dtype=torch.float64, device="cuda")
    target = pdd.eval_field(prob, "u", xy_d) + torch.tensor(
        workloads.target_noise(cfg, cv.N), dtype=torch.float64, device="cuda")
    lam, info_t = sysm.solve(rhs=2.0 * (u - target), transpose=True, rtol=1e-12)
    assert info_t.converged
    g = {k: v.cpu().numpy() for k, v in sysm.backward(u, lam).items()}
    lam_h = lam.cpu().numpy()
    nxy, off, ids = cv.nodes()
    pos = {int(m): f for f, m in enumerate(ids)}
    for m in circles[:8]:
        grid = spectral.local_grid(ref_cover.Nr[m], ref_cover.Ntheta[m])
        s_ref = spectral.node_samples(prob, grid, *ref_cover.centres[m], ref_cover.radii[m])
        ref, slack = gradient_terms(ref_cover, m, s_ref, u_h, lam_h)
        f = pos[int(m)]
        check_circle_gradient(ref, slack, {k: g[k][off[f]:off[f + 1]] for k in NAMES})
    _say(f"[gpu] scale: BiCGStab {info.iterations}/{info_t.iterations} iterations, MC r_i within 1e-9: {frac:.2f}")


def test_scale_workload_bench_configuration():
    """Config 5 in the launch configuration the benchmark times: autotuned
    schedule with graph replay and the factors kept (48 GB).  Sampled rows,
    C and r bitwise equal to the chunked-recompute assembly, and BiCGStab on
    C and C^T to 1e-12 with the residual checked on the host."""
    pdd, torch = _gpu()
    cfg = workloads.config5()
    prob = cfg["problem"]
    _say("[gpu] scale workload, benchmark launch configuration")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"], keep_factors=True, plan="autotuned", use_graph=True)
    st = sysm.stats
    assert st.breakdowns == 0 and st.capped_paths == 0 and st.recompute == 0 and st.factor_bytes > 40e9
    val, b, _, _ = (t.cpu().numpy() for t in sysm.copy())
    chunked = pdd.System(cv, prob, cfg["mc"], keep_factors=True, hbm_budget_bytes=8 << 30, plan="autotuned",
                         use_graph=True)
    v2, b2, _, _ = (t.cpu().numpy() for t in chunked.copy())
    assert np.array_equal(val, v2) and np.array_equal(b, b2)
    del chunked
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    rng = np.random.default_rng(506)
    fl = np.nonzero(ref_cover.floating)[0]
    circles = np.concatenate([fl[:1], fl[-1:], rng.choice(fl[1:-1], size=30, replace=False)])
    frac = sampled_parity(prob, ref_cover, cfg["mc"], val, b, circles, pick_mc_knots(ref_cover, rng, 16))
    assert frac >= 0.9
    rowptr, cols = cv.pattern()
    C = sp.csr_matrix((val, cols, rowptr), shape=(cv.N, cv.N))
    u, info = sysm.solve(rtol=1e-12)
    assert info.converged
    assert np.linalg.norm(C @ u.cpu().numpy() - b) <= 1e-11 * np.linalg.norm(b)
    g = np.random.default_rng(7).standard_normal(cv.N)
    lam, info_t = sysm.solve(rhs=torch.tensor(g, device="cuda"), transpose=True, rtol=1e-12)
    assert info_t.converged
    assert np.linalg.norm(C.T @ lam.cpu().numpy() - g) <= 1e-11 * np.linalg.norm(g)
    _say(f"[gpu] scale (bench configuration): BiCGStab {info.iterations}/{info_t.iterations}, "
         f"MC r_i within 1e-9: {frac:.2f}")

