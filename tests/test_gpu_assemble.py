"""GPU parity of the assembled system against the FP64 CPU oracle.

Floating (spectral) rows: per row, max_j |dC_ij| <= 1e-10 max_j |C_ij|; for r,
|dr_i| <= 1e-10 (|r_i| + r_m^2 max |f| on circle m).  Monte Carlo rows use the
same Philox streams as the oracle: every entry must lie within 3 of the
oracle's standard errors (in practice they agree to rounding).  Boundary rows
must match to rounding of g.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import assemble, fields, geometry, montecarlo, spectral
from oracle.geometry import ROW_BOUNDARY, ROW_MC, ROW_SPECTRAL

pytestmark = pytest.mark.gpu

from helpers_parity import (TOL_G, _check_mc_rows, _check_rhs, _check_spectral_rows, _fscale,
                            _gpu_system, _row, _say, pick_mc_knots, sampled_parity)


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_08946_amd.binding as pdd
    pdd.lib()
    return pdd


@pytest.mark.parametrize("name", ["config1", "small_variable"])
def test_small_configs_match_oracle(name):
    pdd = _gpu()
    cfg = workloads.config1() if name == "config1" else workloads.small_variable(paths=256)
    prob = cfg["problem"]
    _say(f"[gpu] assemble {name}")
    cv, sysm, val, b, se, se_b = _gpu_system(pdd, cfg)
    assert sysm.stats.breakdowns == 0 and sysm.stats.capped_paths == 0
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    ref = assemble.assemble(prob, ref_cover, cfg["mc"])
    assert abs(sysm.stats.path_steps - ref.path_steps) <= 1e-4 * ref.path_steps
    spec = np.nonzero(ref_cover.row_class == ROW_SPECTRAL)[0]
    mcr = np.nonzero(ref_cover.row_class == ROW_MC)[0]
    bnd = np.nonzero(ref_cover.row_class == ROW_BOUNDARY)[0]
    worst = _check_spectral_rows(ref_cover, ref.val, ref.b, val, b, spec, prob)
    _check_rhs(ref_cover, ref.b, b, spec, _fscale(prob, ref_cover, np.nonzero(ref_cover.floating)[0]))
    frac = _check_mc_rows(ref_cover, ref.val, ref.se, ref.b, ref.se_b, val, b, mcr)
    assert frac > 0.99
    for i in bnd:
        assert _row(ref_cover, val, i)[0] == 1.0
        assert abs(b[i] - ref.b[i]) <= 1e-14 * (1 + abs(ref.b[i]))
    _say(f"[gpu] {name}: worst spectral row diff {worst:.2e}, MC r_i within 1e-9: {frac:.4f}")


@pytest.mark.parametrize("kind", ["no_floating", "one_floating"])
def test_degenerate_covers_match_oracle(kind):
    # no floating circle at all (no LU launches) and a single one (a batch of one)
    pdd = _gpu()
    cfg = workloads.degenerate(kind)
    prob = cfg["problem"]
    _say(f"[gpu] assemble {kind}")
    cv, sysm, val, b, se, se_b = _gpu_system(pdd, cfg)
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    assert cv.N == ref_cover.N and int(cv.info.n_float) == int(np.sum(ref_cover.floating))
    ref = assemble.assemble(prob, ref_cover, cfg["mc"])
    spec = np.nonzero(ref_cover.row_class == ROW_SPECTRAL)[0]
    mcr = np.nonzero(ref_cover.row_class == ROW_MC)[0]
    if len(spec):
        _check_spectral_rows(ref_cover, ref.val, ref.b, val, b, spec, prob)
        _check_rhs(ref_cover, ref.b, b, spec, _fscale(prob, ref_cover, np.nonzero(ref_cover.floating)[0]))
    assert _check_mc_rows(ref_cover, ref.val, ref.se, ref.b, ref.se_b, val, b, mcr) > 0.99
    u, info = sysm.solve(rtol=1e-12)
    assert info.converged


def test_per_circle_plan_is_bitwise_equal_to_batched():
    pdd = _gpu()
    cfg = workloads.small_variable(paths=64)
    _say("[gpu] per-circle vs batched plan")
    _, _, v1, b1, _, _ = _gpu_system(pdd, cfg)
    _, _, v2, b2, _, _ = _gpu_system(pdd, cfg, plan="per_circle")
    assert np.array_equal(v1, v2) and np.array_equal(b1, b2)


def test_mixed_resolution_buckets_match_oracle():
    """Uneven resolutions in one assembly (collocation sizes 576 to 4096, one
    size bucket each): every floating row against the oracle, and the batched
    plan bitwise equal to the plain per-circle loop."""
    pdd = _gpu()
    cfg = workloads.mixed_small()
    prob = cfg["problem"]
    _say("[gpu] assemble mixed_small (n = 576 .. 4096)")
    cv, sysm, val, b, se, se_b = _gpu_system(pdd, cfg)
    assert sysm.stats.breakdowns == 0 and sysm.stats.capped_paths == 0
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    fl = np.nonzero(ref_cover.floating)[0]
    assert sorted(int(ref_cover.Nr[m] * ref_cover.Ntheta[m]) for m in fl) == [576, 1024, 2304, 4096]
    ref = assemble.assemble(prob, ref_cover, cfg["mc"])
    spec = np.nonzero(ref_cover.row_class == ROW_SPECTRAL)[0]
    mcr = np.nonzero(ref_cover.row_class == ROW_MC)[0]
    worst = _check_spectral_rows(ref_cover, ref.val, ref.b, val, b, spec, prob)
    _check_rhs(ref_cover, ref.b, b, spec, _fscale(prob, ref_cover, fl))
    _check_mc_rows(ref_cover, ref.val, ref.se, ref.b, ref.se_b, val, b, mcr)
    _, _, v2, b2, _, _ = _gpu_system(pdd, cfg, plan="per_circle")
    assert np.array_equal(val, v2) and np.array_equal(b, b2)
    _say(f"[gpu] mixed_small: worst spectral row diff {worst:.2e}")


def test_config2_full_size_sampled():
    """Config 2 at its full size (900 floating circles, n = 1024, 10^4 paths)
    in the launch configuration the benchmark times (autotuned schedule, graph
    replay, factors kept); the oracle recomputes 10 % of the floating circles
    -- the first and last of the LU batch among them -- and 10 % of the Monte
    Carlo knots one by one."""
    pdd = _gpu()
    cfg = workloads.config2()
    prob = cfg["problem"]
    _say("[gpu] assemble config2 (full size)")
    cv, sysm, val, b, se, se_b = _gpu_system(pdd, cfg, plan="autotuned", use_graph=True, keep_factors=True)
    assert sysm.stats.breakdowns == 0 and sysm.stats.capped_paths == 0
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    rng = np.random.default_rng(123)
    fl = np.nonzero(ref_cover.floating)[0]
    circles = np.concatenate([fl[:1], fl[-1:], rng.choice(fl[1:-1], size=88, replace=False)])
    n_mc = int(np.sum(ref_cover.row_class == ROW_MC))
    knots = pick_mc_knots(ref_cover, rng, (n_mc + 9) // 10)
    _say(f"[gpu] config2: {len(circles)} of {len(fl)} circles, {len(knots)} of {n_mc} MC knots")
    frac = sampled_parity(prob, ref_cover, cfg["mc"], val, b, circles, knots)
    _say(f"[gpu] config2: MC r_i within 1e-9: {frac:.3f}")
    assert frac > 0.97


def test_schedules_are_bitwise_equal():
    """Every schedule of the floating circles -- mixed-bucket or per-bucket
    groups, persistent grids of one or two workgroups per compute unit, graph
    replay, the autotuned choice, small factor budgets that split the work into
    many groups, the Monte Carlo rows beside or after them -- runs the same
    arithmetic per circle and per path, so C and r are bitwise equal."""
    pdd = _gpu()
    import torch
    _say("[gpu] schedules")
    for cfg in (workloads.mixed_small(paths=32), workloads.small_variable(paths=32)):
        prob = cfg["problem"]
        cv = pdd.Cover(prob["domain"], cfg["cover"])
        ref = pdd.System(cv, prob, cfg["mc"])
        rv = ref.copy()
        keep = pdd.System(cv, prob, cfg["mc"], keep_factors=True)
        per = keep.stats.factor_bytes // cv.info.n_float
        variants = [
            dict(mixed_buckets=False),
            dict(grid_cap=1),
            dict(grid_cap=2, use_graph=True),
            dict(hbm_budget_bytes=int(1.5 * per), use_graph=True),
            dict(hbm_budget_bytes=int(1.5 * per), mixed_buckets=False, use_graph=True),
            dict(plan="autotuned"),
            dict(plan="autotuned", use_graph=True),
            dict(mc_order="after"),
            dict(plan="autotuned", mc_order="beside"),
        ]
        for kw in variants:
            s = pdd.System(cv, prob, cfg["mc"], **kw)
            for a, b in zip(rv, s.copy()):
                assert torch.equal(a, b), (cfg["name"], kw)
            _say(f"[gpu] {cfg['name']} {kw}: groups {s.stats.n_groups}, graph replays {s.stats.graph_replays}, "
                 f"mixed {s.stats.mixed_buckets}, cap {s.stats.grid_cap}")
            if "mc_order" in kw:
                assert s.stats.mc_after_floating == (kw["mc_order"] == "after")
            if kw.get("hbm_budget_bytes") and cfg["name"] == "small_variable":
                assert s.stats.n_groups > 1 and s.stats.graph_replays > 0
