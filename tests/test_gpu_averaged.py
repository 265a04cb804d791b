"""GPU parity of the averaged rows (eqs. 38-39) against the FP64 CPU oracle.

The library assembles every pair (knot i, containing circle m) as a row of its
own and combines them; the oracle builds the same pairs and combines them
itself.  Bars: the CSR pattern is identical; C_ii equals the number of
containing circles exactly; entries within 3 of the oracle's standard errors
plus 1e-10 of the row's largest entry (floating pairs have zero standard
error, so they are held to the floating-row bar); r_i within 3 standard
errors plus 1e-10 (|r_i| + 1), and to 1e-9 on all but rare rows (an exit
decided by the last ulp of a libm result); the adjoint per floating circle
within 1e-8 of its largest entry.
"""
import sys

import numpy as np
import pytest

import workloads
from oracle import adjoint, assemble, geometry, spectral
from oracle.geometry import ROW_BOUNDARY, RULE_AVERAGED

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_08946_amd.binding as pdd
    pdd.lib()
    return pdd, torch


def _averaged(cfg):
    cfg = dict(cfg)
    cfg["cover"] = dict(cfg["cover"])
    cfg["cover"]["rule"] = RULE_AVERAGED
    return cfg


@pytest.mark.parametrize("name", ["config1", "small_variable"])
def test_averaged_rows_match_oracle(name):
    pdd, torch = _gpu()
    cfg = _averaged(workloads.config1(paths=256) if name == "config1"
                    else workloads.small_variable(paths=128))
    prob = cfg["problem"]
    _say(f"[gpu] averaged rows {name}")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"])
    assert sysm.stats.breakdowns == 0 and sysm.stats.capped_paths == 0
    val, b, se, se_b = (t.cpu().numpy() for t in sysm.copy())
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    ref = assemble.assemble(prob, ref_cover, cfg["mc"])
    rowptr, cols = cv.pattern()
    assert np.array_equal(rowptr, ref_cover.rowptr) and np.array_equal(cols, ref_cover.cols)
    assert abs(sysm.stats.path_steps - ref.path_steps) <= 1e-4 * max(ref.path_steps, 1)
    close, n_mc, worst = 0, 0, 0.0
    for i in range(ref_cover.N):
        sl = slice(ref_cover.rowptr[i], ref_cover.rowptr[i + 1])
        g, o, s = val[sl], ref.val[sl], ref.se[sl]
        if ref_cover.row_class[i] == ROW_BOUNDARY:
            assert g[0] == 1.0 and abs(b[i] - ref.b[i]) <= 1e-14 * (1 + abs(ref.b[i]))
            continue
        d = list(ref_cover.cols[sl]).index(i)
        assert g[d] == float(len(ref_cover.containers[i])), (i, g[d])
        bound = 3 * s + TOL * np.max(np.abs(o))
        diff = np.abs(g - o)
        assert np.all(diff <= bound), (i, float(np.max(diff - bound)))
        worst = max(worst, float(np.max(diff)) / float(np.max(np.abs(o))))
        assert abs(b[i] - ref.b[i]) <= 3 * ref.se_b[i] + TOL * (abs(ref.b[i]) + 1), (i, b[i], ref.b[i])
        assert (se_b[i] == 0.0) == (ref.se_b[i] == 0.0)
        assert abs(se_b[i] - ref.se_b[i]) <= 0.5 * ref.se_b[i]
        if ref.se_b[i] > 0:
            n_mc += 1
            close += int(abs(b[i] - ref.b[i]) <= 1e-9 * (1 + abs(ref.b[i])))
    assert n_mc == 0 or close / n_mc > 0.99
    u, info = sysm.solve(rtol=1e-12)
    assert info.converged
    _say(f"[gpu] {name}: worst row diff {worst:.2e}, r_i within 1e-9 on {close}/{n_mc} MC rows")


def test_averaged_adjoint_matches_oracle():
    pdd, torch = _gpu()
    cfg = _averaged(workloads.small_variable(paths=64))
    prob = cfg["problem"]
    _say("[gpu] averaged adjoint vs oracle")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    pc, pknot = geometry.pair_cover(ref_cover)
    results = []
    for budget in (0, 1):   # factors kept, then recomputed chunk by chunk
        sysm = pdd.System(cv, prob, cfg["mc"], keep_factors=True, hbm_budget_bytes=budget)
        u, _ = sysm.solve(rtol=1e-13)
        rng = np.random.default_rng(5)
        target = torch.tensor(u.cpu().numpy() + rng.normal(0, 1e-2, cv.N), device="cuda")
        lam, _ = sysm.solve(rhs=2.0 * (u - target), transpose=True, rtol=1e-13)
        g = {k: v.cpu().numpy() for k, v in sysm.backward(u, lam).items()}
        results.append(g)
        xy, off, ids = cv.nodes()
        u_h, lam_h = u.cpu().numpy(), lam.cpu().numpy()
        for f, m in enumerate(ids):
            grid = spectral.local_grid(ref_cover.Nr[m], ref_cover.Ntheta[m])
            samples = spectral.node_samples(prob, grid, *ref_cover.centres[m], ref_cover.radii[m])
            ref = adjoint.circle_gradient(pc, m, samples, u_h, lam_h[pknot])
            for k in ("axx", "axy", "ayy", "bx", "by", "c", "f"):
                gg = g[k][off[f]:off[f + 1]]
                scale = np.max(np.abs(ref[k])) + 1e-300
                assert np.max(np.abs(gg - ref[k])) <= 1e-8 * scale, (budget, m, k)
    for k in results[0]:
        assert np.array_equal(results[0][k], results[1][k]), k
