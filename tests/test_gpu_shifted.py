"""GPU parity of the boundary-shifted Euler scheme (Gobet-Menozzi, the paper's
ref. [15]) against the oracle: the same Philox streams, so the Monte Carlo
rows agree as in the plain scheme's parity (every entry within 3 standard
errors, r_i to 1e-9 on all but rare rows), the path-step totals agree, and
the floating rows are untouched."""
import numpy as np
import pytest

import workloads
from oracle import assemble, geometry
from oracle.geometry import ROW_MC, ROW_SPECTRAL

from helpers_parity import _check_mc_rows, _check_spectral_rows, _gpu_system, _say

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_08946_amd.binding as pdd
    pdd.lib()
    return pdd


@pytest.mark.parametrize("name", ["config1", "small_variable", "disk", "config1_averaged"])
def test_shifted_rows_match_oracle(name):
    pdd = _gpu()
    if name == "config1":
        cfg = workloads.config1(paths=256)
    elif name == "config1_averaged":           # the paper's combination: averaged rows, shifted scheme
        cfg = workloads.config1(paths=256)
        cfg["cover"] = dict(cfg["cover"])
        cfg["cover"]["rule"] = 2
    elif name == "small_variable":
        cfg = workloads.small_variable(paths=128)
    else:                                      # unit disk minus a hole: circle pieces of both kinds
        dom = workloads.disk(0.0, 0.0, 1.0, holes=[(0.3, 0.0, 0.2)])
        cen = workloads.lattice_centres(14, 14, -1.05, 1.05, -1.05, 1.05)
        keep = (np.hypot(cen[:, 0], cen[:, 1]) - 0.12 < 1.0) & \
               (np.hypot(cen[:, 0] - 0.3, cen[:, 1]) + 0.12 > 0.2)
        g = workloads.degenerate("no_floating")["problem"]["g"]
        cfg = {"problem": workloads.laplace_problem(dom, g),
               "cover": workloads._cover(cen[keep], np.full(keep.sum(), 0.12), 16, 16, 4),
               "mc": workloads.mc_opts(64, 1e-3, seed=5)}
    cfg["mc"] = dict(cfg["mc"])
    cfg["mc"]["scheme"] = 1
    prob = cfg["problem"]
    _say(f"[gpu] shifted scheme {name}")
    cv, sysm, val, b, se, se_b = _gpu_system(pdd, cfg)
    assert sysm.stats.capped_paths == 0
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    ref = assemble.assemble(prob, ref_cover, cfg["mc"])
    assert abs(sysm.stats.path_steps - ref.path_steps) <= 1e-4 * ref.path_steps
    plain = dict(cfg["mc"])
    plain["scheme"] = 0
    sys0 = pdd.System(cv, prob, plain)
    assert sysm.stats.path_steps < sys0.stats.path_steps     # paths stop earlier
    if ref_cover.containers is not None:
        # averaged rows: each row against the oracle's, entries within 3 standard errors
        # plus 1e-10 of the row's largest entry, r_i to 1e-9 on all but rare rows
        close = n_mc = 0
        for i in range(ref_cover.N):
            sl = slice(ref_cover.rowptr[i], ref_cover.rowptr[i + 1])
            o = ref.val[sl]
            assert np.all(np.abs(val[sl] - o) <= 3 * ref.se[sl] + 1e-10 * np.max(np.abs(o))), i
            assert abs(b[i] - ref.b[i]) <= 3 * ref.se_b[i] + 1e-10 * (abs(ref.b[i]) + 1), i
            if ref.se_b[i] > 0:
                n_mc += 1
                close += int(abs(b[i] - ref.b[i]) <= 1e-9 * (1 + abs(ref.b[i])))
        frac = close / max(n_mc, 1)
        assert frac > 0.99
    else:
        mcr = np.nonzero(ref_cover.row_class == ROW_MC)[0]
        frac = _check_mc_rows(ref_cover, ref.val, ref.se, ref.b, ref.se_b, val, b, mcr)
        assert frac > 0.99
        spec = np.nonzero(ref_cover.row_class == ROW_SPECTRAL)[0]
        if len(spec):
            _check_spectral_rows(ref_cover, ref.val, ref.b, val, b, spec, prob)
    _say(f"[gpu] {name}: {sysm.stats.path_steps} path steps (plain {sys0.stats.path_steps}), "
         f"MC r_i within 1e-9: {frac:.4f}")
