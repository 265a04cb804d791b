"""Shared checks of the GPU parity tests (imported by the test modules; holds
no tests).  Tolerances: floating rows per row max_j |dC_ij| <= 1e-10
max_j |C_ij|, r within 1e-10 (|r_i| + r_m^2 max |f|); Monte Carlo entries
within 3 of the oracle's standard errors."""
import sys

import numpy as np

from oracle import assemble, montecarlo, spectral
from oracle.geometry import ROW_MC

TOL_G = 1e-10


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _gpu_system(pdd, cfg, **kw):
    prob = cfg["problem"]
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"], **kw)
    val, b, se, se_b = (t.cpu().numpy() for t in sysm.copy())
    return cv, sysm, val, b, se, se_b


def _row(cover, vals, i):
    lo, hi = cover.rowptr[i], cover.rowptr[i + 1]
    return vals[lo:hi]


def _check_spectral_rows(ref_cover, ref_val, ref_b, val, b, rows, prob, samples=None):
    worst = 0.0
    for i in rows:
        g = _row(ref_cover, val, i)
        o = _row(ref_cover, ref_val, i)
        d = np.max(np.abs(g - o)) / np.max(np.abs(o))
        worst = max(worst, d)
        assert d <= TOL_G, (i, d)
    return worst


def _check_rhs(ref_cover, ref_b, b, rows, fscale):
    for i in rows:
        m = ref_cover.assigned[i]
        bound = TOL_G * (abs(ref_b[i]) + ref_cover.radii[m] ** 2 * fscale.get(m, 0.0))
        assert abs(b[i] - ref_b[i]) <= bound + 1e-300, (i, b[i], ref_b[i])


def _fscale(prob, cv, circles):
    out = {}
    for m in circles:
        grid = spectral.local_grid(cv.Nr[m], cv.Ntheta[m])
        s = spectral.node_samples(prob, grid, *cv.centres[m], cv.radii[m])
        out[m] = float(np.max(np.abs(s["f"])))
    return out


def _check_mc_rows(ref_cover, ref_val, ref_se, ref_b, ref_se_b, val, b, rows):
    """Every entry within 3 standard errors.  With identical Philox streams the
    path sums agree to rounding: r_i (a plain path average) must match to
    1e-9 on all but rare rows (an exit decided by the last ulp of a libm
    result).  C entries pass through K^-1 of the IMQ Gram matrix (condition
    about 1e11), which amplifies summation-order rounding to about 1e-5, so
    they are only held to the statistical bar."""
    close = 0
    for i in rows:
        g = _row(ref_cover, val, i)
        o = _row(ref_cover, ref_val, i)
        s = _row(ref_cover, ref_se, i)
        diff = np.abs(g - o)
        assert np.all(diff <= 3 * s + 1e-12), (i, np.max(diff / (s + 1e-300)))
        assert abs(b[i] - ref_b[i]) <= 3 * ref_se_b[i] + 1e-12
        close += int(abs(b[i] - ref_b[i]) <= 1e-9 * (1 + abs(ref_b[i])))
    return close / max(len(rows), 1)


def sampled_parity(prob, ref_cover, mc, val, b, circles, mc_knots):
    """Oracle rows of the given floating circles and Monte Carlo knots, one by
    one, against the GPU arrays; returns the fraction of MC rows whose r_i
    agrees to 1e-9."""
    fsc = _fscale(prob, ref_cover, circles)
    for m in circles:
        knots, Crows, rv = spectral.floating_rows(prob, ref_cover, m)
        ref_val = np.zeros(len(ref_cover.cols))
        ref_b = np.zeros(ref_cover.N)
        for t, i in enumerate(knots):
            assemble._put_row(ref_cover, ref_val, ref_val.copy(), i, m, Crows[t])
            ref_b[i] = rv[t]
        _check_spectral_rows(ref_cover, ref_val, ref_b, val, b, knots, prob)
        _check_rhs(ref_cover, ref_b, b, knots, fsc)
    if len(mc_knots) == 0:
        return 1.0
    knots, rows, ses, rv, se_r, steps = montecarlo.mc_rows(prob, ref_cover, mc, np.asarray(mc_knots))
    ref_val = np.zeros(len(ref_cover.cols))
    ref_se = np.zeros(len(ref_cover.cols))
    ref_b = np.zeros(ref_cover.N)
    ref_se_b = np.zeros(ref_cover.N)
    for t, i in enumerate(knots):
        assemble._put_row(ref_cover, ref_val, ref_se, i, ref_cover.assigned[i], rows[t], ses[t])
        ref_b[i] = rv[t]
        ref_se_b[i] = se_r[t]
    return _check_mc_rows(ref_cover, ref_val, ref_se, ref_b, ref_se_b, val, b, knots)


def pick_mc_knots(ref_cover, rng, k):
    cand = np.nonzero(ref_cover.row_class == ROW_MC)[0]
    return rng.choice(cand, size=min(k, len(cand)), replace=False)


COEFS = ("axx", "axy", "ayy", "bx", "by", "c")
GRAD_REL = 1e-8


def gradient_terms(ref_cover, m, samples, u, lam):
    """Oracle adjoint of floating circle m and the rounding scale of each
    gradient entry.  Entry q of a coefficient's gradient is
    -mu_q (Op[q, :] . w), a dot product of an operator row with the local
    solution w.  On small circles the second-derivative rows are large
    (about (2 Nr + 1)^4 / r^2) while the result is small, so the dot product
    cancels: an error e in w moves it by up to |Op[q, :]| . |w| * e.  Both
    sides solve for w with LU, so e is about cond(A_II) times the unit
    round-off; the allowance per entry is 4 cond(A_II) eps |mu_q|
    (|Op[q, :]| . |w|)."""
    from oracle import adjoint, spectral
    mu, w, ops = adjoint.circle_terms(ref_cover, m, samples, u, lam)
    grid = spectral.local_grid(ref_cover.Nr[m], ref_cover.Ntheta[m])
    A_II, _ = grid.collocation(float(ref_cover.radii[m]), samples)
    tau = 4.0 * np.linalg.cond(A_II) * np.finfo(np.float64).eps
    ref, slack = {}, {}
    for k in COEFS:
        ref[k] = -mu * (ops[k] @ w)
        slack[k] = tau * np.abs(mu) * (np.abs(ops[k]) @ np.abs(w))
    ref["f"] = -mu
    slack["f"] = np.zeros_like(mu)
    return ref, slack


def check_circle_gradient(ref, slack, g_gpu):
    """GPU gradients of one circle (dict of node-layout slices) against the
    oracle's: |dg_q| <= 1e-8 max_q |g_q| + slack_q (see gradient_terms)."""
    for k, r in ref.items():
        bound = GRAD_REL * np.max(np.abs(r)) + slack[k]
        d = np.abs(g_gpu[k] - r)
        assert np.all(d <= bound), (k, float(np.max(d / (bound + 1e-300))))
