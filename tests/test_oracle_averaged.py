"""Pins for the oracle's averaged rows (eqs. 38-39): every circle containing a
knot contributes its own expectation row, C_ii counts them.

* the CSR pattern of row i is the knot and the stencils of exactly the circles
  whose open disc holds x_i (brute force over every circle);
* a knot inside a single circle gets the row of the default rule unchanged;
* on a harmonic solution (Laplace, g = Re of a polynomial) every row built
  only from floating circles vanishes to rounding, which needs the diagonal
  count, the placement of every pair's entries and the summed r_i all right;
* the adjoint of the averaged assembly agrees with central differences of the
  loss through full re-assembly.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import adjoint, assemble, fields, geometry
from oracle.geometry import ROW_BOUNDARY, RULE_AVERAGED


def _averaged(cfg):
    cov = dict(cfg["cover"])
    cov["rule"] = RULE_AVERAGED
    return geometry.build_cover(cfg["problem"]["domain"], cov)


@pytest.fixture(scope="module")
def c1_pair():
    cfg = workloads.config1(paths=64)
    prob = cfg["problem"]
    c0 = geometry.build_cover(prob["domain"], cfg["cover"])
    c2 = _averaged(cfg)
    s0 = assemble.assemble(prob, c0, cfg["mc"], with_mc=False)
    s2 = assemble.assemble(prob, c2, cfg["mc"], with_mc=False)
    return cfg, c0, c2, s0, s2


def test_pattern_is_the_union_of_containing_stencils(c1_pair):
    cfg, c0, c2, s0, s2 = c1_pair
    assert np.array_equal(c0.knot_xy, c2.knot_xy)
    assert np.array_equal(c0.row_class, c2.row_class)
    for i in range(c2.N):
        cols = c2.cols[c2.rowptr[i]:c2.rowptr[i + 1]]
        if c2.row_class[i] == ROW_BOUNDARY:
            assert list(cols) == [i]
            continue
        x, y = c2.knot_xy[i]
        inside = [m for m in range(len(c2.radii))
                  if c2.radii[m] - math.hypot(x - c2.centres[m][0], y - c2.centres[m][1])
                  > 1e-9 * c2.radii[m]]
        assert inside == list(c2.containers[i])
        want = {i}
        for m in inside:
            want |= set(range(c2.knot_off[m], c2.knot_off[m + 1]))
        assert list(cols) == sorted(want)
    # bandwidth grows by the extra stencils only
    assert len(c2.cols) > len(c0.cols)


def test_single_container_rows_equal_the_default_rule(c1_pair):
    cfg, c0, c2, s0, s2 = c1_pair
    one = [i for i in range(c2.N) if c2.row_class[i] != ROW_BOUNDARY
           and len(c2.containers[i]) == 1 and c2.floating[c2.containers[i][0]]]
    assert len(one) > 10
    for i in one:
        a = slice(c0.rowptr[i], c0.rowptr[i + 1])
        b = slice(c2.rowptr[i], c2.rowptr[i + 1])
        assert np.array_equal(c0.cols[a], c2.cols[b])
        assert np.array_equal(s0.val[a], s2.val[b])
        assert s0.b[i] == s2.b[i]


def test_floating_rows_vanish_on_a_harmonic_solution(c1_pair):
    cfg, c0, c2, s0, s2 = c1_pair
    prob = cfg["problem"]
    u = fields.value(prob["g"], c2.knot_xy[:, 0], c2.knot_xy[:, 1], prob)
    rows = [i for i in range(c2.N) if c2.row_class[i] != ROW_BOUNDARY
            and all(c2.floating[m] for m in c2.containers[i])]
    multi = [i for i in rows if len(c2.containers[i]) > 1]
    assert len(multi) > 10
    scale = np.max(np.abs(u))
    for i in rows:
        sl = slice(c2.rowptr[i], c2.rowptr[i + 1])
        cols, v = c2.cols[sl], s2.val[sl]
        d = list(cols).index(i)
        assert v[d] == float(len(c2.containers[i]))
        res = float(v @ u[cols]) - s2.b[i]
        assert abs(res) <= 1e-10 * scale, (i, res)


def test_averaged_adjoint_matches_central_differences():
    cfg = workloads.small_variable(paths=64)
    prob = cfg["problem"]
    cv = _averaged(cfg)
    from oracle import spectral
    samples = {}
    for m in np.nonzero(cv.floating)[0]:
        grid = spectral.local_grid(cv.Nr[m], cv.Ntheta[m])
        samples[m] = spectral.node_samples(prob, grid, *cv.centres[m], cv.radii[m])
    sysm = assemble.assemble(prob, cv, cfg["mc"], samples=samples)
    ue = fields.value(prob["u_exact"], cv.knot_xy[:, 0], cv.knot_xy[:, 1])
    target = ue + np.random.default_rng(0).normal(0, 1e-3, cv.N)
    L, grads, lam, u = adjoint.gradient(prob, cv, sysm, samples, target)
    names = ["axx", "axy", "ayy", "bx", "by", "c", "f"]
    gmax = max(np.max(np.abs(g[k])) for g in grads.values() for k in names)
    rng = np.random.default_rng(3)
    fl = list(samples)
    for _ in range(5):
        m = fl[rng.integers(len(fl))]
        name = names[rng.integers(len(names))]
        q = int(rng.integers(len(samples[m][name])))
        eps = 1e-5 * max(1.0, abs(samples[m][name][q]))

        def loss(sign):
            s = dict(samples)
            s[m] = {k: v.copy() for k, v in samples[m].items()}
            s[m][name][q] += sign * eps
            return adjoint.loss_sq(assemble.solve(assemble.assemble(prob, cv, cfg["mc"], samples=s)),
                                   target)

        fd = (loss(+1) - loss(-1)) / (2 * eps)
        ga = grads[m][name][q]
        assert abs(fd - ga) <= 1e-5 * abs(ga) + 1e-8 * gmax, (m, name, q, fd, ga)
