"""Pins for the oracle's cover, knots, stencils and row choice (Section 2.1,
eqs. 4-12; Section 3.2)."""
import math

import numpy as np
import pytest

import workloads
from oracle import geometry
from oracle.geometry import ROW_BOUNDARY, ROW_MC, ROW_SPECTRAL, CoverError


@pytest.fixture(scope="module")
def c1():
    cfg = workloads.config1()
    return cfg, geometry.build_cover(cfg["problem"]["domain"], cfg["cover"])


def test_config1_counts(c1):
    cfg, cv = c1
    assert cv.floating.sum() == 4 and (~cv.floating).sum() == 12
    assert np.array_equal(np.nonzero(cv.floating)[0], [5, 6, 9, 10])
    for m in np.nonzero(cv.floating)[0]:
        assert cv.knot_off[m + 1] - cv.knot_off[m] == 32
    assert cv.knot_boundary.sum() == 24          # two junctions per perimeter circle


def test_corner_arc_matches_analytic_crossings(c1):
    cfg, cv = c1
    # circle 0: centre (0.05, 0.05), r = 0.25 meets y = 0 and x = 0 at
    # distance sqrt(0.25^2 - 0.05^2) from the foot of the perpendicular
    t0, t1 = cv.arc[0]
    d = math.sqrt(0.25 ** 2 - 0.05 ** 2)
    p0 = (0.05 + 0.25 * math.cos(t0), 0.05 + 0.25 * math.sin(t0))
    p1 = (0.05 + 0.25 * math.cos(t1), 0.05 + 0.25 * math.sin(t1))
    assert abs(p0[0] - (0.05 + d)) < 1e-14 and abs(p0[1]) < 1e-14
    assert abs(p1[0]) < 1e-14 and abs(p1[1] - (0.05 + d)) < 1e-14


def test_knots_lie_on_their_circles_and_junctions_on_boundary(c1):
    cfg, cv = c1
    dom = cfg["problem"]["domain"]
    own = cv.knot_owner
    dist = np.hypot(cv.knot_xy[:, 0] - cv.centres[own, 0], cv.knot_xy[:, 1] - cv.centres[own, 1])
    assert np.max(np.abs(dist - cv.radii[own])) < 1e-15
    sd = geometry.signed_distance(dom, cv.knot_xy[:, 0], cv.knot_xy[:, 1])
    assert np.max(np.abs(sd[cv.knot_boundary])) < 1e-15
    assert np.all(sd[~cv.knot_boundary] > 1e-9)
    # local angles increase along each stencil (eq. 12)
    for m in range(len(cv.radii)):
        th = cv.knot_theta[cv.knot_off[m]:cv.knot_off[m + 1]]
        assert np.all(np.diff(th) > 0)


def test_row_choice_against_brute_force(c1):
    cfg, cv = c1
    for i in range(cv.N):
        if cv.knot_boundary[i]:
            assert cv.row_class[i] == ROW_BOUNDARY
            continue
        x = cv.knot_xy[i]
        depth = cv.radii - np.hypot(*(x - cv.centres).T)
        depth[cv.knot_owner[i]] = -1.0
        flo = np.where(cv.floating & (depth > 0), depth, -np.inf)
        if np.isfinite(flo).any():
            assert cv.row_class[i] == ROW_SPECTRAL
            assert cv.assigned[i] == int(np.argmax(flo))
        else:
            per = np.where(~cv.floating & (depth > 0), depth, -np.inf)
            assert cv.row_class[i] == ROW_MC
            assert cv.assigned[i] == int(np.argmax(per))


def test_csr_rows(c1):
    cfg, cv = c1
    for i in range(cv.N):
        cols = cv.cols[cv.rowptr[i]:cv.rowptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
        if cv.row_class[i] != ROW_BOUNDARY:
            m = cv.assigned[i]
            assert len(cols) == 1 + cv.knot_off[m + 1] - cv.knot_off[m]


def test_disk_with_hole_cover_is_valid():
    dom = workloads.disk(0.0, 0.0, 1.0, holes=[(0.3, 0.0, 0.2)])
    cen = workloads.lattice_centres(14, 14, -1.05, 1.05, -1.05, 1.05)
    keep = (np.hypot(cen[:, 0], cen[:, 1]) - 0.12 < 1.0) & (np.hypot(cen[:, 0] - 0.3, cen[:, 1]) + 0.12 > 0.2)
    cov = workloads._cover(cen[keep], np.full(keep.sum(), 0.12), 16, 16, 4)
    cv = geometry.build_cover(dom, cov)
    sd = geometry.signed_distance(dom, cv.knot_xy[:, 0], cv.knot_xy[:, 1])
    assert np.max(np.abs(sd[cv.knot_boundary])) < 1e-14
    assert cv.floating.any() and (~cv.floating).any()


def test_uncovered_knot_is_rejected():
    cov = workloads._cover(np.array([[0.25, 0.5], [0.75, 0.5]]), np.array([0.3, 0.3]), 8, 8, 2)
    with pytest.raises(CoverError):
        geometry.build_cover(workloads.box(), cov)


def test_two_arc_interface_is_rejected():
    dom = workloads.box(0.0, 1.0, 0.0, 0.1)
    cov = workloads._cover(np.array([[0.5, 0.05]]), np.array([0.2]), 8, 8, 2)
    with pytest.raises(CoverError):
        geometry.build_cover(dom, cov)
