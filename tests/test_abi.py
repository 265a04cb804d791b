"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and its host-side cover geometry matches the oracle's."""
import os
import re

import numpy as np
import pytest

import workloads
from oracle import geometry

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pdd = pytest.importorskip("paper_2311_08946_amd.binding")


def _lib_or_skip():
    try:
        return pdd.lib()
    except ImportError as e:
        pytest.skip(str(e))


def test_library_exports_every_declared_symbol():
    L = _lib_or_skip()
    header = open(os.path.join(ROOT, "include", "pdd.h")).read()
    declared = set(re.findall(r"\b(pdd_[a-z_A-Z0-9]+)\s*\(", header))
    assert declared, "no declarations found"
    assert declared == set(pdd.EXPORTED)
    for name in declared:
        assert hasattr(L, name), name


def _compare(cfg_cover, dom):
    ref = geometry.build_cover(dom, cfg_cover)
    cv = pdd.Cover(dom, cfg_cover)
    xy, rc, asg, own = cv.knots()
    assert cv.N == ref.N
    assert np.max(np.abs(xy - ref.knot_xy)) < 1e-15
    assert np.array_equal(rc, ref.row_class)
    assert np.array_equal(asg, ref.assigned)
    assert np.array_equal(own, ref.knot_owner)
    rowptr, cols = cv.pattern()
    assert np.array_equal(rowptr, ref.rowptr)
    assert np.array_equal(cols, ref.cols)
    return ref, cv


@pytest.mark.parametrize("name", ["config1", "small_variable"])
def test_cover_matches_oracle(name):
    _lib_or_skip()
    cfg = workloads.config1() if name == "config1" else workloads.small_variable()
    _compare(cfg["cover"], cfg["problem"]["domain"])


def test_cover_matches_oracle_config2_lattice():
    _lib_or_skip()
    cfg = workloads.config2()
    ref, cv = _compare(cfg["cover"], cfg["problem"]["domain"])
    assert int(cv.info.n_float) == 900 and int(cv.info.n_perim) == 124


def test_cover_matches_oracle_disk_with_hole():
    _lib_or_skip()
    dom = workloads.disk(0.0, 0.0, 1.0, holes=[(0.3, 0.0, 0.2)])
    cen = workloads.lattice_centres(14, 14, -1.05, 1.05, -1.05, 1.05)
    keep = (np.hypot(cen[:, 0], cen[:, 1]) - 0.12 < 1.0) & \
           (np.hypot(cen[:, 0] - 0.3, cen[:, 1]) + 0.12 > 0.2)
    cov = workloads._cover(cen[keep], np.full(keep.sum(), 0.12), 16, 16, 4)
    _compare(cov, dom)


def test_nodes_layout():
    _lib_or_skip()
    cfg = workloads.config1()
    cv = pdd.Cover(cfg["problem"]["domain"], cfg["cover"])
    xy, off, ids = cv.nodes()
    assert list(ids) == [5, 6, 9, 10]
    assert np.array_equal(off, np.arange(5) * 384)
    from oracle import spectral
    grid = spectral.local_grid(12, 32)
    for f, m in enumerate(ids):
        x, y = grid.node_xy(*cfg["cover"]["centres"][m], cfg["cover"]["radii"][m])
        assert np.max(np.abs(xy[off[f]:off[f + 1], 0] - x)) < 1e-15
        assert np.max(np.abs(xy[off[f]:off[f + 1], 1] - y)) < 1e-15


def test_invalid_covers_are_rejected():
    _lib_or_skip()
    cov = workloads._cover(np.array([[0.25, 0.5], [0.75, 0.5]]), np.array([0.3, 0.3]), 8, 8, 2)
    with pytest.raises(pdd.PddError) as e:
        pdd.Cover(workloads.box(), cov)
    assert e.value.code == pdd.PDD_ECOVER
    cov = workloads._cover(np.array([[0.5, 0.05]]), np.array([0.2]), 8, 8, 2)
    with pytest.raises(pdd.PddError) as e:
        pdd.Cover(workloads.box(0.0, 1.0, 0.0, 0.1), cov)
    assert e.value.code == pdd.PDD_ECOVER


@pytest.mark.parametrize("name", ["config1", "small_variable", "disk"])
def test_averaged_cover_matches_oracle(name):
    # rule AVERAGED (eqs. 38-39): the wider rows of every containing circle
    _lib_or_skip()
    if name == "disk":
        dom = workloads.disk(0.0, 0.0, 1.0, holes=[(0.3, 0.0, 0.2)])
        cen = workloads.lattice_centres(14, 14, -1.05, 1.05, -1.05, 1.05)
        keep = (np.hypot(cen[:, 0], cen[:, 1]) - 0.12 < 1.0) & \
               (np.hypot(cen[:, 0] - 0.3, cen[:, 1]) + 0.12 > 0.2)
        cov = workloads._cover(cen[keep], np.full(keep.sum(), 0.12), 16, 16, 4)
    else:
        cfg = workloads.config1() if name == "config1" else workloads.small_variable()
        dom, cov = cfg["problem"]["domain"], dict(cfg["cover"])
    cov["rule"] = geometry.RULE_AVERAGED
    ref, cv = _compare(cov, dom)
    assert int(cv.info.nnz) == len(ref.cols)


def test_unknown_rule_is_rejected():
    _lib_or_skip()
    cfg = workloads.config1()
    cov = dict(cfg["cover"])
    cov["rule"] = 3
    with pytest.raises(pdd.PddError) as e:
        pdd.Cover(cfg["problem"]["domain"], cov)
    assert e.value.code == pdd.PDD_EINVAL


def test_null_handles_are_rejected_without_device_work():
    # argument checks of the RAS and GMRES entry points happen on the host
    L = _lib_or_skip()
    import ctypes as C
    out = C.c_void_p()
    assert L.pdd_ras_build(None, None, None, C.byref(out)) == pdd.PDD_EINVAL
    assert out.value is None
    assert L.pdd_ras_get_parts(None, None, None, None) == pdd.PDD_EINVAL
    assert L.pdd_ras_apply(None, None, None, None) == pdd.PDD_EINVAL
    assert L.pdd_solve_gmres(None, None, None, None, None, None, None) == pdd.PDD_EINVAL
    assert b"null" in L.pdd_last_error()
    L.pdd_destroy_ras(None)


def test_header_is_plain_c():
    # the boundary is a C ABI: the public header compiles as C99 on its own
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pdd.h")
    r = subprocess.run([gcc, "-fsyntax-only", "-std=c99", "-Wall", "-Wextra", "-Werror", "-x", "c", hdr],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
