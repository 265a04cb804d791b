"""GPU parity of the RAS preconditioner and GMRES (Section 4, eqs. 42-45)
against the oracle.

The oracle is run on the GPU's own assembled C (copied to the host), so the
comparison isolates the solver.  Bars: the parts omega_p are identical
(integer lists); M^-1 x within 1e-10 of max |M^-1 x| (the device keeps
explicit inverses, the oracle LU factors); GMRES converges, its solution is
within 1e-9 of the direct solve's largest entry, and its iteration count is
within 2 of the oracle's (classical Gram-Schmidt twice on the device,
modified Gram-Schmidt in the oracle: equal in exact arithmetic).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import geometry, ras
from oracle.geometry import RULE_AVERAGED

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_08946_amd.binding as pdd
    pdd.lib()
    return pdd, torch


def _case(name):
    if name == "config1":
        return workloads.config1(paths=128)
    if name == "small_variable":
        return workloads.small_variable(paths=128)
    if name == "disk_hole":                     # unit disk minus a hole, 14 x 14 lattice
        dom = workloads.disk(0.0, 0.0, 1.0, holes=[(0.3, 0.0, 0.2)])
        cen = workloads.lattice_centres(14, 14, -1.05, 1.05, -1.05, 1.05)
        keep = (np.hypot(cen[:, 0], cen[:, 1]) - 0.12 < 1.0) & \
               (np.hypot(cen[:, 0] - 0.3, cen[:, 1]) + 0.12 > 0.2)
        g = workloads.degenerate("no_floating")["problem"]["g"]
        return {"problem": workloads.laplace_problem(dom, g),
                "cover": workloads._cover(cen[keep], np.full(keep.sum(), 0.12), 16, 16, 4),
                "mc": workloads.mc_opts(64, 1e-3, seed=5)}
    cfg = workloads.config1(paths=128)
    cfg["cover"] = dict(cfg["cover"])
    cfg["cover"]["rule"] = RULE_AVERAGED
    return cfg


def _system(pdd, cfg):
    prob = cfg["problem"]
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"])
    val, b, _, _ = (t.cpu().numpy() for t in sysm.copy())
    rowptr, cols = cv.pattern()
    C = sp.csr_matrix((val, cols, rowptr), shape=(cv.N, cv.N))
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    return cv, sysm, C, b, ref_cover


@pytest.mark.parametrize("name,parts", [("config1", (2, 2)), ("small_variable", (2, 2)),
                                        ("config1_averaged", (2, 2)), ("config1", (4, 1)),
                                        ("disk_hole", (3, 2))])
def test_ras_matches_oracle(name, parts):
    pdd, torch = _gpu()
    cfg = _case(name)
    _say(f"[gpu] ras {name} {parts}")
    cv, sysm, C, b, ref_cover = _system(pdd, cfg)
    R = pdd.Ras(sysm, *parts)
    omegas, _ = ras.subdomains(ref_cover, *parts)
    got = R.parts()
    assert len(got) == len(omegas)
    for g, o in zip(got, omegas):
        assert np.array_equal(g, o)
    M = ras.RAS(C, ref_cover, *parts)
    x = np.random.default_rng(3).standard_normal(cv.N)
    y = R.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    y_ref = M.apply(x)
    assert np.max(np.abs(y - y_ref)) <= 1e-10 * np.max(np.abs(y_ref))
    u_ref = spla.spsolve(sp.csc_matrix(C), b)
    for prec, Mo in ((R, M), (None, None)):
        u, info = sysm.solve_gmres(prec, rtol=1e-11, restart=30)
        assert info.converged
        u = u.cpu().numpy()
        assert np.max(np.abs(u - u_ref)) <= 1e-9 * np.max(np.abs(u_ref))
        _, it_ref, _ = ras.gmres(C, b, Mo, rtol=1e-11, restart=30)
        assert abs(info.iterations - it_ref) <= 2, (info.iterations, it_ref)
        _say(f"[gpu] {name} {'RAS' if prec else 'none'}: {info.iterations} GMRES iterations "
             f"(oracle {it_ref})")


def test_ras_on_the_benchmark_lattice():
    # 32 x 32 circles (900 floating), 8 x 8 parts of at most 2304 knots
    pdd, torch = _gpu()
    cfg = workloads.config2(paths=1000)
    prob = cfg["problem"]
    _say("[gpu] ras on the 32x32 lattice")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"])
    with pytest.raises(pdd.PddError) as e:
        pdd.Ras(sysm, 1, 1)            # one part of every knot: above the 4096 limit
    assert e.value.code == pdd.PDD_EINVAL
    R = pdd.Ras(sysm, 8, 8)
    u_b, info_b = sysm.solve(rtol=1e-12)
    u_r, info_r = sysm.solve_gmres(R, rtol=1e-12, restart=30)
    u_n, info_n = sysm.solve_gmres(None, rtol=1e-12, restart=30)
    assert info_b.converged and info_r.converged and info_n.converged
    scale = float(torch.max(torch.abs(u_b)))
    assert float(torch.max(torch.abs(u_r - u_b))) <= 1e-9 * scale
    assert float(torch.max(torch.abs(u_n - u_b))) <= 1e-9 * scale
    assert info_r.iterations < info_n.iterations
    _say(f"[gpu] 32x32: GMRES+RAS {info_r.iterations}, GMRES {info_n.iterations}, "
         f"BiCGStab {info_b.iterations} iterations")


@pytest.mark.parametrize("name", ["config1", "small_variable"])
def test_fp32_inverses(name):
    # Inverses rounded to FP32: each entry moves by at most 2^-24 of itself, so
    # |dy_i| <= 2^-24 sum_p D_ii sum_c |(C_p^-1)_rc| |x_c| (bound doubled below);
    # GMRES with the preconditioner on the right still meets the FP64 tolerance.
    pdd, torch = _gpu()
    cfg = _case(name)
    _say(f"[gpu] ras fp32 inverses {name}")
    cv, sysm, C, b, ref_cover = _system(pdd, cfg)
    R32 = pdd.Ras(sysm, 2, 2, fp32_inverses=True)
    omegas, D = ras.subdomains(ref_cover, 2, 2)
    x = np.random.default_rng(4).standard_normal(cv.N)
    y = R32.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    y_ref = ras.RAS(C, ref_cover, 2, 2).apply(x)
    bound = np.zeros(cv.N)
    for w, d in zip(omegas, D):
        Xp = np.linalg.inv(C[w][:, w].toarray())
        bound[w] += d * (np.abs(Xp) @ np.abs(x[w]))
    bound = 2.0 ** -23 * bound + 1e-12 * np.max(np.abs(y_ref))
    assert np.all(np.abs(y - y_ref) <= bound), float(np.max(np.abs(y - y_ref) / bound))
    u, info = sysm.solve_gmres(R32, rtol=1e-11)
    assert info.converged
    u_ref = spla.spsolve(sp.csc_matrix(C), b)
    assert np.max(np.abs(u.cpu().numpy() - u_ref)) <= 1e-9 * np.max(np.abs(u_ref))
    _say(f"[gpu] {name} fp32 RAS: {info.iterations} GMRES iterations")


def test_one_part_is_a_direct_solve():
    # one part: omega = every knot, M^-1 = C^-1 (eq. 44 with R = I); GMRES stops
    # after one iteration at the direct solution
    pdd, torch = _gpu()
    cfg = _case("config1")
    _say("[gpu] ras one part")
    cv, sysm, C, b, ref_cover = _system(pdd, cfg)
    R = pdd.Ras(sysm, 1, 1)
    assert len(R.parts()) == 1 and np.array_equal(R.parts()[0], np.arange(cv.N))
    x = np.random.default_rng(6).standard_normal(cv.N)
    y = R.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    ref = spla.spsolve(sp.csc_matrix(C), x)
    assert np.max(np.abs(y - ref)) <= 1e-11 * np.max(np.abs(ref))
    u, info = sysm.solve_gmres(R, rtol=1e-12)
    assert info.converged and info.iterations == 1
    u_ref = spla.spsolve(sp.csc_matrix(C), b)
    assert np.max(np.abs(u.cpu().numpy() - u_ref)) <= 1e-11 * np.max(np.abs(u_ref))
