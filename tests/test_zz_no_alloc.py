"""GPU check of pdd_solve_G_noalloc (the BiCGStab solve whose work area is
the library's static device memory) against pdd_solve_G, through the C ABI:
two calls in a row, the second on a smaller system, on C and on C^T."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_08946_amd.binding as pdd
    pdd.lib()
    return pdd, torch


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _solve(pdd, torch, entry, sysm, rhs, transpose, rtol=1e-13):
    u = torch.zeros(sysm.cover.N, dtype=torch.float64, device="cuda")
    so = pdd.SolveOpts(rtol, 2000, 0)
    info = pdd.SolveInfo()
    code = getattr(pdd.lib(), entry)(sysm.handle, pdd._tptr(rhs), pdd._tptr(u), int(transpose), C.byref(so),
                                     pdd._stream_ptr(None), C.byref(info))
    pdd._check(code, entry + ": ")
    torch.cuda.synchronize()
    return u, info


def test_noalloc_solve_matches_solve_on_two_calls():
    pdd, torch = _gpu()
    systems = []
    for name, cfg in (("config1", workloads.config1()), ("small_variable", workloads.small_variable(paths=128))):
        prob = cfg["problem"]
        cv = pdd.Cover(prob["domain"], cfg["cover"])
        systems.append((name, cv, pdd.System(cv, prob, cfg["mc"])))
    assert systems[1][1].N < systems[0][1].N
    for name, cv, sysm in systems:
        _say(f"[gpu] noalloc solve, {name}, N={cv.N}")
        u_ref, i_ref = _solve(pdd, torch, "pdd_solve_G", sysm, None, 0)
        u, info = _solve(pdd, torch, "pdd_solve_G_noalloc", sysm, None, 0)
        assert info.converged and info.iterations == i_ref.iterations
        assert np.max(np.abs((u - u_ref).cpu().numpy())) <= 1e-10 * float(torch.max(torch.abs(u_ref)))
        assert torch.equal(u, u_ref)          # the same kernels in the same order
        g = torch.tensor(np.random.default_rng(3).standard_normal(cv.N), device="cuda")
        lam_ref, it_ref = _solve(pdd, torch, "pdd_solve_G", sysm, g, 1)
        lam, it = _solve(pdd, torch, "pdd_solve_G_noalloc", sysm, g, 1)
        assert it.converged and it.iterations == it_ref.iterations
        assert torch.equal(lam, lam_ref)


def test_noalloc_transpose_needs_formed_transpose():
    pdd, torch = _gpu()
    cfg = workloads.config1()
    prob = cfg["problem"]
    _say("[gpu] noalloc transpose before C^T exists")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"])
    with pytest.raises(pdd.PddError) as e:
        _solve(pdd, torch, "pdd_solve_G_noalloc", sysm, None, 1)
    assert e.value.code == pdd.PDD_EINVAL
