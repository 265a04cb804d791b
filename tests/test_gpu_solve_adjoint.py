"""GPU parity of solve_G (BiCGStab on C and C^T) and of the adjoint
assemble_G_backward against the oracle, plus central differences through the
library and the torch.autograd.Function."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import adjoint, geometry, spectral

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


def _host_matrix(cv, val):
    rowptr, cols = cv.pattern()
    return sp.csr_matrix((val, cols, rowptr), shape=(cv.N, cv.N))


@pytest.mark.parametrize("name", ["config1", "small_variable"])
def test_solve_matches_direct_solve(name):
    pdd, torch = _gpu()
    cfg = workloads.config1() if name == "config1" else workloads.small_variable(paths=128)
    prob = cfg["problem"]
    _say(f"[gpu] solve {name}")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"])
    val, b, _, _ = (t.cpu().numpy() for t in sysm.copy())
    A = sp.csc_matrix(_host_matrix(cv, val))
    u_ref = spla.splu(A).solve(b)
    u, info = sysm.solve(rtol=1e-13)
    assert info.converged
    u = u.cpu().numpy()
    assert np.max(np.abs(u - u_ref)) <= 1e-10 * np.max(np.abs(u_ref))
    g = np.random.default_rng(1).standard_normal(cv.N)
    lam, info_t = sysm.solve(rhs=torch.tensor(g, device="cuda"), transpose=True, rtol=1e-13)
    lam_ref = spla.splu(sp.csc_matrix(A.T)).solve(g)
    assert np.max(np.abs(lam.cpu().numpy() - lam_ref)) <= 1e-10 * np.max(np.abs(lam_ref))
    _say(f"[gpu] {name}: {info.iterations} / {info_t.iterations} BiCGStab iterations")


@pytest.mark.parametrize("name", ["config1", "small_variable", "no_floating"])
def test_direct_small_matches_direct_solve(name):
    # PDD_SOLVE_DIRECT_SMALL: dense LU of [C | r] on the device (one matrix of
    # the batched LU) against scipy's sparse LU, on C and on C^T
    pdd, torch = _gpu()
    cfg = {"config1": workloads.config1, "no_floating": lambda: workloads.degenerate("no_floating"),
           "small_variable": lambda: workloads.small_variable(paths=128)}[name]()
    prob = cfg["problem"]
    _say(f"[gpu] direct solve {name}")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"])
    val, b, _, _ = (t.cpu().numpy() for t in sysm.copy())
    A = sp.csc_matrix(_host_matrix(cv, val))
    u_ref = spla.splu(A).solve(b)
    u, info = sysm.solve(method="direct")
    assert info.converged and info.iterations == 1 and info.rel_residual < 1e-13
    assert np.max(np.abs(u.cpu().numpy() - u_ref)) <= 1e-12 * np.max(np.abs(u_ref))
    g = np.random.default_rng(2).standard_normal(cv.N)
    lam, info_t = sysm.solve(rhs=torch.tensor(g, device="cuda"), transpose=True, method="direct")
    lam_ref = spla.splu(sp.csc_matrix(A.T)).solve(g)
    assert info_t.converged and info_t.rel_residual < 1e-13
    assert np.max(np.abs(lam.cpu().numpy() - lam_ref)) <= 1e-12 * np.max(np.abs(lam_ref))


def _setup_variable():
    cfg = workloads.small_variable(paths=64)
    prob = cfg["problem"]
    return cfg, prob


def test_adjoint_matches_oracle_adjoint():
    pdd, torch = _gpu()
    cfg, prob = _setup_variable()
    _say("[gpu] adjoint vs oracle")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"], keep_factors=True)
    u, _ = sysm.solve(rtol=1e-13)
    rng = np.random.default_rng(5)
    target = torch.tensor(u.cpu().numpy() + rng.normal(0, 1e-2, cv.N), device="cuda")
    lam, _ = sysm.solve(rhs=2.0 * (u - target), transpose=True, rtol=1e-13)
    g = {k: v.cpu().numpy() for k, v in sysm.backward(u, lam, names=("axx", "axy", "ayy", "bx", "by", "c",
                                                                       "f", "r")).items()}
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    xy, off, ids = cv.nodes()
    u_h, lam_h = u.cpu().numpy(), lam.cpu().numpy()
    assert np.array_equal(g["r"], lam_h)          # dL/dr = lambda (r enters C u = r linearly)
    for f, m in enumerate(ids):
        grid = spectral.local_grid(ref_cover.Nr[m], ref_cover.Ntheta[m])
        samples = spectral.node_samples(prob, grid, *ref_cover.centres[m], ref_cover.radii[m])
        ref = adjoint.circle_gradient(ref_cover, m, samples, u_h, lam_h)
        for k in ("axx", "axy", "ayy", "bx", "by", "c", "f"):
            gg = g[k][off[f]:off[f + 1]]
            scale = np.max(np.abs(ref[k])) + 1e-300
            assert np.max(np.abs(gg - ref[k])) <= 1e-8 * scale, (m, k, np.max(np.abs(gg - ref[k])) / scale)


def test_adjoint_matches_central_differences_through_the_library():
    pdd, torch = _gpu()
    from paper_2311_08946_amd import autograd as pag
    cfg, prob = _setup_variable()
    _say("[gpu] adjoint vs central differences")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    samples = pag.node_samples(cv, prob)
    rng = np.random.default_rng(7)
    target = None

    def loss_host(s):
        sysm = pdd.System(cv, prob, cfg["mc"], samples=s)
        val, b, _, _ = (t.cpu().numpy() for t in sysm.copy())
        u = spla.splu(sp.csc_matrix(_host_matrix(cv, val))).solve(b)
        return float(np.sum((u - target) ** 2))

    leaves = {k: v.clone().requires_grad_(True) for k, v in samples.items()}
    u = pag.solve(leaves, cv, prob, cfg["mc"], rtol=1e-13)
    target = u.detach().cpu().numpy() + rng.normal(0, 1e-2, cv.N)
    loss = torch.sum((u - torch.tensor(target, device="cuda")) ** 2)
    loss.backward()
    grads = {k: v.grad.cpu().numpy() for k, v in leaves.items()}
    gmax = max(np.max(np.abs(g)) for g in grads.values())
    n = len(samples["axx"])
    for t in range(16):
        k = list(grads)[t % 7]
        q = int(rng.integers(n))
        base = samples[k][q].item()
        eps = 1e-5 * max(1.0, abs(base))
        s_p = {kk: vv.clone() for kk, vv in samples.items()}
        s_m = {kk: vv.clone() for kk, vv in samples.items()}
        s_p[k][q] += eps
        s_m[k][q] -= eps
        fd = (loss_host(s_p) - loss_host(s_m)) / (2 * eps)
        ga = grads[k][q]
        assert abs(fd - ga) <= 1e-5 * abs(ga) + 1e-8 * gmax, (k, q, fd, ga)


def test_chunked_factor_recompute_matches_stored_factors():
    """With keep_factors and an HBM budget smaller than the factors, the
    system keeps the node samples and the backward pass rebuilds the factors
    chunk by chunk: assembly and gradients are bitwise those of the stored-
    factor path (same kernels on the same inputs)."""
    pdd, torch = _gpu()
    cfg, prob = _setup_variable()
    _say("[gpu] chunked factor recompute")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    s1 = pdd.System(cv, prob, cfg["mc"], keep_factors=True)
    assert s1.stats.recompute == 0 and s1.stats.factor_bytes > 0
    per = s1.stats.factor_bytes // cv.info.n_float
    s2 = pdd.System(cv, prob, cfg["mc"], keep_factors=True, hbm_budget_bytes=int(1.5 * per))
    assert s2.stats.recompute == 1 and s2.stats.factor_bytes == 0
    for a, b in zip(s1.copy(), s2.copy()):
        assert torch.equal(a, b)
    u, _ = s1.solve(rtol=1e-13)
    rng = np.random.default_rng(11)
    lam = torch.tensor(rng.standard_normal(cv.N), device="cuda")
    g1 = s1.backward(u, lam)
    g2 = s2.backward(u, lam)
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k


@pytest.mark.parametrize("rule", [0, 2])
def test_system_csr_matches_pattern_and_values(rule):
    # pdd_system_csr: the CSR of C and r in one call, equal to the host
    # pattern and to pdd_system_copy (rule 2: the averaged rows of eqs. 38-39)
    pdd, torch = _gpu()
    cfg = workloads.config1(paths=64)
    prob = cfg["problem"]
    cov = dict(cfg["cover"], rule=rule)
    _say(f"[gpu] system_csr rule {rule}")
    cv = pdd.Cover(prob["domain"], cov)
    sysm = pdd.System(cv, prob, cfg["mc"])
    rowptr, cols, val, b, se = (t.cpu().numpy() for t in sysm.csr())
    rp_h, cols_h = cv.pattern()
    assert np.array_equal(rowptr, rp_h) and np.array_equal(cols, cols_h)
    val2, b2, se2, _ = (t.cpu().numpy() for t in sysm.copy())
    assert np.array_equal(val, val2) and np.array_equal(b, b2) and np.array_equal(se, se2)


@pytest.mark.parametrize("chunked", [False, True])
def test_adjoint_uneven_buckets_matches_oracle(chunked):
    """The adjoint on the four collocation sizes of the uneven-resolution
    family (n = 576, 1024, 2304, 4096; the two largest need the wide panel
    classes and the largest adjoint LDS layout), with the factors kept and
    with them recomputed chunk by chunk, against the oracle's adjoint."""
    pdd, torch = _gpu()
    from helpers_parity import check_circle_gradient, gradient_terms
    cfg = workloads.mixed_small()
    prob = cfg["problem"]
    _say(f"[gpu] adjoint, uneven buckets, chunked={chunked}")
    cv = pdd.Cover(prob["domain"], cfg["cover"])
    sysm = pdd.System(cv, prob, cfg["mc"], keep_factors=True)
    if chunked:
        budget = sysm.stats.factor_bytes // 3
        sysm = pdd.System(cv, prob, cfg["mc"], keep_factors=True, hbm_budget_bytes=int(budget))
        assert sysm.stats.recompute == 1
    u, _ = sysm.solve(rtol=1e-13)
    rng = np.random.default_rng(17)
    lam = torch.tensor(rng.standard_normal(cv.N), device="cuda")
    g = {k: v.cpu().numpy() for k, v in sysm.backward(u, lam).items()}
    ref_cover = geometry.build_cover(prob["domain"], cfg["cover"])
    xy, off, ids = cv.nodes()
    u_h, lam_h = u.cpu().numpy(), lam.cpu().numpy()
    sizes = []
    for f, m in enumerate(ids):
        grid = spectral.local_grid(ref_cover.Nr[m], ref_cover.Ntheta[m])
        samples = spectral.node_samples(prob, grid, *ref_cover.centres[m], ref_cover.radii[m])
        ref, slack = gradient_terms(ref_cover, m, samples, u_h, lam_h)
        check_circle_gradient(ref, slack, {k: g[k][off[f]:off[f + 1]] for k in ref})
        sizes.append(int(off[f + 1] - off[f]))
    assert sorted(sizes) == [576, 1024, 2304, 4096]
