"""Pins for the oracle's RAS preconditioner and GMRES (Section 4, eqs. 42-45).

* eq. 43: the weighted restrictions add up to the identity;
* the overlap is exactly one layer of the symmetric graph of C (brute force
  over the pattern);
* with one part, M_RAS^-1 is C^-1 (eq. 44 with R_1 = I) and GMRES stops after
  one iteration at the direct solution;
* GMRES, preconditioned or not, reaches the direct solution, and with RAS in
  fewer iterations;
* after k unrestarted iterations GMRES holds the minimal-residual iterate over
  the k-th Krylov space, computed independently by least squares on an
  orthonormal basis of [b, C b, ..., C^{k-1} b].
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import assemble, geometry, ras


@pytest.fixture(scope="module")
def c1():
    cfg = workloads.config1(paths=64)
    prob = cfg["problem"]
    cv = geometry.build_cover(prob["domain"], cfg["cover"])
    s = assemble.assemble(prob, cv, cfg["mc"])
    C = sp.csr_matrix((s.val, cv.cols, cv.rowptr), shape=(cv.N, cv.N))
    return cv, C, s.b


def test_weights_are_a_partition_of_unity(c1):
    cv, C, b = c1
    omegas, D = ras.subdomains(cv, 2, 2)
    tot = np.zeros(cv.N)
    for w, d in zip(omegas, D):
        assert np.all(np.diff(w) > 0)
        tot[w] += d
    assert np.allclose(tot, 1.0, rtol=0, atol=1e-15)
    part, P = ras.partition(cv, 2, 2)
    assert P == 4 and set(part) == {0, 1, 2, 3}


def test_overlap_is_one_layer_of_the_graph(c1):
    cv, C, b = c1
    part, P = ras.partition(cv, 2, 2)
    omegas, _ = ras.subdomains(cv, 2, 2)
    for p in range(P):
        want = set(np.nonzero(part == p)[0])
        own = set(want)
        for i in range(cv.N):
            for j in cv.cols[cv.rowptr[i]:cv.rowptr[i + 1]]:
                if i in own:
                    want.add(int(j))
                if int(j) in own:
                    want.add(i)
        assert sorted(want) == list(omegas[p]), p


def test_partition_follows_the_circle_order(c1):
    cv, C, b = c1
    part, P = ras.partition(cv, 2, 1)
    # config1's 4x4 lattice: two slabs of two columns each, split by x
    cx = cv.centres[:, 0]
    for i in range(cv.N):
        assert part[i] == (0 if cx[cv.knot_owner[i]] < 0.5 else 1)


def test_one_part_is_the_exact_inverse(c1):
    cv, C, b = c1
    M = ras.RAS(C, cv, 1, 1)
    x = np.random.default_rng(0).standard_normal(cv.N)
    ref = spla.spsolve(sp.csc_matrix(C), x)
    assert np.max(np.abs(M.apply(x) - ref)) <= 1e-12 * np.max(np.abs(ref))
    u, it, rel = ras.gmres(C, b, M, rtol=1e-12)
    assert it == 1
    u_ref = spla.spsolve(sp.csc_matrix(C), b)
    assert np.max(np.abs(u - u_ref)) <= 1e-11 * np.max(np.abs(u_ref))


@pytest.mark.parametrize("parts", [None, (2, 2), (4, 4)])
def test_gmres_reaches_the_direct_solution(c1, parts):
    cv, C, b = c1
    M = None if parts is None else ras.RAS(C, cv, *parts)
    u, it, rel = ras.gmres(C, b, M, rtol=1e-12, restart=30)
    u_ref = spla.spsolve(sp.csc_matrix(C), b)
    assert rel <= 1e-12
    assert np.linalg.norm(b - C @ u) <= 1e-11 * np.linalg.norm(b)
    assert np.max(np.abs(u - u_ref)) <= 1e-9 * np.max(np.abs(u_ref))
    if parts == (2, 2):
        _, it0, _ = ras.gmres(C, b, None, rtol=1e-12, restart=30)
        assert it < it0


def test_gmres_iterate_is_the_krylov_minimal_residual(c1):
    cv, C, b = c1
    for k in (3, 7):
        u, it, rel = ras.gmres(C, b, None, rtol=0.0, restart=50, max_iter=k)
        assert it == k
        K = np.empty((cv.N, k))
        v = b.copy()
        for t in range(k):
            K[:, t] = v
            v = C @ v
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(C @ Q, b, rcond=None)
        best = np.linalg.norm(b - C @ (Q @ y))
        assert abs(np.linalg.norm(b - C @ u) - best) <= 1e-10 * np.linalg.norm(b)
        assert abs(rel * np.linalg.norm(b) - best) <= 1e-10 * np.linalg.norm(b)
