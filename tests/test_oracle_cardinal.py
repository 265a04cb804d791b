"""Pins for the Fourier (eq. 18) and inverse-multiquadric (eqs. 19-22) cardinal
functions of the oracle."""
import math

import numpy as np
import pytest

from oracle import cardinal


@pytest.mark.parametrize("n", [8, 32, 44, 64])
def test_fourier_cardinal_is_periodic_sinc(n):
    # textbook closed form of the band-limited interpolant on n even points
    x = np.linspace(-math.pi, math.pi, 1001)
    x = x[np.abs(np.sin(x / 2)) > 1e-3]
    closed = np.sin(n * x / 2) / (n * np.tan(x / 2))
    assert np.max(np.abs(cardinal.fourier_cardinal(x, 0.0, n) - closed)) < 1e-13


@pytest.mark.parametrize("n", [8, 32])
def test_fourier_kronecker_and_partition_of_unity(n):
    th = 2 * math.pi * np.arange(n) / n
    H = cardinal.fourier_matrix(th, n)
    assert np.max(np.abs(H - np.eye(n))) < 1e-14
    t = np.random.default_rng(1).uniform(0, 2 * math.pi, 200)
    assert np.max(np.abs(cardinal.fourier_matrix(t, n).sum(axis=1) - 1.0)) < 1e-13


def test_fourier_interpolates_trig_polynomials_exactly():
    n = 16
    th = 2 * math.pi * np.arange(n) / n
    f = lambda t: 0.3 + np.cos(3 * t) - 0.7 * np.sin(7 * t) + 0.2 * np.cos(8 * t)
    t = np.random.default_rng(2).uniform(0, 2 * math.pi, 100)
    interp = cardinal.fourier_matrix(t, n) @ f(th)
    # the Nyquist mode cos(8 t) is represented as cos(8 t) (sin(8 theta_j) = 0)
    assert np.max(np.abs(interp - f(t))) < 1e-13


def test_fourier_derivatives_include_nyquist_second_derivative():
    n = 16
    th = 2 * math.pi * np.arange(n) / n
    d1, d2 = cardinal.fourier_cardinal_derivs(th[:, None], th[None, :], n)
    assert np.max(np.abs(d1 @ np.sin(5 * th) - 5 * np.cos(5 * th))) < 1e-12
    assert np.max(np.abs(d2 @ np.sin(5 * th) + 25 * np.sin(5 * th))) < 1e-11
    nyq = np.cos(n / 2 * th)
    assert np.max(np.abs(d2 @ nyq + (n / 2) ** 2 * nyq)) < 1e-10
    assert np.max(np.abs(d1 @ nyq)) < 1e-12


def _arc(M, span):
    dth = 2 * math.pi / M
    grid = np.arange(0.0, span, dth)[1:]
    return np.concatenate([[0.0], grid[grid < span - 0.25 * dth], [span]])


@pytest.mark.parametrize("M", [32, 64])
def test_imq_kronecker_and_smooth_interpolation(M):
    th = _arc(M, 3.5)
    c2 = cardinal.default_rbf_c2(M)
    H = cardinal.imq_cardinal(th, th, c2)
    assert np.max(np.abs(H - np.eye(len(th)))) < 1e-4
    f = lambda t: np.exp(np.sin(t)) + 0.3 * t
    t = np.random.default_rng(3).uniform(0, 3.5, 300)
    err = np.max(np.abs(cardinal.imq_cardinal(t, th, c2) @ f(th) - f(t)))
    assert err < 1e-3
    # Cholesky cardinal values agree with an LU solve of the same Gram matrix
    K = cardinal.imq_gram(th, c2)
    phi = cardinal.imq(t[:, None], th[None, :], c2)
    H_lu = np.linalg.solve(K, phi.T).T
    assert np.max(np.abs(H_lu - cardinal.imq_cardinal(t, th, c2))) < 1e-3


def test_imq_gram_is_symmetric_definition():
    th = _arc(32, 2.0)
    K = cardinal.imq_gram(th, 0.5)
    assert np.array_equal(K, K.T)
    assert K[0, 2] == 1.0 / math.sqrt((th[0] - th[2]) ** 2 + 0.5)
