"""Cardinal functions of the two interface interpolators (Section 2.2).

* Floating interfaces (full circles, n equispaced knots, n even): eq. 18,
  H_j(theta) = (1/n) sum_{k=-n/2}^{n/2-1} cos k (theta - theta_j).
* Perimeter interfaces (arcs): inverse multiquadric RBFs, eqs. 19-22,
  phi_j(theta) = ((theta - theta_j)^2 + c^2)^(-1/2),  K_lk = phi_k(theta_l),
  H_j(theta) = sum_l (K^-1)_lj phi_l(theta).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def fourier_cardinal(theta, theta_j, n):
    """Eq. 18 written out as the sum over k = -n/2 .. n/2 - 1.

    Broadcasts theta against theta_j; returns H_j(theta)."""
    if n % 2:
        raise ValueError("eq. 18 is stated for an even number of knots")
    x = np.asarray(theta, dtype=np.float64) - np.asarray(theta_j, dtype=np.float64)
    total = np.zeros_like(x)
    for k in range(-n // 2, n // 2):
        total = total + np.cos(k * x)
    return total / n


def fourier_cardinal_derivs(theta, theta_j, n):
    """First and second theta-derivatives of eq. 18, term by term."""
    x = np.asarray(theta, dtype=np.float64) - np.asarray(theta_j, dtype=np.float64)
    d1 = np.zeros_like(x)
    d2 = np.zeros_like(x)
    for k in range(-n // 2, n // 2):
        d1 = d1 - k * np.sin(k * x)
        d2 = d2 - k * k * np.cos(k * x)
    return d1 / n, d2 / n


def fourier_matrix(theta_eval, n):
    """H[l, j] = H_j(theta_eval[l]) for the n-knot grid theta_j = 2 pi j / n."""
    theta_knots = 2.0 * np.pi * np.arange(n) / n
    return fourier_cardinal(np.asarray(theta_eval)[:, None], theta_knots[None, :], n)


def default_rbf_c2(M):
    """Shape parameter: the paper's c^2 = 1.5 at 44 knots per circle (Section 4),
    scaled with the knot spacing so that c / dtheta stays at its value there."""
    return 1.5 * (44.0 / M) ** 2


def imq(theta, theta_l, c2):
    """Eq. 19."""
    d = np.asarray(theta, dtype=np.float64) - np.asarray(theta_l, dtype=np.float64)
    return 1.0 / np.sqrt(d * d + c2)


def imq_gram(theta_knots, c2):
    """Eq. 20: K_lk = phi_k(theta_l)."""
    t = np.asarray(theta_knots, dtype=np.float64)
    return imq(t[:, None], t[None, :], c2)


def imq_cardinal(theta, theta_knots, c2):
    """Eq. 22: H[., j] = sum_l (K^-1)_lj phi_l(theta), via a Cholesky solve of the
    symmetric positive definite Gram matrix.  Returns shape (len(theta), n)."""
    K = imq_gram(theta_knots, c2)
    phi = imq(np.asarray(theta)[:, None], np.asarray(theta_knots)[None, :], c2)
    cho = sla.cho_factor(K, lower=True)
    # H = phi K^-1 (K symmetric)
    return sla.cho_solve(cho, phi.T).T
