"""Plain FP64 oracle of the resampling and transmission steps (§2.6, §2.1).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by
``tests/`` alone; it shares no code with the GPU library.

* Resampling (§2.6): per bin, a least-squares fit of ln kappa(y) by
  Chebyshev polynomials, solved by a QR decomposition of the design matrix.
  Readings: the i-th smallest of a bin's M values sits at y_i = (i + 1/2)/M
  (the middle of its interval of the cumulative coordinate); the fit
  variable is t = 2y - 1 on [-1, 1]; n_coef = 20 coefficients (T_0 ..
  T_19); values <= 0 are clamped to the smallest positive normal binary64
  before the logarithm.
* Transmission (eq. 5): T(m) = int_0^1 exp(-kappa(y) m) dy.  From the fit it
  is evaluated with the 100-node Gauss-Legendre rule on [0, 1] (a reading:
  the paper does not state the quadrature); "direct" from the sorted values
  it is the mean of exp(-kappa_i m) over the bin.
"""
from __future__ import annotations

import numpy as np

TINY = np.finfo(np.float64).tiny
N_QUAD = 100


def design(m: int, n_coef: int = 20) -> np.ndarray:
    """A[i][c] = T_c(t_i), t_i = 2 (i + 1/2)/m - 1, by the three-term
    recurrence T_{c+1} = 2 t T_c - T_{c-1}."""
    t = 2.0 * (np.arange(m) + 0.5) / m - 1.0
    A = np.empty((m, n_coef))
    A[:, 0] = 1.0
    if n_coef > 1:
        A[:, 1] = t
    for c in range(2, n_coef):
        A[:, c] = 2.0 * t * A[:, c - 1] - A[:, c - 2]
    return A


def fit_bin(sorted_kappa, n_coef: int = 20) -> np.ndarray:
    """Chebyshev coefficients of ln kappa(y) for one sorted bin, by QR:
    A = QR, R C = Q^T d."""
    d = np.log(np.maximum(np.asarray(sorted_kappa, dtype=np.float64), TINY))
    A = design(len(d), n_coef)
    Q, R = np.linalg.qr(A)
    return np.linalg.solve(R, Q.T @ d)


def fit(kappa, points_per_bin: int, n_coef: int = 20) -> np.ndarray:
    """[n_bins][n_coef] for a whole grid (bins of consecutive points, the
    last one possibly shorter)."""
    kappa = np.asarray(kappa, dtype=np.float64)
    n_bins = -(-len(kappa) // points_per_bin)
    out = np.empty((n_bins, n_coef))
    for b in range(n_bins):
        out[b] = fit_bin(np.sort(kappa[b * points_per_bin:(b + 1) * points_per_bin]), n_coef)
    return out


def chebval(coef, t) -> np.ndarray:
    """sum_c coef[c] T_c(t) by the recurrence (no library)."""
    t = np.asarray(t, dtype=np.float64)
    Tm, T = np.ones_like(t), t
    s = coef[0] * Tm
    if len(coef) > 1:
        s = s + coef[1] * T
    for c in range(2, len(coef)):
        Tm, T = T, 2.0 * t * T - Tm
        s = s + coef[c] * T
    return s


def quad_rule(n: int = N_QUAD):
    """Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def transmission_fit(coef, m) -> np.ndarray:
    """T(m) from one bin's coefficients, for each column mass in m."""
    y, w = quad_rule()
    k = np.exp(chebval(coef, 2.0 * y - 1.0))
    m = np.asarray(m, dtype=np.float64)
    return np.exp(-np.outer(m, k)) @ w


def transmission_direct(sorted_kappa, m) -> np.ndarray:
    """T(m) as the bin mean of exp(-kappa_i m)."""
    k = np.asarray(sorted_kappa, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    return np.exp(-np.outer(m, k)).mean(axis=1)
