"""Pins of the resampling / transmission oracle (oracle/resample.py): a
library's Chebyshev basis and least-squares fit, exact polynomials,
closed-form transmissions, quadrature exactness, sorting invariance.  The
paper's claim about the resampling error is reported, not asserted (its
data are not available; the synthetic bins span 25 decades of kappa)."""
import numpy as np
import pytest

import oracle
from oracle import resample as R
import synth

scipy_special = pytest.importorskip("scipy.special")


def test_design_matrix_is_the_chebyshev_basis():
    for m in (1, 7, 1000):
        A = R.design(m, 20)
        t = 2.0 * (np.arange(m) + 0.5) / m - 1.0
        assert np.allclose(A, np.polynomial.chebyshev.chebvander(t, 19), rtol=0, atol=1e-12)


def test_fit_recovers_an_exact_polynomial():
    rng = np.random.default_rng(1)
    c = rng.normal(size=20) / (1 + np.arange(20)) ** 2
    m = 5000
    t = 2.0 * (np.arange(m) + 0.5) / m - 1.0
    lnk = np.polynomial.chebyshev.chebval(t, c)
    got = R.fit_bin(np.exp(lnk))
    assert np.max(np.abs(got - c)) < 1e-10


def test_fit_matches_library_least_squares():
    rng = np.random.default_rng(2)
    k = np.sort(10.0 ** rng.uniform(-25, -18, 3000))
    t = 2.0 * (np.arange(3000) + 0.5) / 3000 - 1.0
    ref = np.polynomial.chebyshev.chebfit(t, np.log(k), 19)
    got = R.fit_bin(k)
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))
    assert np.allclose(R.chebval(got, t), np.polynomial.chebyshev.chebval(t, got), rtol=1e-13, atol=1e-12)


def test_quadrature_is_exact_for_polynomials():
    y, w = R.quad_rule()
    for k in (0, 1, 5, 50, 150, 199):
        assert abs(np.dot(w, y ** k) - 1.0 / (k + 1)) < 1e-14


def test_transmission_of_constant_and_exponential_kappa():
    m = np.logspace(-3, 3, 50)
    # constant kappa: T = exp(-kappa m)
    c = np.zeros(20); c[0] = np.log(2.5)
    assert np.allclose(R.transmission_fit(c, m), np.exp(-2.5 * m), rtol=1e-13, atol=0)
    # ln kappa = a + s y: T = (E1(k0 m) - E1(k0 e^s m)) / s
    a, s = np.log(0.3), 4.0
    c = np.zeros(20); c[0] = a + s / 2; c[1] = s / 2
    k0 = np.exp(a)
    ref = (scipy_special.exp1(k0 * m) - scipy_special.exp1(k0 * np.exp(s) * m)) / s
    assert np.allclose(R.transmission_fit(c, m), ref, rtol=1e-10, atol=1e-14)


def test_direct_transmission_closed_forms():
    """Eq. (5) on bins whose k-distribution is a step function: a constant
    bin gives exp(-k m); a bin of two values in proportions p and 1 - p gives
    p exp(-k1 m) + (1 - p) exp(-k2 m); a bin of values k_i = i c (i = 0 ..
    M-1) gives the geometric sum (1 - r^M) / (M (1 - r)), r = exp(-c m)."""
    m = np.logspace(-4, 4, 41)
    k = np.full(1000, 0.37)
    assert np.allclose(R.transmission_direct(k, m), np.exp(-0.37 * m), rtol=1e-14, atol=0)
    k1, k2 = 0.02, 5.0
    k = np.array([k1] * 300 + [k2] * 700)
    ref = 0.3 * np.exp(-k1 * m) + 0.7 * np.exp(-k2 * m)
    assert np.allclose(R.transmission_direct(k, m), ref, rtol=1e-13, atol=1e-300)
    M, c = 257, 0.01
    k = c * np.arange(M)
    r = np.exp(-c * m)
    ref = (1.0 - r ** M) / (M * (1.0 - r))
    assert np.allclose(R.transmission_direct(k, m), ref, rtol=1e-12, atol=0)


def test_direct_transmission_ignores_the_order():
    rng = np.random.default_rng(3)
    k = 10.0 ** rng.uniform(-3, 3, 777)
    m = np.logspace(-4, 4, 30)
    assert np.allclose(R.transmission_direct(np.sort(k), m), R.transmission_direct(k, m), rtol=1e-14)
    assert np.all(np.diff(R.transmission_direct(np.sort(k), m)) <= 0)


def test_resampling_error_on_the_small_workload_is_reported():
    w = synth.WORKLOADS["lines1e4_grid3e5"]
    kap, _ = oracle.opacity(w.lines(), w.conditions(), w.grid())
    ppb = w.points_per_bin
    coef = R.fit(kap, ppb)
    for b in range(3):
        s = np.sort(kap[b * ppb:(b + 1) * ppb])
        m = np.logspace(np.log10(1e-3 / s[-1]), np.log10(1e3 / s[0]), 1000)
        d = np.abs(R.transmission_fit(coef[b], m) - R.transmission_direct(s, m)).max()
        print("bin %d: kappa %.1e..%.1e, max |T_fit - T_direct| = %.2e" % (b, s[0], s[-1], d))
        assert np.isfinite(d) and d < 0.1
