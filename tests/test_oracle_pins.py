"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

The paper prints no worked numerical example (its numbers are in figures), so
every pin here is a closed form, a limit, an invariant, an independent library
routine, or brute force on tiny inputs.  Each is chosen so that a plausible
slip in the oracle (a dropped term, a wrong sign or factor, a transposed
operand, an off-by-one window) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import oracle
import synth

SQPI = math.sqrt(math.pi)


def _plane(rng, n, rmax2, rmin2=0.0):
    """Random (a, u) with rmin2 <= a^2 + u^2 < rmax2, a mixture of uniform-in-
    radius points and points with very small a."""
    r = np.sqrt(rng.uniform(rmin2, rmax2, n))
    th = rng.uniform(0.0, np.pi / 2, n)
    a, u = r * np.sin(th), r * np.cos(th)
    small = rng.uniform(size=n) < 0.3
    a[small] = 10.0 ** rng.uniform(-8, 0, small.sum())
    u[small] = np.sqrt(np.maximum(r[small] ** 2 - a[small] ** 2, 0.0))
    sign = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    keep = (a * a + u * u >= rmin2) & (a * a + u * u < rmax2)
    return a[keep], (u * sign)[keep]


# ---- P1/P2/P3/P4: the Voigt scheme against the exact Faddeeva function ----

def test_p1_core_series_at_line_centre_is_erfcx():
    # H_V(a, 0) = Re w(i a) = exp(a^2) erfc(a): at u = 0 the three sums
    # coincide and cancel, leaving the erfcx term.
    a = np.concatenate([np.geomspace(1e-8, 9.99, 200), [0.5, 1.0, 2.0, 5.0]])
    got = oracle.voigt_series(a, np.zeros_like(a))
    ref = special.erfcx(a)
    assert np.max(np.abs(got / ref - 1.0)) < 1e-13


def test_p2_gaussian_limit():
    # a -> 0: H_V(0, u) = exp(-u^2) (pure Doppler profile).
    u = np.linspace(-9.99, 9.99, 401)
    got = oracle.voigt_H(np.zeros_like(u), u)
    ref = np.exp(-u * u)
    assert np.max(np.abs(got / ref - 1.0)) < 1e-13
    # and continuity as a -> 0+ near the core, where the Lorentz part
    # a / (sqrt(pi) u^2) is still negligible against exp(-u^2)
    c = np.abs(u) <= 3.0
    got2 = oracle.voigt_H(np.full_like(u[c], 1e-12), u[c])
    assert np.max(np.abs(got2 / ref[c] - 1.0)) < 1e-9


def test_p3_lorentz_limit_far_region():
    rng = np.random.default_rng(11)
    a, u = _plane(rng, 4000, 1e10, 1e6)
    got = oracle.voigt_H(a, u)
    ref = special.wofz(u + 1j * a).real
    assert np.max(np.abs(got / ref - 1.0)) < 1.6e-6
    # the 1-node rule is the Lorentz profile a / (sqrt(pi) (u^2 + a^2))
    lor = a / (SQPI * (u * u + a * a))
    assert np.max(np.abs(got / lor - 1.0)) < 1e-15


@pytest.mark.parametrize("lo,hi,tol", [(0.0, 100.0, 2e-13),
                                       (100.0, 1e6, 5.7e-6),
                                       (1e6, 1e12, 1.6e-6)])
def test_p4_scheme_vs_faddeeva_over_plane(lo, hi, tol):
    rng = np.random.default_rng(4)
    a, u = _plane(rng, 20000, hi, lo)
    got = oracle.voigt_H(a, u)
    ref = special.wofz(u + 1j * a).real
    err = np.abs(got / ref - 1.0)
    assert err.max() < tol, (err.max(), a[err.argmax()], u[err.argmax()])


def test_p4_series_vs_mpmath_high_precision():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    pts = [(1e-6, 0.3), (0.01, 2.5), (0.3, 7.9), (2.0, 4.0), (9.0, 3.0),
           (0.5, 9.9), (5.0, 0.0), (1e-3, 6.0)]
    for a, u in pts:
        z = mp.mpc(u, a)
        ref = float(mp.re(mp.exp(-z * z) * mp.erfc(-1j * z)))
        got = oracle.voigt_series(a, u)[0]
        assert abs(got / ref - 1.0) < 2e-13, (a, u, got, ref)


def test_region_switch_thresholds():
    # just below / at the switch radii the scheme picks series / GH3 / GH1
    a = 3.0
    u_100 = math.sqrt(100.0 - a * a)
    below = np.nextafter(u_100, 0.0)
    assert oracle.voigt_H(a, below)[0] == oracle.voigt_series(a, below)[0]
    u_hi = np.nextafter(u_100, 20.0) * (1 + 1e-15)
    assert oracle.voigt_H(a, u_hi)[0] == oracle.voigt_gh3(a, u_hi)[0]
    u_1e6 = math.sqrt(1e6 - a * a) * (1 + 1e-15)
    assert oracle.voigt_H(a, u_1e6)[0] == oracle.voigt_gh1(a, u_1e6)[0]


# ---- P5: unit area of the profile ----

@pytest.mark.parametrize("a", [1e-3, 0.1, 1.0, 5.0])
def test_p5_unit_area(a):
    """int H_V du = sqrt(pi), hence int Phi dnu = 1 (eq. (19)).  The scheme is
    integrated piecewise over its regions; the tail beyond the last breakpoint
    is the 1-node (Lorentz) rule, integrated in closed form.  Tolerance: the
    scheme's relative error bound 5.7e-6 (3-node rule at a^2+u^2 = 100)."""
    f = lambda u: oracle.voigt_H(a, u)[0]
    u1 = math.sqrt(max(100.0 - a * a, 0.0))
    u2 = math.sqrt(1e6 - a * a)
    U = 1e5
    pieces = [(0.0, u1), (u1, 30.0), (30.0, 300.0), (300.0, u2), (u2, U)]
    tot = 0.0
    for lo, hi in pieces:
        if hi > lo:
            v, _ = integrate.quad(f, lo, hi, limit=400, epsabs=0, epsrel=1e-13)
            tot += v
    tot += (math.pi / 2 - math.atan(U / a)) / SQPI  # int_U^inf a/(sqrt(pi)(u^2+a^2))
    assert abs(2.0 * tot / SQPI - 1.0) < 5.7e-6


# ---- P6: quadrature nodes ----

def test_p6_gauss_hermite_3_matches_hermgauss():
    t, w = np.polynomial.hermite.hermgauss(3)
    rng = np.random.default_rng(6)
    a, u = _plane(rng, 500, 1e6, 100.0)
    ref = (a / np.pi) * sum(wi / ((u - ti) ** 2 + a * a) for ti, wi in zip(t, w))
    got = oracle.voigt_gh3(a, u)
    assert np.max(np.abs(got / ref - 1.0)) < 1e-14
    t1, w1 = np.polynomial.hermite.hermgauss(1)
    ref1 = (a / np.pi) * w1[0] / ((u - t1[0]) ** 2 + a * a)
    assert np.max(np.abs(oracle.voigt_gh1(a, u) / ref1 - 1.0)) < 1e-15


def test_p6_gauss_legendre_matches_leggauss():
    for n in (1, 2, 5, 20, 33):
        x, w = oracle.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.max(np.abs(x - xr)) < 2e-15
        assert np.max(np.abs(w - wr)) < 2e-15
    g, wg = oracle.g_nodes(20)
    assert np.all((g > 0) & (g < 1)) and abs(wg.sum() - 1.0) < 1e-14


# ---- P7: line strength and widths (§2.3) ----

def test_p7_line_strength_limits():
    S0 = np.array([1e-20, 3e-25, 7e-30])
    E = np.array([0.0, 1234.5, 6000.0])
    nu = np.array([0.5, 1500.0, 25000.0])
    # at the reference temperature with Q(T) = Q(T0) nothing changes
    assert np.all(oracle.line_strength(S0, E, nu, 296.0, 296.0, 1.0) == S0)
    c2 = oracle.const("c2")
    assert abs(c2 / 1.438776877 - 1.0) < 1e-9  # second radiation constant, cm K
    T = 1500.0
    # nu -> 0: the stimulated-emission ratio is (T0/T)(1 - z (1/T - 1/T0)/2
    # + O(z^2)) with z = c2 nu; E = 0 removes the Boltzmann factor.  A naive
    # 1 - exp(-z) would lose ~7 digits here.
    for nu_small in (1e-6, 1e-3):
        s = oracle.line_strength(1.0, 0.0, nu_small, T, 296.0, 1.0)
        ref = (296.0 / T) * (1 - c2 * nu_small * (1 / T - 1 / 296.0) / 2)
        assert abs(s / ref - 1.0) < 1e-13 + (c2 * nu_small / 296.0) ** 2
    # c2 nu / T >> 1: ratio -> 1, leaving q * exp(-c2 E (1/T - 1/T0))
    s = oracle.line_strength(1.0, 2000.0, 1e5, T, 296.0, 0.7)
    ref = 0.7 * math.exp(-c2 * 2000.0 * (1 / T - 1 / 296.0))
    assert abs(s / ref - 1.0) < 1e-13
    # a mid-range line against an independent 30-digit evaluation of eq. (18)
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    h, c, k = mp.mpf("6.62607015e-27"), mp.mpf("2.99792458e10"), mp.mpf("1.380649e-16")
    nu_, E_, T_, T0 = mp.mpf(1500), mp.mpf("1234.5"), mp.mpf(1500), mp.mpf(296)
    q = (T0 / T_) ** mp.mpf(1.5)
    ref = q * mp.exp(-h * c * E_ / (k * T_) + h * c * E_ / (k * T0)) * \
        (1 - mp.exp(-h * c * nu_ / (k * T_))) / (1 - mp.exp(-h * c * nu_ / (k * T0)))
    got = oracle.line_strength(1.0, 1234.5, 1500.0, 1500.0, 296.0, float(q))
    assert abs(got / float(ref) - 1.0) < 1e-14


def test_p7_doppler_width():
    # Textbook Doppler FWHM: 7.162e-7 nu sqrt(T / M) with M in amu; the
    # paper's Gamma_D is the half width.
    g = oracle.doppler_hwhm(1000.0, 300.0, 18.0)
    assert abs(2.0 * g / (7.162e-7 * 1000.0 * math.sqrt(300.0 / 18.0)) - 1.0) < 1e-4
    # and it is the half width at half maximum of the a -> 0 profile
    u_half = math.sqrt(math.log(2.0)) * g / g
    assert abs(oracle.voigt_H(0.0, u_half)[0] - 0.5) < 1e-15
    # scaling laws: proportional to nu and sqrt(T/m)
    assert abs(oracle.doppler_hwhm(3000.0, 300.0, 18.0) / g - 3.0) < 1e-14
    assert abs(oracle.doppler_hwhm(1000.0, 1200.0, 18.0) / g - 2.0) < 1e-14
    assert abs(oracle.doppler_hwhm(1000.0, 300.0, 72.0) / g - 0.5) < 1e-14


def test_p7_lorentz_width():
    # T = T0, P = 1 atm, equal air/self widths: Gamma_L = gamma
    assert abs(oracle.lorentz_hwhm(0.0, 0.7, 0.05, 0.05, 296.0, 296.0, 1.0, 0.5) - 0.05) < 1e-17
    # P = 0 leaves the natural width A21 / (4 pi c)
    A = 1e8
    nat = oracle.lorentz_hwhm(A, 0.7, 0.05, 0.05, 1500.0, 296.0, 0.0, 0.0)
    assert abs(nat / (A / (4 * math.pi * oracle.const("c"))) - 1.0) < 1e-15
    # temperature scaling (T0/T)^n and separate air / self parts
    g = oracle.lorentz_hwhm(0.0, 0.5, 0.04, 0.2, 1184.0, 296.0, 2.0, 0.5)
    assert abs(g / ((0.04 * 1.5 + 0.2 * 0.5) * 0.5) - 1.0) < 1e-15


# ---- windows ----

def test_cutoff_window_closed_and_clipped():
    # dyadic values make every bound exact: [ (10-2)/0.25, (10+2)/0.25 ]
    assert oracle.window(10.0, 2.0, 0.0, 0.25, 1000) == (32, 48, 17)
    assert oracle.window(1.0, 2.0, 0.0, 0.25, 1000) == (0, 12, 13)       # clipped low
    assert oracle.window(249.0, 2.0, 0.0, 0.25, 1000) == (988, 999, 12)  # clipped high
    assert oracle.window(300.0, 2.0, 0.0, 0.25, 1000)[2] == 0            # off the grid
    assert oracle.window(10.0, 0.0, 0.0, 0.25, 1000) == (40, 40, 1)      # zero cutoff
    assert oracle.window(10.1, 0.0, 0.0, 0.25, 1000)[2] == 0             # between points


# ---- P8: integrated opacity of a single resolved line ----

@pytest.mark.parametrize("nu0,P,dnu,cut", [(1000.0037, 1.0, 0.01, 25.0),
                                            (2500.0, 1.0, 0.01, 5.0),
                                            (700.123, 3.0, 0.01, 2.0)])
def test_p8_integrated_line_opacity(nu0, P, dnu, cut):
    """sum_j kappa_j dnu = S(T) (1 - L - D + C).

    L: the Lorentz wing beyond the window's cell edges.
    D: the scheme's wing term.  The 3-node rule is a weighted sum of
       Lorentzians centred at nu0 and nu0 +- sqrt(3/2) alpha_D, so its area is
       exactly S and its far wing is Lorentz x (1 + 1.5 alpha^2 / dnu^2);
       cutting it at m = min(cutoff, 1-node switch distance) removes
       G_L alpha^2 / (pi m^3) more than a Lorentzian would.
    C: inside a^2 + u^2 < 100 the exact function replaces the 3-node rule;
       C = int (Re w - H_GH3) du / sqrt(pi) over that range, with scipy's
       Faddeeva function and numpy's Gauss-Hermite nodes.
    The sum is a midpoint rule; for a resolved line its interior error is
    bounded (Poisson summation) by 2 exp(-2 pi G_L/dnu - (pi alpha_D/dnu)^2),
    plus Euler-Maclaurin end terms at the window edges and the jump of the
    scheme (<= 5.7e-6 relative) at the core boundary."""
    T = 1500.0
    lines = {"nu": np.array([nu0]), "S_ref": np.array([1e-20]), "E_lower": np.array([500.0]),
             "gamma_air": np.array([0.1]), "n_air": np.array([0.5])}
    cond = synth.conditions(T, P)
    grid = {"nu_min": nu0 - 40.0 - 0.00123, "dnu": dnu, "n_points": int(80 / dnu), "cutoff": cut}
    kap, n = oracle.opacity(lines, cond, grid)
    S = oracle.line_strength(1e-20, 500.0, nu0, T, 296.0, cond["q_ratio"])
    GL = oracle.lorentz_hwhm(0.0, 0.5, 0.1, 0.1, T, 296.0, P, 0.5 * P)
    aD = oracle.doppler_hwhm(nu0, T, 18.0) / math.sqrt(math.log(2.0))
    y = GL / aD
    lo, hi, cnt = oracle.window(nu0, cut, grid["nu_min"], dnu, grid["n_points"])
    assert cnt == n
    e_lo = grid["nu_min"] + lo * dnu - 0.5 * dnu
    e_hi = grid["nu_min"] + hi * dnu + 0.5 * dnu
    inside = (math.atan((nu0 - e_lo) / GL) + math.atan((e_hi - nu0) / GL)) / math.pi
    d1 = aD * math.sqrt(1e6 - y * y)
    m = min(cut, d1)
    D = GL * aD ** 2 / (math.pi * m ** 3)
    C = 0.0
    jump = 0.0
    if y < 10.0:
        t, w = np.polynomial.hermite.hermgauss(3)
        gh3 = lambda u: (y / np.pi) * sum(wi / ((u - ti) ** 2 + y * y) for ti, wi in zip(t, w))
        uc = math.sqrt(100.0 - y * y)
        v, _ = integrate.quad(lambda u: special.wofz(u + 1j * y).real - gh3(u), -uc, uc,
                              limit=400, epsabs=1e-15, epsrel=1e-12)
        C = v / SQPI
        # a step of height dH at a point inside a cell moves the midpoint sum
        # by at most dnu/2 times the step in Phi = H / (sqrt(pi) alpha_D)
        dH = abs(special.wofz(uc + 1j * y).real - gh3(uc))
        jump = 2 * (dnu / 2) * dH / (SQPI * aD)
    # midpoint-rule end corrections (Euler-Maclaurin): dnu^2/24 |f'| at the
    # two cell edges, f' of the normalised Lorentzian
    fp = lambda d: 2 * GL * d / (math.pi * (d * d + GL * GL) ** 2)
    em = dnu ** 2 / 24 * (fp(nu0 - e_lo) + fp(e_hi - nu0))
    bound = 2 * math.exp(-2 * math.pi * GL / dnu - (math.pi * aD / dnu) ** 2) + \
        10 * GL * aD ** 4 / (math.pi * m ** 5) + 2 * em + jump + 1e-12
    assert abs(kap.sum() * dnu / (S * (inside - D + C)) - 1.0) < bound


# ---- P9: superposition, scaling, symmetry ----

def test_p9_superposition_scaling_symmetry():
    L = synth.line_list(60, 100.0, seed=9)
    cond = synth.conditions(1200.0, 0.5)
    grid = {"nu_min": 0.0, "dnu": 0.01, "n_points": 10000, "cutoff": 5.0}
    kab, _ = oracle.opacity(L, cond, grid)
    A = {k: v[:25] for k, v in L.items()}
    B = {k: v[25:] for k, v in L.items()}
    ka, _ = oracle.opacity(A, cond, grid)
    kb, _ = oracle.opacity(B, cond, grid)
    m = kab > 0
    assert np.max(np.abs((ka + kb)[m] / kab[m] - 1.0)) < 1e-13
    assert np.all((ka + kb)[~m] == 0)
    L3 = dict(L); L3["S_ref"] = L["S_ref"] * 3.0
    k3, _ = oracle.opacity(L3, cond, grid)
    assert np.max(np.abs(k3[m] / (3.0 * kab[m]) - 1.0)) < 1e-14
    # a line centred on a grid point is mirror symmetric about it
    one = {"nu": np.array([50.0]), "S_ref": np.array([1e-21]), "E_lower": np.array([10.0]),
           "gamma_air": np.array([0.03]), "n_air": np.array([0.6])}
    grid2 = {"nu_min": 0.0, "dnu": 0.0625, "n_points": 1601, "cutoff": 20.0}
    k1, _ = oracle.opacity(one, cond, grid2)
    c = 800
    assert np.max(np.abs(k1[c - 320:c + 1][::-1] / k1[c:c + 321] - 1.0)) < 1e-12


# ---- P10: brute force on a tiny input with the exact Voigt function ----

def test_p10_brute_force_tiny():
    """Independent assembly: kappa_j = sum_i S_i sqrt(ln2/pi) Re w(u+ia)/G_D
    with scipy's Faddeeva function and a window test written from the
    definition.  Difference bounded by the scheme's 5.7e-6."""
    L = synth.line_list(10, 4.0, seed=10)
    cond = synth.conditions(900.0, 0.2)
    grid = {"nu_min": 0.0, "dnu": 0.02, "n_points": 200, "cutoff": 1.5}
    kap, n = oracle.opacity(L, cond, grid)
    T, P = cond["T"], cond["P"]
    ref = np.zeros(200)
    cnt = 0
    ln2 = math.log(2.0)
    for i in range(10):
        nu0 = L["nu"][i]
        S = oracle.line_strength(L["S_ref"][i], L["E_lower"][i], nu0, T, 296.0, cond["q_ratio"])
        GD = nu0 * math.sqrt(2 * ln2 * 1.380649e-16 * T / (18 * 1.66053906660e-24)) / 2.99792458e10
        GL = (T / 296.0) ** (-L["n_air"][i]) * L["gamma_air"][i] * P
        for j in range(200):
            nuj = j * 0.02
            if abs(nuj - nu0) <= 1.5 + 1e-12:
                a = math.sqrt(ln2) * GL / GD
                u = math.sqrt(ln2) * (nuj - nu0) / GD
                ref[j] += S * math.sqrt(ln2 / math.pi) * special.wofz(u + 1j * a).real / GD
                cnt += 1
    assert cnt == n
    m = ref > 0
    assert np.all(kap[~m] == 0)
    assert np.max(np.abs(kap[m] / ref[m] - 1.0)) < 5.7e-6


def test_eval_counts_brute_force():
    L = synth.line_list(40, 30.0, seed=12)
    L["nu"] = L["nu"] + 2000.0  # Doppler cores resolved, 1-node wings inside 10 cm^-1
    cond = synth.conditions(1500.0, 1.0)
    grid = {"nu_min": 2000.0, "dnu": 0.01, "n_points": 3000, "cutoff": 10.0}
    tot, core, g3, g1 = oracle.eval_counts(L, cond, grid)
    assert tot == core + g3 + g1
    n_brute = 0
    for i in range(40):
        lo, hi, n = oracle.window(L["nu"][i], 10.0, 2000.0, 0.01, 3000)
        n_brute += n
    assert tot == n_brute
    _, n = oracle.opacity(L, cond, grid)
    assert n == tot and core > 0 and g3 > 0 and g1 > 0


# ---- P11/P12/P13: k-distribution (§2.2) ----

def test_p11_kdist_equals_counting_definition():
    """eq. (14): y(kappa_0) = N_x / N_nu with N_x = #{kappa <= kappa_0}.  k(g)
    is the smallest bin value whose y reaches g, found here by brute-force
    counting (no sort)."""
    rng = np.random.default_rng(13)
    g, _ = oracle.g_nodes(20)
    for m in (1, 2, 7, 100, 333):
        kap = 10.0 ** rng.uniform(-30, -20, m)
        kap[rng.integers(0, m, m // 5)] = kap[0]  # ties
        k, srt = oracle.kdist_bin(kap, g)
        for q, gq in enumerate(g):
            y = np.array([(kap <= v).sum() / m for v in kap])
            ref = kap[y >= gq].min()
            assert k[q] == ref
        assert np.array_equal(srt, np.sort(kap))


def test_p12_kdist_monotone_constant_permutation():
    rng = np.random.default_rng(14)
    g, _ = oracle.g_nodes(20)
    kap = 10.0 ** rng.uniform(-28, -18, 3 * 1000 + 17)
    k = oracle.kdist(kap, 1000, g)
    assert k.shape == (4, 20)
    assert np.all(np.diff(k, axis=1) >= 0)
    perm = kap.copy()
    for b in range(4):
        seg = perm[b * 1000:(b + 1) * 1000]
        rng.shuffle(seg)
    assert np.array_equal(oracle.kdist(perm, 1000, g), k)
    assert np.all(oracle.kdist(np.full(500, 3.5e-22), 100, g) == 3.5e-22)
    # ragged last bin uses its own size
    k_last, _ = oracle.kdist_bin(kap[3000:], g)
    assert np.array_equal(k[3], k_last)


def test_p13_bin_mean_transmission_invariant_under_sorting():
    """eq. (5): T = int exp(-kappa m) dx = int_0^1 exp(-kappa(y) m) dy; on the
    uniform grid both are bin means, before and after sorting."""
    L = synth.line_list(300, 60.0, seed=15)
    cond = synth.conditions(1500.0, 1.0)
    grid = {"nu_min": 0.0, "dnu": 0.01, "n_points": 6000, "cutoff": 10.0}
    kap, _ = oracle.opacity(L, cond, grid)
    g, wg = oracle.g_nodes(20)
    for b in range(3):
        seg = kap[b * 2000:(b + 1) * 2000]
        _, srt = oracle.kdist_bin(seg, g)
        # column masses 1e-7 .. 1e7 g cm^-2 (§3.4's range); kappa per gram is
        # kappa / (m amu)
        for m_col in np.geomspace(1e-7, 1e7, 15) / (18 * 1.66053906660e-24):
            t_x = np.mean(np.exp(-seg * m_col))
            t_y = np.mean(np.exp(-srt * m_col))
            assert abs(t_x - t_y) <= 1e-14 * max(t_x, 1e-300) + 1e-300


def test_lorentz_width_cutoff_is_the_absolute_cutoff_of_each_line():
    """A cutoff of k Gamma_L per line (§2.4, §3.4) equals, line by line, the
    absolute cutoff k Gamma_L; a no-cutoff grid (cutoff beyond the span)
    takes every line at every point."""
    lines = synth.line_list(6, 300.0, seed=21)
    lines["nu"] = lines["nu"] + 1000.0
    cond = synth.conditions(1200.0, 3.0)
    grid = {"nu_min": 1000.0, "dnu": 0.02, "n_points": 15000, "cutoff": 0.0, "cutoff_lorentz": 40.0}
    kap, n = oracle.opacity(lines, cond, grid)
    total = np.zeros_like(kap)
    n_sum = 0
    for i in range(6):
        one = {k: v[i:i + 1] for k, v in lines.items()}
        GL = oracle.lorentz_hwhm(0.0, one["n_air"][0], one["gamma_air"][0], one["gamma_air"][0],
                                 cond["T"], cond["T0"], cond["P"], cond["P_self"])
        g1 = dict(grid, cutoff=40.0 * GL, cutoff_lorentz=0.0)
        k1, n1 = oracle.opacity(one, cond, g1)
        total += k1
        n_sum += n1
        lo, hi = oracle.window(one["nu"][0], 40.0 * GL, grid["nu_min"], grid["dnu"], grid["n_points"])[:2]
        assert n1 == hi - lo + 1
    assert n == n_sum
    assert np.allclose(kap, total, rtol=1e-14, atol=0)
    # no cutoff: every line at every point
    big = dict(grid, cutoff=1e9, cutoff_lorentz=0.0)
    _, nb = oracle.opacity(lines, cond, big)
    assert nb == 6 * grid["n_points"]


def test_p12b_midpoint_linear_rule_pins():
    """Rule 1: the i-th smallest at y_i = (i + 1/2)/M, straight lines between
    neighbours, end values held.  Pinned by numpy.interp (a library's
    piecewise-linear interpolation), exact dyadic nodes, a closed form on
    evenly spaced values and the one-value bin."""
    rng = np.random.default_rng(41)
    g = np.concatenate([oracle.g_nodes(20)[0], [1e-9, 0.3e-3, 0.5, 0.9995, 1 - 1e-12]])
    for m in (1, 2, 3, 1000, 4097):
        kap = 10.0 ** rng.uniform(-28, -18, m)
        kap[: m // 3] = kap[0]  # ties
        k, srt = oracle.kdist_bin(kap, g, rule=1)
        srt_ref = np.sort(kap)
        ref = np.interp(g, (np.arange(m) + 0.5) / m, srt_ref)
        # numpy rounds in the abscissa (x - x_j), which the slope amplifies:
        # allow (M + 1) eps of the larger neighbour, a few times over
        i = np.clip(np.floor(g * m - 0.5).astype(np.int64), 0, m - 1)
        nb = np.maximum(srt_ref[i], srt_ref[np.minimum(i + 1, m - 1)])
        assert np.all(np.abs(k - ref) <= 8 * (m + 1) * np.finfo(float).eps * nb), m
        assert np.all(np.diff(k[np.argsort(g)]) >= 0)
        assert np.array_equal(srt, np.sort(kap))
    # dyadic: g = (i + 1/2)/1024 is exact, so k is the i-th smallest exactly
    m = 1024
    kap = rng.permutation(10.0 ** rng.uniform(-25, -20, m))
    i = np.array([0, 1, 17, 511, 1022, 1023])
    k, srt = oracle.kdist_bin(kap, (i + 0.5) / m, rule=1)
    assert np.array_equal(k, srt[i])
    # evenly spaced values a + b i: k(g) = a + b (g M - 1/2), clamped to the ends
    a, b, m = 2.0, 0.25, 64
    kap = rng.permutation(a + b * np.arange(m))
    gg = np.linspace(0.001, 0.999, 97)
    ref = a + b * np.clip(gg * m - 0.5, 0, m - 1)
    assert np.allclose(oracle.kdist_bin(kap, gg, rule=1)[0], ref, rtol=0, atol=1e-14)
    # the step rule and the linear rule agree on a constant bin and on M = 1
    assert np.all(oracle.kdist(np.full(500, 3.5e-22), 100, g, rule=1) == 3.5e-22)
    assert np.all(oracle.kdist_bin([7.0], g, rule=1)[0] == 7.0)
    # whole grid with a ragged last bin = per-bin calls
    kap = 10.0 ** rng.uniform(-28, -18, 3 * 1000 + 17)
    k = oracle.kdist(kap, 1000, g, rule=1)
    assert np.array_equal(k[3], oracle.kdist_bin(kap[3000:], g, rule=1)[0])
    with pytest.raises(ValueError):
        oracle.kdist_bin(kap, g, rule=2)


def _scheme_constants():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "scheme_constants.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, value, section = line.split()[:3]
            assert section.startswith("§"), line
            out[name] = float(value)
    return out


def test_golden_scheme_constants():
    """The oracle against the numbers the paper prints (tests/golden)."""
    c = _scheme_constants()
    # region thresholds: H_V is the series just below a^2 + u^2 = 100, the
    # 3-node rule from there, the 1-node rule from 1e6 on (exact branches)
    for a in (0.0, 0.3, 4.0):
        for r2, below, above in ((c["core_region_r2"], oracle.voigt_series, oracle.voigt_gh3),
                                 (c["gh1_region_r2"], oracle.voigt_gh3, oracle.voigt_gh1)):
            u = math.sqrt(r2 - a * a)
            lo, hi = u * (1 - 1e-9), u * (1 + 1e-9)
            assert a * a + lo * lo < r2 <= a * a + hi * hi
            assert oracle.voigt_H(a, lo)[0] == below(a, lo)[0]
            assert oracle.voigt_H(a, hi)[0] == above(a, hi)[0]
    # reference conditions: S(T0) = S0 and, at T0 and P0 with no self
    # broadening or natural width, Gamma_L is the tabulated coefficient
    T0, P0 = c["reference_temperature_K"], c["reference_pressure_atm"]
    assert synth.conditions(1500.0, 1.0)["T0"] == T0
    assert oracle.line_strength(3.7e-21, 1234.5, 2500.0, T0, T0)[()] == 3.7e-21
    g = oracle.lorentz_hwhm(0.0, 0.6, 0.0731, 0.31, T0, T0, P0, 0.0)[()]
    assert abs(g - 0.0731) <= 1e-16
    # the Lorentz-width cutoff: 500 widths is the absolute cutoff 500 Gamma_L
    L = {"nu": np.array([1000.0]), "S_ref": np.array([1e-20]), "E_lower": np.array([300.0]),
         "gamma_air": np.array([0.05]), "n_air": np.array([0.5])}
    cond = synth.conditions(1500.0, 0.01)
    GL = oracle.lorentz_hwhm(0.0, 0.5, 0.05, 0.05, cond["T"], cond["T0"], cond["P"], cond["P_self"])[()]
    n_w = c["lorentz_cutoff_widths"]
    grid = {"nu_min": 990.0, "dnu": 1e-4, "n_points": 200001, "cutoff": 0.0, "cutoff_lorentz": n_w}
    k1, e1 = oracle.opacity(L, cond, grid)
    k2, e2 = oracle.opacity(L, cond, dict(grid, cutoff=n_w * GL, cutoff_lorentz=0.0))
    assert e1 == e2 and np.array_equal(k1, k2) and 0 < e1 < grid["n_points"]
    # the resampling's coefficient count
    from oracle import resample
    assert len(resample.fit_bin(np.sort(10.0 ** np.random.default_rng(5).uniform(-25, -20, 500)))) == \
        int(c["chebyshev_coefficients"])
