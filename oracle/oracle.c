/*
 * oracle.c -- plain FP64 CPU oracle for the HELIOS-K line-by-line opacity and
 * k-distribution method (Grimm & Heng 2015, arXiv:1503.03806).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product library.  It is written
 * for a reader holding the paper: each function names the section and
 * equation it follows and uses the paper's notation (Gamma_D, Gamma_L, a, u,
 * H_V).  No blocking, fusion or reordering beyond what the formulas state;
 * a per-term exp() in the series, a division per evaluation.
 *
 * Readings of the paper taken here (where it is silent or garbled):
 *  - The H_V integrand of eq. (19) carries exp(-u'^2) (the printed sign makes
 *    the integral diverge).
 *  - Delta E of eq. (18) is the lower-state energy E'' in cm^-1, so
 *    Delta E / (k_B T) = c2 E'' / T with c2 = h c / k_B.
 *  - "Third-order" / "first-order" Gauss-Hermite quadrature (§2.4) are the
 *    3-node and 1-node rules for the weight exp(-t^2).
 *  - Region switch on a^2 + u^2 exactly at 100 and 1e6 (§2.4).
 *  - The core region uses a series form of the Faddeeva function equivalent
 *    to Algorithm 916's ingredients (cos, sin, erfcx and three exponential
 *    series summed in one loop, §2.4).  It is derived from the textbook
 *    series for the error function of complex argument (Abramowitz & Stegun
 *    7.1.29) applied to w(z) = exp(-z^2) erfc(-iz), with step h = 1/2 and
 *    n = 1 .. 2*ceil(|u|) + 14 terms.
 *  - Cutoff window: the closed interval of grid indices within the cutoff of
 *    the pressure-shifted centre, plain truncation, no renormalisation.
 *  - The unshifted centre enters Gamma_D and S(T); the shifted one the
 *    profile.  Grid points are nu_j = nu_min + j * dnu (point sampling).
 *  - k(g) step rule: g_i = (i+1)/M for the i-th smallest of M values,
 *    k(g) = kappa_(ceil(g M) - 1).  The midpoint-linear rule places the
 *    i-th smallest at (i + 1/2)/M (the Chebyshev fit's abscissae, §2.6) and
 *    joins neighbours by straight lines, holding the end values.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018: c, k_B and h are exact; the atomic mass unit is recommended. */
static const double C_LIGHT = 2.99792458e10;   /* cm s^-1 */
static const double K_BOLTZ = 1.380649e-16;    /* erg K^-1 */
static const double H_PLANCK = 6.62607015e-27; /* erg s */
static const double AMU = 1.66053906660e-24;   /* g */
static const double P0_ATM = 1.0;              /* reference pressure, §2.3 */

double ora_const(int which)
{
    switch (which) {
    case 0: return C_LIGHT;
    case 1: return K_BOLTZ;
    case 2: return H_PLANCK;
    case 3: return AMU;
    case 4: return H_PLANCK * C_LIGHT / K_BOLTZ;
    default: return NAN;
    }
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (n >= 1); returns the count in
 * effect afterwards.  Results do not depend on it: every point and bin is
 * computed by one thread in the same order. */
int ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return ora_num_threads();
}

/* ---------------------------------------------------------------- §2.3 -- */

/* eq. (18): S/S0 = (Q0/Q) exp(-dE/kT + dE/kT0) [1-exp(-hc nu/kT)] /
 * [1-exp(-hc nu/kT0)].  1 - exp(-z) is written -expm1(-z) so that the ratio
 * stays exact as nu -> 0 (it tends to T0/T). */
double ora_line_strength(double S0, double E_lower, double nu, double T,
                         double T0, double q_ratio)
{
    const double c2 = H_PLANCK * C_LIGHT / K_BOLTZ;
    double boltz = exp(-c2 * E_lower / T + c2 * E_lower / T0);
    double stim = expm1(-c2 * nu / T) / expm1(-c2 * nu / T0);
    return S0 * q_ratio * boltz * stim;
}

/* eq. (19): Gamma_D = nu0 sqrt(2 ln2 k_B T / m) / c. */
double ora_doppler_hwhm(double nu, double T, double mass_amu)
{
    double m = mass_amu * AMU;
    return nu * sqrt(2.0 * log(2.0) * K_BOLTZ * T / m) / C_LIGHT;
}

/* eq. (20): Gamma_L = A21/(4 pi c) + (T/T0)^(-n) [g_air (P - Ps)/P0 +
 * g_self Ps/P0]. */
double ora_lorentz_hwhm(double A21, double n_coll, double gamma_air,
                        double gamma_self, double T, double T0, double P,
                        double P_self)
{
    double natural = A21 / (4.0 * M_PI * C_LIGHT);
    double pressure = pow(T / T0, -n_coll) *
                      (gamma_air * (P - P_self) / P0_ATM +
                       gamma_self * P_self / P0_ATM);
    return natural + pressure;
}

/* ---------------------------------------------------------------- §2.4 -- */

double ora_erfcx(double t)
{
    /* exp(t^2) erfc(t); adequate for 0 <= t < 26, which covers the core
     * region (a < 10). */
    return exp(t * t) * erfc(t);
}

/* Core region: H_V(a,u) = Re w(u + i a) by the series form (see header).
 * With x = |u|, y = a, h = 1/2 and N = 2 ceil(x) + 14:
 *   H = e^{-x^2} erfcx(y) cos(2xy) + (2h/pi) e^{-x^2} sin^2(xy) / y
 *     + (2h/pi) [ -y cos(2xy) S1 + (y/2)(S2 + S3) ],
 *   S1 = sum e^{-(h^2 n^2 + x^2)} / (h^2 n^2 + y^2),
 *   S2 = sum e^{-(h n + x)^2}    / (h^2 n^2 + y^2),
 *   S3 = sum e^{-(h n - x)^2}    / (h^2 n^2 + y^2).
 * The three series share one loop, as §2.4 describes for Algorithm 916. */
double ora_voigt_series(double a, double u)
{
    const double h = 0.5;
    double x = fabs(u), y = a;
    int N = 2 * (int)ceil(x) + 14;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int n = 1; n <= N; ++n) {
        double hn = h * n;
        double den = hn * hn + y * y;
        s1 += exp(-(hn * hn + x * x)) / den;
        s2 += exp(-(hn + x) * (hn + x)) / den;
        s3 += exp(-(hn - x) * (hn - x)) / den;
    }
    double ex2 = exp(-x * x);
    double t0 = ex2 * ora_erfcx(y) * cos(2.0 * x * y);
    double t1 = 0.0;
    if (y > 0.0) {
        double s = sin(x * y);
        t1 = (2.0 * h / M_PI) * ex2 * s * s / y;
    }
    double t2 = (2.0 * h / M_PI) * (-y * cos(2.0 * x * y) * s1 +
                                     0.5 * y * (s2 + s3));
    return t0 + t1 + t2;
}

/* H_V = (a/pi) int exp(-t^2) / ((u - t)^2 + a^2) dt by Gauss-Hermite
 * quadrature.  The 3-node rule has nodes 0, +-sqrt(3/2) (roots of
 * H_3(t) = 8t^3 - 12t) and weights 2 sqrt(pi)/3, sqrt(pi)/6. */
double ora_voigt_gh3(double a, double u)
{
    const double t1 = sqrt(1.5);
    const double w0 = 2.0 * sqrt(M_PI) / 3.0;
    const double w1 = sqrt(M_PI) / 6.0;
    double d0 = u * u + a * a;
    double dm = (u - t1) * (u - t1) + a * a;
    double dp = (u + t1) * (u + t1) + a * a;
    return (a / M_PI) * (w0 / d0 + w1 / dm + w1 / dp);
}

/* 1-node rule: node 0, weight sqrt(pi). */
double ora_voigt_gh1(double a, double u)
{
    return (a / M_PI) * (sqrt(M_PI) / (u * u + a * a));
}

double ora_voigt_H(double a, double u)
{
    double r = a * a + u * u;
    if (r < 100.0) return ora_voigt_series(a, u);
    if (r < 1.0e6) return ora_voigt_gh3(a, u);
    return ora_voigt_gh1(a, u);
}

int ora_voigt_vec(int which, int64_t n, const double* a, const double* u,
                  double* out)
{
    if (n < 0 || (n > 0 && (!a || !u || !out))) return -1;
    for (int64_t i = 0; i < n; ++i) {
        switch (which) {
        case 0: out[i] = ora_voigt_H(a[i], u[i]); break;
        case 1: out[i] = ora_voigt_series(a[i], u[i]); break;
        case 2: out[i] = ora_voigt_gh3(a[i], u[i]); break;
        case 3: out[i] = ora_voigt_gh1(a[i], u[i]); break;
        default: return -1;
        }
    }
    return 0;
}

int64_t ora_window(double nu0_shifted, double cutoff, double nu_min,
                   double dnu, int64_t n_points, int64_t* lo, int64_t* hi)
{
    double flo = ceil((nu0_shifted - cutoff - nu_min) / dnu);
    double fhi = floor((nu0_shifted + cutoff - nu_min) / dnu);
    if (flo < 0.0) flo = 0.0;
    if (fhi > (double)(n_points - 1)) fhi = (double)(n_points - 1);
    if (fhi < flo) {
        *lo = 0;
        *hi = -1;
        return 0;
    }
    *lo = (int64_t)flo;
    *hi = (int64_t)fhi;
    return *hi - *lo + 1;
}

/* ------------------------------------------------------- opacity grid -- */

typedef struct {
    double nu;  /* for sorting */
    int64_t idx;
} key_t_;

static int cmp_key(const void* pa, const void* pb)
{
    const key_t_* a = (const key_t_*)pa;
    const key_t_* b = (const key_t_*)pb;
    if (a->nu < b->nu) return -1;
    if (a->nu > b->nu) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

typedef struct {
    int64_t n;
    double* nu;     /* unshifted centre, ascending */
    double* nu0p;   /* shifted centre */
    double* S;      /* S(T) */
    double* GD;     /* Gamma_D */
    double* GL;     /* Gamma_L */
    int64_t* wlo;
    int64_t* whi;
    double max_shift;
    double max_cut;  /* largest cutoff over the lines */
} prepped_t;

static void free_prepped(prepped_t* p)
{
    free(p->nu); free(p->nu0p); free(p->S); free(p->GD); free(p->GL);
    free(p->wlo); free(p->whi);
}

static int check_inputs(const ora_lines* L, const ora_conditions* c,
                        const ora_grid* g)
{
    if (!L || !c || !g) return -1;
    if (L->n < 0) return -1;
    if (L->n > 0 && (!L->nu || !L->S_ref || !L->E_lower || !L->gamma_air ||
                     !L->n_air))
        return -1;
    if (!(c->T > 0.0) || !(c->T0 > 0.0) || !(c->mass_amu > 0.0) ||
        !(c->P >= 0.0) || !(c->P_self >= 0.0) || !(c->P_self <= c->P) ||
        !(c->q_ratio > 0.0))
        return -1;
    if (!(g->dnu > 0.0) || g->n_points < 0 || !(g->cutoff >= 0.0)) return -1;
    if (!(g->cutoff_lorentz >= 0.0) || !isfinite(g->cutoff_lorentz)) return -1;
    for (int64_t i = 0; i < L->n; ++i)
        if (!(L->nu[i] > 0.0)) return -1;
    return 0;
}

/* "Line" stage of Fig. 5: per-line S(T), Gamma_D, Gamma_L, shifted centre
 * and cutoff window, in ascending (nu, index) order. */
static int prep_lines(const ora_lines* L, const ora_conditions* c,
                      const ora_grid* g, prepped_t* p)
{
    int64_t n = L->n;
    memset(p, 0, sizeof(*p));
    p->n = n;
    size_t nb = (size_t)(n > 0 ? n : 1);
    key_t_* keys = (key_t_*)malloc(nb * sizeof(key_t_));
    p->nu = (double*)malloc(nb * sizeof(double));
    p->nu0p = (double*)malloc(nb * sizeof(double));
    p->S = (double*)malloc(nb * sizeof(double));
    p->GD = (double*)malloc(nb * sizeof(double));
    p->GL = (double*)malloc(nb * sizeof(double));
    p->wlo = (int64_t*)malloc(nb * sizeof(int64_t));
    p->whi = (int64_t*)malloc(nb * sizeof(int64_t));
    if (!keys || !p->nu || !p->nu0p || !p->S || !p->GD || !p->GL || !p->wlo ||
        !p->whi) {
        free(keys);
        free_prepped(p);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) {
        keys[i].nu = L->nu[i];
        keys[i].idx = i;
    }
    qsort(keys, (size_t)n, sizeof(key_t_), cmp_key);
    p->max_shift = 0.0;
    p->max_cut = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = keys[k].idx;
        double nu = L->nu[i];
        double gs = L->gamma_self ? L->gamma_self[i] : L->gamma_air[i];
        double dl = L->delta ? L->delta[i] : 0.0;
        double A = L->A21 ? L->A21[i] : 0.0;
        p->nu[k] = nu;
        p->S[k] = ora_line_strength(L->S_ref[i], L->E_lower[i], nu, c->T,
                                    c->T0, c->q_ratio);
        p->GD[k] = ora_doppler_hwhm(nu, c->T, c->mass_amu);
        p->GL[k] = ora_lorentz_hwhm(A, L->n_air[i], L->gamma_air[i], gs, c->T,
                                    c->T0, c->P, c->P_self);
        /* eq. (21): nu0 -> nu0 + delta P / P0 */
        p->nu0p[k] = nu + dl * c->P / P0_ATM;
        double shift = fabs(p->nu0p[k] - nu);
        if (shift > p->max_shift) p->max_shift = shift;
        /* the cutoff: absolute, or a multiple of the line's Lorentz HWHM */
        double cut = g->cutoff_lorentz > 0.0 ? g->cutoff_lorentz * p->GL[k] : g->cutoff;
        if (cut > p->max_cut) p->max_cut = cut;
        ora_window(p->nu0p[k], cut, g->nu_min, g->dnu, g->n_points,
                   &p->wlo[k], &p->whi[k]);
    }
    free(keys);
    return 0;
}

/* First index k with nu[k] >= v. */
static int64_t lower_bound(const double* nu, int64_t n, double v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (nu[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

int64_t ora_opacity(const ora_lines* L, const ora_conditions* c,
                    const ora_grid* g, int64_t j_begin, int64_t j_end,
                    double* kappa_out)
{
    if (check_inputs(L, c, g) != 0) return -1;
    if (j_begin < 0 || j_end < j_begin || j_end > g->n_points) return -1;
    if (j_end > j_begin && !kappa_out) return -1;
    prepped_t p;
    if (prep_lines(L, c, g, &p) != 0) return -2;

    const double sqrt_ln2 = sqrt(log(2.0));
    const double phi_norm = sqrt(log(2.0) / M_PI);
    /* A line can reach point j only if its unshifted centre lies within
     * cutoff + max shift of nu_j; one grid step of slack covers the
     * rounding of the window bounds.  Each candidate is then tested against
     * its exact window. */
    const double reach = p.max_cut + p.max_shift + g->dnu;
    int64_t total = 0;

#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t j = j_begin; j < j_end; ++j) {
        double nu_j = g->nu_min + (double)j * g->dnu;
        double kappa = 0.0;
        int64_t k = lower_bound(p.nu, p.n, nu_j - reach);
        for (; k < p.n && p.nu[k] <= nu_j + reach; ++k) {
            if (j < p.wlo[k] || j > p.whi[k]) continue;
            /* eq. (19): a, u and Phi = sqrt(ln2/pi) H_V / Gamma_D;
             * eq. (16): kappa = S Phi. */
            double a = sqrt_ln2 * p.GL[k] / p.GD[k];
            double u = sqrt_ln2 * (nu_j - p.nu0p[k]) / p.GD[k];
            double phi = phi_norm * ora_voigt_H(a, u) / p.GD[k];
            kappa += p.S[k] * phi;
            total += 1;
        }
        kappa_out[j - j_begin] = kappa;
    }
    free_prepped(&p);
    return total;
}

int ora_eval_counts(const ora_lines* L, const ora_conditions* c,
                    const ora_grid* g, int64_t counts[4])
{
    if (check_inputs(L, c, g) != 0 || !counts) return -1;
    prepped_t p;
    if (prep_lines(L, c, g, &p) != 0) return -2;
    const double sqrt_ln2 = sqrt(log(2.0));
    int64_t tot = 0, core = 0, gh3 = 0, gh1 = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : tot, core, gh3, gh1)
    for (int64_t k = 0; k < p.n; ++k) {
        double a = sqrt_ln2 * p.GL[k] / p.GD[k];
        for (int64_t j = p.wlo[k]; j <= p.whi[k]; ++j) {
            double nu_j = g->nu_min + (double)j * g->dnu;
            double u = sqrt_ln2 * (nu_j - p.nu0p[k]) / p.GD[k];
            double r = a * a + u * u;
            tot += 1;
            if (r < 100.0) core += 1;
            else if (r < 1.0e6) gh3 += 1;
            else gh1 += 1;
        }
    }
    counts[0] = tot;
    counts[1] = core;
    counts[2] = gh3;
    counts[3] = gh1;
    free_prepped(&p);
    return 0;
}

/* ---------------------------------------------------------------- §2.2 -- */

/* Gauss-Legendre nodes: roots of P_n by Newton's method, with P_n and P_n'
 * from the three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1};
 * weights 2 / ((1 - x^2) P_n'(x)^2).  Nodes ascending. */
int ora_gauss_legendre(int n, double* x, double* w)
{
    if (n < 1 || !x || !w) return -1;
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            /* P_n = p1, P_{n-1} = p0 */
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 1; k < n; ++k) {
                double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

static int cmp_double(const void* pa, const void* pb)
{
    double a = *(const double*)pa, b = *(const double*)pb;
    return (a > b) - (a < b);
}

int ora_kdist_bin(const double* kappa, int64_t m, int n_g, const double* g,
                  int rule, double* k_out, double* sorted_out)
{
    if (m < 1 || n_g < 0 || !kappa || (n_g > 0 && (!g || !k_out))) return -1;
    if (rule != 0 && rule != 1) return -1;
    double* s = (double*)malloc((size_t)m * sizeof(double));
    if (!s) return -2;
    memcpy(s, kappa, (size_t)m * sizeof(double));
    qsort(s, (size_t)m, sizeof(double), cmp_double);
    for (int q = 0; q < n_g; ++q) {
        if (!(g[q] > 0.0) || !(g[q] < 1.0)) {
            free(s);
            return -1;
        }
        if (rule == 0) {
            /* smallest rank i with g_i = (i+1)/m >= g_q */
            int64_t r = (int64_t)ceil(g[q] * (double)m) - 1;
            if (r < 0) r = 0;
            if (r > m - 1) r = m - 1;
            k_out[q] = s[r];
        } else {
            /* the i-th smallest value sits at y_i = (i + 1/2)/m; straight
             * line between neighbours, the end values held beyond y_0 and
             * y_{m-1}.  u = g m - 1/2 is g in units of the spacing from y_0. */
            double u = g[q] * (double)m - 0.5;
            double fl = floor(u);
            if (u <= 0.0) {
                k_out[q] = s[0];
            } else if (fl >= (double)(m - 1)) {
                k_out[q] = s[m - 1];
            } else {
                int64_t i = (int64_t)fl;
                double f = u - fl;
                k_out[q] = s[i] + f * (s[i + 1] - s[i]);
            }
        }
    }
    if (sorted_out) memcpy(sorted_out, s, (size_t)m * sizeof(double));
    free(s);
    return 0;
}

int ora_kdist(const double* kappa, int64_t n_points, int64_t points_per_bin,
              int n_g, const double* g, int rule, double* k_out)
{
    if (n_points < 1 || points_per_bin < 1) return -1;
    int64_t n_bins = (n_points + points_per_bin - 1) / points_per_bin;
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rc)
    for (int64_t b = 0; b < n_bins; ++b) {
        int64_t j0 = b * points_per_bin;
        int64_t m = n_points - j0 < points_per_bin ? n_points - j0
                                                   : points_per_bin;
        rc |= ora_kdist_bin(kappa + j0, m, n_g, g, rule, k_out + b * n_g, NULL);
    }
    return rc ? -1 : 0;
}
