/*
 * oracle.h -- plain FP64 CPU oracle for the line-by-line opacity and
 * k-distribution method of Grimm & Heng (2015), "HELIOS-K: an ultrafast,
 * open-source opacity calculator for radiative transfer" (arXiv:1503.03806).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library (include/hk.h); the two are
 * compared, never combined.
 *
 * Everything is IEEE binary64, built without fast-math and without
 * floating-point contraction, so each expression is evaluated exactly as it
 * is written.  Units: wavenumbers, widths and cutoffs in cm^-1, pressure in
 * atm, temperature in K, line strength in cm/molecule, opacity (a cross
 * section) in cm^2/molecule.
 */
#ifndef HK_ORACLE_H
#define HK_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Physical constants (CGS; CODATA 2018 exact values or recommended). */
double ora_const(int which); /* 0 c, 1 k_B, 2 h, 3 amu, 4 c2 = h c / k_B */

/* Line strength at temperature T from its value S0 at T0, §2.3 eq. (18).
 * E_lower is the lower-state energy in cm^-1 (the paper's Delta E, read as
 * E''), q_ratio = Q(T0)/Q(T). */
double ora_line_strength(double S0, double E_lower, double nu, double T,
                         double T0, double q_ratio);

/* Doppler half-width at half maximum Gamma_D, §2.3 eq. (19). */
double ora_doppler_hwhm(double nu, double T, double mass_amu);

/* Lorentz half-width Gamma_L including natural and pressure broadening,
 * §2.3 eq. (20); pressures in atm, reference pressure P0 = 1 atm. */
double ora_lorentz_hwhm(double A21, double n_coll, double gamma_air,
                        double gamma_self, double T, double T0, double P,
                        double P_self);

/* Voigt function H_V(a,u) of §2.3 eq. (19) evaluated by the three-region
 * scheme of §2.4: series form of the Faddeeva function for a^2+u^2 < 100,
 * 3-node Gauss-Hermite for 100 <= a^2+u^2 < 1e6, 1-node beyond. */
double ora_voigt_H(double a, double u);
/* The pieces of that scheme, exposed for the pins. */
double ora_voigt_series(double a, double u);  /* core series, any (a,u) */
double ora_voigt_gh3(double a, double u);
double ora_voigt_gh1(double a, double u);
/* Vector form for tests: which = 0 scheme, 1 series, 2 GH3, 3 GH1. */
int ora_voigt_vec(int which, int64_t n, const double* a, const double* u,
                  double* out);
/* Scaled complementary error function exp(t^2) erfc(t), t >= 0, t < 26. */
double ora_erfcx(double t);

/* Cutoff window of a line in grid-index space: the closed interval
 * [ceil((nu0 - cut - nu_min)/dnu), floor((nu0 + cut - nu_min)/dnu)]
 * intersected with [0, n_points).  Returns the number of points (0 if
 * empty) and stores the bounds. */
int64_t ora_window(double nu0_shifted, double cutoff, double nu_min,
                   double dnu, int64_t n_points, int64_t* lo, int64_t* hi);

/* Line list and conditions, mirroring the paper's problem statement. */
typedef struct {
    int64_t n;
    const double* nu;         /* line centre at zero pressure, cm^-1 */
    const double* S_ref;      /* line strength at T0, cm/molecule */
    const double* E_lower;    /* lower-state energy, cm^-1 */
    const double* gamma_air;  /* air-broadened HWHM at T0 and P0, cm^-1/atm */
    const double* n_air;      /* temperature exponent of the widths */
    const double* gamma_self; /* self-broadened HWHM; NULL -> gamma_air */
    const double* delta;      /* pressure shift, cm^-1/atm; NULL -> 0 */
    const double* A21;        /* Einstein A coefficient, s^-1; NULL -> 0 */
} ora_lines;

typedef struct {
    double T0;       /* reference temperature of the line list (296 K) */
    double mass_amu; /* molecular mass */
    double T;        /* K */
    double P;        /* atm */
    double P_self;   /* atm */
    double q_ratio;  /* Q(T0)/Q(T) */
} ora_conditions;

typedef struct {
    double nu_min;
    double dnu;
    int64_t n_points;
    double cutoff;          /* cm^-1, used when cutoff_lorentz == 0 */
    double cutoff_lorentz;  /* > 0: each line's cutoff is this many Gamma_L (§2.4, §3.4) */
} ora_grid;

/* Opacity kappa_j for the grid points j in [j_begin, j_end), written to
 * kappa_out[0 .. j_end-j_begin).  kappa_j = sum over lines whose cutoff window
 * contains j, in ascending (nu, original index) order, of S(T) Phi(nu_j)
 * (§2.3 eq. (16), §2.4).  Returns the number of line-point evaluations or a
 * negative value on invalid input.  Runs on all OpenMP threads. */
int64_t ora_opacity(const ora_lines* lines, const ora_conditions* cond,
                    const ora_grid* grid, int64_t j_begin, int64_t j_end,
                    double* kappa_out);

/* Count of line-point evaluations sum_i |W_i| and its split by region
 * (core series, 3-node, 1-node) over the whole grid; counts[0..3]. */
int ora_eval_counts(const ora_lines* lines, const ora_conditions* cond,
                    const ora_grid* grid, int64_t counts[4]);

/* Gauss-Legendre nodes and weights on [-1, 1]. */
int ora_gauss_legendre(int n, double* x, double* w);

/* k-distribution of §2.2 for one bin of m opacity values: sort ascending,
 * cumulative coordinate g_i = (i+1)/m (eq. (14) with delta y = 1/N_nu,
 * eq. (15)), and, for the n_g given g values in (0, 1):
 *   rule 0 (step):  k(g_q) = kappa_sorted[ceil(g_q m) - 1];
 *   rule 1 (midpoint-linear): the i-th smallest sits at y_i = (i + 1/2)/m,
 *     k(g_q) interpolates linearly between neighbouring y_i and holds
 *     kappa_sorted[0] below y_0 and kappa_sorted[m-1] above y_{m-1}.
 * sorted_out may be NULL. */
int ora_kdist_bin(const double* kappa, int64_t m, int n_g, const double* g,
                  int rule, double* k_out, double* sorted_out);

/* k-distribution of a whole grid cut into consecutive bins of
 * points_per_bin points (the last bin may be shorter).  k_out is
 * [n_bins][n_g]. */
int ora_kdist(const double* kappa, int64_t n_points, int64_t points_per_bin,
              int n_g, const double* g, int rule, double* k_out);

int ora_num_threads(void);
int ora_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
