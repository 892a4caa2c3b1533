/*
 * hk.h -- C ABI of the MI355X (gfx950) line-by-line opacity and
 * k-distribution library.
 *
 * The method is that of Grimm & Heng (2015), "HELIOS-K: an ultrafast,
 * open-source opacity calculator for radiative transfer", arXiv:1503.03806:
 * a line list goes in; for given temperature and pressure every line's
 * strength and widths are scaled (§2.3), its Voigt profile is evaluated at
 * every grid point within the line-wing cutoff and summed into the opacity
 * function (§2.4, §2.5), and each wavenumber bin is reduced to its
 * k-distribution (§2.2, §2.6).
 *
 * Conventions
 *  - Every call returns an int status: HK_OK (0) or a negative HK_E* code.
 *    hk_last_error() gives a message.  No C++ exception crosses the ABI.
 *  - Host pointers are marked [host], device pointers [device].  The caller
 *    owns every buffer it passes; the context owns only its private device
 *    copy of the line list and its scratch space.
 *  - Device work is enqueued on the context's HIP stream (hk_set_stream) and
 *    is asynchronous; hk_sync() waits for it.  Calls on one context must not
 *    overlap (one host thread per context).
 *  - Units: wavenumber, widths, cutoff in cm^-1; gamma in cm^-1/atm; pressure
 *    in atm (the reference pressure P0 is 1 atm); temperature in K; line
 *    strength S in cm/molecule; the opacity written is a cross section in
 *    cm^2/molecule (divide by the molecular mass for cm^2/g, §2.3).
 *  - Grid points are nu_j = nu_min + j * dnu, j = 0 .. n_points-1 (uniform
 *    spacing, §2.2).
 */
#ifndef HK_H
#define HK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HK_OK 0
#define HK_EINVAL (-1)        /* invalid argument; nothing was enqueued */
#define HK_ENOMEM (-2)        /* device or host allocation failed */
#define HK_EDEVICE (-3)       /* a HIP runtime call failed */
#define HK_EUNSUPPORTED (-4)  /* valid request the library does not provide */
#define HK_ENOTREADY (-5)     /* call order: e.g. opacity before lines */

#define HK_MAX_G 64           /* most g values per k-distribution */

typedef struct hk_ctx hk_ctx;

/* Arithmetic of the profile evaluation and accumulation. */
typedef enum {
    HK_F64 = 0,          /* everything in binary64 */
    HK_F32_KAHAN = 1,    /* binary32 profiles, compensated binary32 sums;
                            line strengths, widths and outputs in binary64 */
    HK_F32_SURROGATE = 2 /* HK_F32_KAHAN, with the learned surrogate in place
                            of the series wherever it is certified */
} hk_precision;

/* Line list, §2.3 (the HITRAN/HITEMP fields the method uses).  [host]
 * arrays of n values each.  Optional arrays may be NULL. */
typedef struct {
    int64_t n;
    const double* nu;         /* line centre at zero pressure, > 0 */
    const double* S_ref;      /* line strength at T_ref, >= 0 */
    const double* E_lower;    /* lower-state energy E'' (the paper's Delta E) */
    const double* gamma_air;  /* air-broadened HWHM at T_ref and P0, >= 0 */
    const double* n_air;      /* temperature exponent of the widths */
    const double* gamma_self; /* self-broadened HWHM; NULL: gamma_air */
    const double* delta;      /* pressure shift per atm (eq. 21); NULL: 0 */
    const double* A21;        /* Einstein A coefficient, s^-1; NULL: 0 */
} hk_lines;

typedef struct {
    double T_ref;     /* reference temperature of S_ref, gamma (296 K) */
    double mass_amu;  /* molecular mass in atomic mass units, > 0 */
} hk_species;

/* One thermodynamic state. */
typedef struct {
    double T;        /* K, > 0 */
    double P;        /* total pressure, atm, >= 0 */
    double P_self;   /* self-broadening partial pressure, 0 <= P_self <= P */
    double q_ratio;  /* partition-function ratio Q(T_ref)/Q(T), > 0 */
    double abundance; /* weight X_s >= 0 of this species in a mixture: the
                         opacity is X_s kappa_s, so that a mixture's is
                         sum_s X_s kappa_s (§2.1; hk_opacity with accumulate
                         over the species' line lists); 1 for one species */
} hk_state;

typedef struct {
    double nu_min;     /* first grid point */
    double dnu;        /* spacing, > 0 */
    int64_t n_points;  /* 0 <= n_points <= HK_MAX_POINTS */
    double cutoff;     /* absolute line-wing cutoff, >= 0 (§2.4, §3.4) */
    double cutoff_lorentz; /* > 0: each line's cutoff is this many of its own
                              Lorentz HWHM Gamma_L instead (§2.4: 500 Gamma_L);
                              0: the absolute cutoff.  A cutoff beyond the grid's
                              span is no cutoff (every line at every point). */
} hk_grid;
#define HK_MAX_POINTS ((int64_t)1 << 30)

/* Bins of consecutive grid points, the g values at which k(g) is reported
 * and the rule that reads k(g) off a sorted bin.  The last bin may hold
 * fewer than points_per_bin points. */
typedef struct {
    int64_t points_per_bin;  /* >= 1 */
    int32_t n_g;             /* 1 .. HK_MAX_G */
    const double* g;         /* [host] n_g values, each in (0, 1) */
    int32_t rule;            /* HK_RULE_STEP or HK_RULE_LINEAR */
} hk_bins;
/* k(g) from a bin's M values sorted ascending, s_0 <= ... <= s_{M-1}:
 *   HK_RULE_STEP:   s_r, r = ceil(g M) - 1, the smallest rank whose
 *                   cumulative coordinate g_r = (r+1)/M reaches g (§2.2);
 *   HK_RULE_LINEAR: s_i placed at y_i = (i + 1/2)/M (the abscissae of the
 *                   Chebyshev fit, §2.6), straight lines between neighbours,
 *                   s_0 below y_0 and s_{M-1} above y_{M-1}; with
 *                   u = g M - 1/2, i = floor(u), k = s_i + (u - i)(s_{i+1} - s_i),
 *                   evaluated in binary64 without contraction. */
#define HK_RULE_STEP 0
#define HK_RULE_LINEAR 1

/* Counts of line-point evaluations of the last hk_opacity call. */
typedef struct {
    int64_t evals;       /* sum over lines of |cutoff window ∩ grid| */
    int64_t evals_core;  /* a^2 + u^2 < 100: series (Algorithm 916 form) */
    int64_t evals_gh3;   /* 100 <= a^2 + u^2 < 1e6: 3-node Gauss-Hermite */
    int64_t evals_gh1;   /* a^2 + u^2 >= 1e6: 1-node Gauss-Hermite */
    int64_t n_lines;     /* lines in the context */
    int64_t evals_surrogate; /* of evals_core, the points the learned
                                surrogate evaluated (HK_F32_SURROGATE; the
                                rest took the series); 0 for other precisions
                                and after hk_tables */
} hk_run_stats;

/* ---- context ------------------------------------------------------------ */

int hk_version(void); /* major * 10000 + minor * 100 + patch */

/* Create a context on HIP device `device` with its own stream.  *out is set
 * to NULL on failure. */
int hk_create(int device, hk_ctx** out);
int hk_destroy(hk_ctx* ctx);

/* Use `hip_stream` (a hipStream_t, e.g. torch's current stream) for all
 * later work.  NULL is HIP's null (legacy default) stream, which is what
 * PyTorch reports for its default stream.  Until this is called the context
 * uses a non-blocking stream of its own. */
int hk_set_stream(hk_ctx* ctx, void* hip_stream);
int hk_sync(hk_ctx* ctx);

/* Message of the last failed call on ctx (ctx may be NULL: last failure on
 * this thread).  Never NULL; valid until the next call. */
const char* hk_last_error(const hk_ctx* ctx);

/* Copy a line list (§2.3: the database fields the method uses) into the
 * context, ordered by ascending (nu, input index) -- the order in which the
 * opacity kernels walk the lines (§2.5) -- replacing any earlier one.
 *   lines_on_device == 0: lines' arrays are [host] memory;
 *   lines_on_device != 0: they are [device] memory of the context's device
 *     (e.g. torch tensors), read but not modified.
 * Inputs are validated (finite values, nu > 0, S_ref, gamma, A21 >= 0; on
 * the host for host arrays, by a kernel for device arrays); HK_EINVAL names
 * the first offending line, and a rejected list leaves the context
 * unchanged.  A list not already in non-decreasing nu is ordered on the
 * device by a stable radix sort of nu's bit patterns (temporary device
 * memory of ~24 B per line, released on return; a host list is first copied
 * as it is).  Synchronous: the arrays may be freed or rewritten on return. */
int hk_load_lines(hk_ctx* ctx, const hk_lines* lines, const hk_species* species, int lines_on_device);

/* ---- Input (§2.3, §3.5): HITRAN / HITEMP line records -------------------- */

/* Writable line arrays of `capacity` values each (the reader's output);
 * every pointer is required. */
typedef struct {
    int64_t capacity;
    double *nu, *S_ref, *E_lower, *gamma_air, *n_air, *gamma_self, *delta, *A21;
} hk_lines_out;

/* Read line records in the HITRAN fixed-width format (Rothman et al. 2005
 * layout, the one HITRAN and HITEMP files share: 160 characters per record,
 * each ended by LF or CR LF) from the file at `path`, starting at record
 * `first` (0-based), into out's arrays.  The fields read, by 1-based
 * column: molecule number 1-2, line centre nu 4-15, S_ref (at 296 K) 16-25,
 * Einstein A 26-35, gamma_air 36-40, gamma_self 41-45, E'' 46-55, n_air
 * 56-59, pressure shift delta 60-67; the rest of the record is not read.
 * molecule > 0 keeps only records of that molecule number; 0 keeps all.
 * Reading stops at the end of the file or when out->capacity records are
 * stored.  *n_read: records stored; *next: the index of the first record
 * not consumed (records skipped by the molecule filter are consumed), so a
 * list is read in chunks by calling again with first = *next until
 * *n_read == 0.  HK_EINVAL for a file that is not in this format (record
 * length, line ends), a truncated last record or an unparsable field,
 * naming the record and the field.  Host only: no device is used. */
int hk_read_par(const char* path, int64_t first, int32_t molecule, const hk_lines_out* out,
                int64_t* n_read, int64_t* next);

/* ---- §2.3-§2.5: opacity function ---------------------------------------- */

/* Opacity kappa(nu_j) on the grid for one state.  For every line: S(T) by
 * eq. (18), Gamma_D and the Voigt parameters by eq. (19), Gamma_L by
 * eq. (20), centre shifted by eq. (21); then kappa_j = sum of S Phi(nu_j)
 * (eq. (16)) over the lines whose cutoff window contains j.  The window is
 * the closed index interval [ceil((nu0' - cutoff - nu_min)/dnu),
 * floor((nu0' + cutoff - nu_min)/dnu)].  H_V(a,u) uses the series form of
 * the Faddeeva function for a^2+u^2 < 100 and 3-node / 1-node Gauss-Hermite
 * quadrature for a^2+u^2 < 1e6 / >= 1e6 (§2.4).  Each point sums its
 * Gauss-Hermite terms, then its series terms, each in ascending (nu, input
 * index) order, with no atomics; where the lines crowd into few grid tiles
 * (a wavenumber-ordered piece of a list, a dense band) the Gauss-Hermite sum
 * is split at fixed line-index segments whose ordered sums are then added in
 * segment order.  Results are bitwise reproducible, do not depend on the
 * tuning options, and agree bit for bit with hk_tables.
 *
 * kappa is [device] double[n_points] for both precisions.  comp must be
 * NULL: it is reserved for a caller-held binary32 compensation term, which
 * this library does not need -- the binary32 path keeps its Kahan pair
 * (sum, compensation) in the context's scratch and folds it into kappa in
 * binary64 at the end of the call, so kappa carries the compensated sum to
 * binary64 rounding, and accumulate adds each call's result to kappa in
 * binary64 (chunks of a list, species of a mixture).
 * precision HK_F64: every step in binary64.
 * precision HK_F32_KAHAN: S(T), widths, windows and region intervals in
 *   binary64; profiles in binary32 with strengths scaled by a per-state power
 *   of two; each point's Gauss-Hermite terms summed in binary32 blocks of at
 *   most 256 lines whose sums are added with Kahan compensation, its series
 *   terms summed in binary32 and then Kahan-added; the compensated sum is
 *   scaled back and stored in binary64.  Requires cutoff/dnu < 2^23 (for a
 *   Lorentz-width cutoff: cutoff_lorentz * max Gamma_L / dnu < 2^23).
 * precision HK_F32_SURROGATE: as HK_F32_KAHAN, except that series-region
 *   points (a^2+u^2 < 100) whose (u, a) cell the last hk_surrogate_certify
 *   call certified take the learned surrogate instead of the series;
 *   HK_ENOTREADY without a certification.
 * accumulate != 0 adds to the values already in kappa, e.g. to process a
 * line list in chunks; accumulate == 0 overwrites them.  The series terms
 * are computed on a second non-blocking stream of the context, concurrently
 * with the Gauss-Hermite terms, into a grid of their own that is then added
 * on ctx's stream (fork and join by events, so the call stays ordered on
 * ctx's stream; hk_tables does the same per batch).  Asynchronous, except
 * on grids above ~2e7 points, where each stage's work plan is read back once
 * (two stream synchronisations) to size its scratch. */
int hk_opacity(hk_ctx* ctx, const hk_state* state, const hk_grid* grid,
               int precision, void* kappa, void* comp, int accumulate);

#define HK_MAX_CHUNKS 65536

/* The opacity of a line list given in chunks (§3.5: a list shipped as many
 * files whose opacities are added), with the host work, the copy to the
 * device and the preparation of chunk c+1 overlapping the kernels of chunk
 * c (whose updates of kappa stay in chunk order).  The result is
 * bitwise that of calling, for c = 0 .. n_chunks-1, hk_load_lines(&chunks[c],
 * species) and then hk_opacity(state, grid, precision, kappa, NULL,
 * accumulate || c > 0); only two chunks are on the device at a time, each
 * with its own set of the context's per-list buffers (records, tile
 * ranges, work plans, sums: about 300 MB per set at 3e6 points).
 *   chunks: [host] n_chunks (0 .. HK_MAX_CHUNKS) line lists, each under the
 *     rules of hk_load_lines.  All are checked before any work is enqueued
 *     (HK_EINVAL names the chunk); chunks in non-decreasing nu are copied
 *     as they are, others are ordered first.
 *   kappa: [device] double[n_points], as in hk_opacity; with n_chunks == 0
 *     it is zeroed (accumulate == 0) or left as it is.
 * The host arrays are copied into pinned staging buffers of the context
 * during the call and may be freed on return; the device work is
 * asynchronous, as for hk_opacity.  Copies, preparation and the updates of
 * kappa run on ctx's stream, the series and the wing kernels on two
 * non-blocking streams of the context, ordered by events; the call ends on
 * ctx's stream.
 * Afterwards the loaded list is the last chunk, and hk_stats counts the
 * whole stream. */
int hk_opacity_stream(hk_ctx* ctx, const hk_lines* chunks, int32_t n_chunks, const hk_species* species,
                      const hk_state* state, const hk_grid* grid, int precision, double* kappa,
                      int accumulate);

/* ---- §2.2, §2.6: k-distribution ------------------------------------------ */

/* For each bin of consecutive points: sort the opacities ascending, form the
 * cumulative coordinate g_i = (i+1)/M of the i-th smallest of the bin's M
 * values (eq. (14) with eq. (15)'s uniform step 1/N_nu), and resample
 * k(g_q) at the requested g values by bins->rule (the step rule
 * k(g_q) = kappa_sorted[ceil(g_q M) - 1], or the midpoint-linear rule;
 * see hk_bins).
 * kappa: [device] double (HK_F64) or float (HK_F32_KAHAN: binary32 keys)
 * [n_points], all values >= 0 (a NaN sorts last).  k_out: [device] double[n_bins][n_g] with
 * n_bins = ceil(n_points / points_per_bin).  sorted_out: NULL, or [device]
 * array of kappa's type [n_points] receiving each bin sorted in place order
 * (the k-distribution function kappa(y) of §2.1.1). */
int hk_kdist(hk_ctx* ctx, const void* kappa, int precision, int64_t n_points,
             const hk_bins* bins, double* k_out, void* sorted_out);

/* hk_kdist without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same arguments and results, bit for bit.  Bins
 * larger than one LDS sort (16384 keys on gfx950) are merged through a
 * fixed device array of HK_KDIST_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends, instead of the
 * context's scratch; such calls need n_points * (8 or 4 key bytes) * 2 <=
 * HK_KDIST_NOALLOC_SCRATCH_BYTES, else HK_EINVAL (nothing enqueued).  Every
 * call on one device shares that array, and nothing in it needs clearing
 * (each call overwrites what it reads); calls that overlap on one device --
 * on different streams or from different contexts -- race on it and must
 * be ordered by the caller.  No timing is recorded for these calls. */
#define HK_KDIST_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hk_kdist_noalloc(hk_ctx* ctx, const void* kappa, int precision, int64_t n_points, const hk_bins* bins,
                     double* k_out, void* sorted_out);

/* Opacity tables over many thermodynamic states (§2.5: the k-distribution
 * is repeated for every combination of temperature and pressure of the
 * table).  For each states[i] the result equals hk_opacity(states[i], grid,
 * precision) followed by hk_kdist of that opacity (binary64 keys), written to
 *   k_out   [device] double [n_states][n_bins][bins->n_g],
 *           n_bins = ceil(grid->n_points / bins->points_per_bin).
 * The states are processed in batches: one batch's line records are prepared
 * per state, then one wing launch and one series launch cover the work items
 * (grid tiles, or a tile's lines in one segment where lines crowd) of every
 * state of the batch, then the bins of each state are sorted.  The opacity
 * grids of a batch stay in device scratch owned by the context (about
 * n_lines * 96 B + n_points * 8 B per state in binary32, n_lines * 160 B +
 * n_points * 8 B in binary64, plus up to 6 n_points * 8 B of partial sums per
 * state whose tiles are split); the batch size is "tables_batch" states, or
 * (0, the default) as many as fit in "tables_mem_mib".  Each batch's work
 * plan is read back once to size its launches (one stream synchronisation
 * per batch).  On the first call for a (precision, line count, grid size,
 * cutoff/dnu) the wing tile shape is chosen by timing 2, 4 and 8 points per
 * lane on up to four states ("tables_autotune", synchronises the stream
 * once); the shapes give identical results.  precision: HK_F64 or
 * HK_F32_KAHAN (cutoff/dnu < 2^23).  Errors: HK_EINVAL (argument, with the
 * index of a bad state), HK_ENOTREADY (no line list), HK_ENOMEM/HK_EDEVICE.
 * hk_stats afterwards reports the evaluation counts summed over the states. */
int hk_tables(hk_ctx* ctx, const hk_state* states, int32_t n_states, const hk_grid* grid,
              const hk_bins* bins, int precision, double* k_out);

/* ---- §2.6, eq. (5): resampling and transmission ---------------------------- */

#define HK_MAX_COEF 32             /* most Chebyshev coefficients per bin */
#define HK_MAX_COLUMNS (1 << 20)   /* most column masses per call */
#define HK_TRANSMISSION_NODES 100  /* Gauss-Legendre nodes of hk_transmission */

/* Least-squares Chebyshev fit of ln kappa(y) per bin (§2.6), solved by the
 * QR decomposition of the design matrix A[i][c] = T_c(t_i),
 * t_i = 2 y_i - 1, y_i = (i + 1/2)/M for the i-th smallest of the bin's M
 * values (one thin Householder QR per bin size, computed on the host and
 * cached; per bin the kernel forms Q^T d and solves R C = Q^T d).
 *   sorted   [device] the bins sorted ascending, as hk_kdist's sorted_out
 *            (double for HK_F64, float for HK_F32_KAHAN keys)
 *   coef_out [device] double [n_bins][n_coef]
 * Values <= 0 are clamped to the smallest positive normal double before
 * the logarithm.  Every bin needs at least n_coef points (HK_EINVAL). */
int hk_resample(hk_ctx* ctx, const void* sorted, int precision, int64_t n_points,
                int64_t points_per_bin, int32_t n_coef, double* coef_out);

/* Transmission function T(m) = int_0^1 exp(-kappa(y) m) dy (eq. 5) from
 * the fitted coefficients, by the HK_TRANSMISSION_NODES-node
 * Gauss-Legendre rule on [0, 1]:
 *   coef  [device] double [n_bins][n_coef];  m_col [device] double [n_m]
 *   T_out [device] double [n_bins][n_m] */
int hk_transmission(hk_ctx* ctx, const double* coef, int64_t n_bins, int32_t n_coef,
                    const double* m_col, int32_t n_m, double* T_out);

/* The same from the sorted values themselves: T(m) = (1/M) sum_i
 * exp(-kappa_i m) per bin (the reference for the resampling error). */
int hk_transmission_direct(hk_ctx* ctx, const void* sorted, int precision, int64_t n_points,
                           int64_t points_per_bin, const double* m_col, int32_t n_m, double* T_out);

/* ---- learned surrogate of K(x, y) = H_V(a = y, u = x) ---------------------
 * Not part of the paper's method: a network that stands in for the series
 * (§2.4) where a certification against the series allows it; the series
 * stays the fallback.  Features f1 = x/25 - 1, f2 = (log10 y + 1)/3; four
 * hidden layers of 64 SiLU units (SiLU(z) = z/(1+e^-z)); one linear output
 * z_hat; K_hat = G3(x, y) exp(tau sinh(z_hat)), tau = 1e-5, G3 the 3-node
 * Gauss-Hermite value.  Parameters: one binary32 vector, row-major
 * W[out][in]: W1[64][2] b1[64] W2[64][64] b2[64] W3[64][64] b3[64]
 * W4[64][64] b4[64] w5[64] b5[1].  Weights are used as bfloat16 (round to
 * nearest even), as are the hidden activations and layer gradients entering
 * the 64-wide products (matrix cores, binary32 sums); biases and features
 * stay binary32.  Training minimises the mean squared error of z_hat against
 * z = asinh(ln(K/G3)/tau), optionally weighted against large |z| where the
 * surrogate cannot be certified anyway, with Adam (Kingma & Ba 2015); every step's
 * gradient is summed in a fixed order (no atomics).  x, y, z, K below are
 * [device] float arrays of n values (x >= 0 is used as |x|, y > 0). */
#define HK_SURR_N_PARAMS 12737
#define HK_SURR_MAX_BATCH 65536
#define HK_SURR_CELLS_X 80   /* certification cells: x in [0, 10) ... */
#define HK_SURR_CELLS_Y 40   /* ... times log10 y in [-4, 1), 0.125 wide */
typedef struct {
    int32_t batch;   /* samples per step, 1 .. HK_SURR_MAX_BATCH */
    int32_t steps;   /* Adam steps */
    double lr, beta1, beta2, eps;
    double wscale;   /* loss weight 1/(1 + (z/wscale)^2); 0: unweighted */
} hk_train_cfg;

/* Training targets z = asinh(ln(K/G3)/tau) with K from the plain method in
 * binary64 (series for x^2+y^2 < 100, 3-node rule below 1e6, 1-node rule
 * beyond, §2.4). */
int hk_surrogate_labels(hk_ctx* ctx, const float* x, const float* y, int64_t n, float* z);
/* [host] theta[HK_SURR_N_PARAMS]: set the parameters (copied; synchronises),
 * reset Adam's moments, step count and sample cursor, drop the
 * certification. */
int hk_surrogate_set_params(hk_ctx* ctx, const float* theta);
/* [host] theta[HK_SURR_N_PARAMS] <- the current parameters (synchronises). */
int hk_surrogate_get_params(hk_ctx* ctx, float* theta);
/* Loss over n (1 .. HK_SURR_MAX_BATCH) samples -- the mean of
 * w(z) (z_hat - z)^2, w(z) = 1/(1 + (z/wscale)^2) (w = 1 for wscale = 0) --
 * and its gradient: grad [device] float[HK_SURR_N_PARAMS], loss [device]
 * float[1] or NULL.  The parameters are not changed. */
int hk_surrogate_grad(hk_ctx* ctx, const float* x, const float* y, const float* z, int64_t n,
                      double wscale, float* grad, float* loss);
/* cfg->steps Adam steps on batches of cfg->batch consecutive samples of the
 * n given (cyclically, continuing where the previous call stopped);
 * loss_hist [device] float[steps] (the loss of each step's batch before its
 * update) or NULL.  Drops the certification. */
int hk_surrogate_train(hk_ctx* ctx, const float* x, const float* y, const float* z, int64_t n,
                       const hk_train_cfg* cfg, float* loss_hist);
/* z_hat and (K != NULL) K_hat at n points. */
int hk_surrogate_eval(hk_ctx* ctx, const float* x, const float* y, int64_t n, float* z, float* K);
/* Certification: for each cell (ix, iy) -- x in [ix, ix+1) * 0.125,
 * log10 y in -4 + [iy, iy+1) * 0.125 -- the largest relative error of K_hat
 * against the binary64 series over the cell's 16x16 lattice of points (edges
 * included); cells with error <= budget are certified for HK_F32_SURROGATE.
 * A dense-sampling check, not a proven bound between lattice points.
 * err: [host] double[HK_SURR_CELLS_Y][HK_SURR_CELLS_X] or NULL;
 * n_certified: [host] or NULL.  Synchronises. */
int hk_surrogate_certify(hk_ctx* ctx, double budget, double* err, int32_t* n_certified);

/* The trained surrogate as one self-contained byte string, to be kept and
 * loaded into another context (or process) without training again:
 * a 32-byte header ("HKSURR01", int32 parameter count, int32 cell count,
 * int32 certified flag, int32 0, binary64 budget), the binary32 parameters
 * (the layout above) and, when certified, the binary64 error of every cell
 * (cell (ix, iy) at iy * HK_SURR_CELLS_X + ix); little-endian.
 * hk_surrogate_save: with blob NULL only *size is set (the bytes needed);
 * else blob [host] of `capacity` bytes receives them (synchronises).
 * HK_ENOTREADY without parameters. */
int hk_surrogate_save(hk_ctx* ctx, void* blob, size_t capacity, size_t* size);
/* hk_surrogate_load: blob [host] of `size` bytes from hk_surrogate_save.
 * Sets the parameters as hk_surrogate_set_params does (Adam's state reset)
 * and, if the blob holds a certification, restores it with its budget, so
 * HK_F32_SURROGATE runs at once.  HK_EINVAL for a blob of another layout,
 * size or with non-finite values; the context is then unchanged. */
int hk_surrogate_load(hk_ctx* ctx, const void* blob, size_t size);

/* ---- helpers -------------------------------------------------------------- */

/* Gauss-Legendre nodes and weights mapped to (0, 1): [host] g[n], w[n],
 * nodes ascending, weights summing to 1.  n in 1 .. 256. */
int hk_gauss_legendre(int32_t n, double* g, double* w);

/* Tuning knobs (results do not depend on them; only speed and memory do):
 *   "f64_points_per_lane"  4 or 8 grid points per lane in the binary64
 *                          opacity kernel (default 4; its points form groups
 *                          of four that share one reciprocal).
 *   "f32_points_per_lane"  2, 4 or 8 for the binary32 kernel (default 4).
 *   "tables_batch"         states per hk_tables launch, 0 = automatic
 *                          (default).
 *   "tables_mem_mib"       device scratch budget of an automatic batch
 *                          (default 32768).
 *   "tables_autotune"      1 (default): hk_tables times the tile shapes;
 *                          0: it uses the *_points_per_lane setting and the
 *                          cached choices are dropped.
 *   "wing_edge_paths"      1 (default): the Gauss-Hermite kernels take a
 *                          wavefront's run that a line's window covers only
 *                          in part on that rule's own path with a window
 *                          mask, and runs that hold series points or both
 *                          rules' points on paths of their own; 0: all of
 *                          these on the general path (a check: both give
 *                          the same bits).
 *   "tables_overlap"       0 (default): hk_tables runs each batch's series
 *                          kernel, then its wing kernel, on the caller's
 *                          stream; 1: the series on a second stream of the
 *                          context while the wing runs (same bits).
 * Unknown names or values: HK_EINVAL. */
int hk_set_option(hk_ctx* ctx, const char* name, int64_t value);
/* Reads a knob into *value; also, read-only: "tables_points_per_lane", the
 * tile shape the last hk_tables call used (0 before any); "wing_items", the
 * work items of the last wing launch (one per grid tile and state unless
 * tiles were split into line segments); "wing_segment_lines", the segment
 * length of that launch's first state (0: not split).  The last two wait
 * for the stream. */
int hk_get_option(hk_ctx* ctx, const char* name, int64_t* value);

/* Evaluation counts of the last hk_opacity call, or summed over the states
 * of the last hk_tables call (synchronises the stream). */
int hk_stats(hk_ctx* ctx, hk_run_stats* out);

/* Per-stage device time, measured with HIP events recorded around each
 * stage's kernels on the stream they run on while timing is enabled, summed
 * over calls since the last reset.  The series stage runs on a second
 * stream, concurrently with the Gauss-Hermite stage, so the two overlap
 * (each includes the time it shares the device); the line-preparation stage
 * includes the tile ranges and work plans.  Stage indices: */
#define HK_STAGE_LINE_PREP 0  /* per-line S(T), widths, windows, tile ranges */
#define HK_STAGE_OPACITY 1    /* Gauss-Hermite (a^2+u^2 >= 100) evaluation kernel */
#define HK_STAGE_KDIST 2      /* per-bin sort and k(g) */
#define HK_STAGE_CORE 3       /* series (a^2+u^2 < 100) evaluation kernel */
#define HK_N_STAGES 4
typedef struct {
    double ms[HK_N_STAGES];     /* summed milliseconds */
    int64_t calls[HK_N_STAGES]; /* number of timed launches */
} hk_timing;
/* enable != 0 starts timing (and resets the sums); 0 stops it. */
int hk_set_timing(hk_ctx* ctx, int enable);
/* Synchronises the stream and returns the sums. */
int hk_get_timing(hk_ctx* ctx, hk_timing* out);

#ifdef __cplusplus
}
#endif
#endif /* HK_H */
