// hk_internal.h -- records, constants and launch declarations shared by the
// HIP kernels and the C-ABI host code of libhk.  Not installed; the public
// interface is include/hk.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

// Physical constants in CGS (SI 2019 exact values for c, k_B, h; CODATA 2018
// atomic mass unit).
constexpr double kC = 2.99792458e10;        // cm s^-1
constexpr double kKB = 1.380649e-16;        // erg K^-1
constexpr double kH = 6.62607015e-27;       // erg s
constexpr double kAMU = 1.66053906660e-24;  // g
constexpr double kC2 = kH * kC / kKB;       // second radiation constant, cm K
constexpr double kPi = 3.14159265358979323846;
constexpr double kInvPi = 0.31830988618379067154;
constexpr double kInvSqrtPi = 0.56418958354775628695;

// Region radii of the Voigt scheme on a^2 + u^2 (§2.4).
// A volatile object in LDS, named with its address space: a volatile access
// through a plain pointer into LDS compiles to a flat access (the generic
// path, with a wait on the vector memory counter), this one to an LDS access.
template <typename T>
using lds_volatile = volatile __attribute__((address_space(3))) T;

constexpr double kCoreR2 = 100.0;
constexpr double kGH1R2 = 1.0e6;

// Per-line record of the binary64 wing evaluation, one per line and state,
// in line order.  With alpha = Gamma_D / sqrt(ln 2) the Doppler 1/e width,
// G = Gamma_L, dv = nu_j - nu0 and q = dv^2:
//   1-node:  S Phi = Lg / (q + G2)                       (a Lorentzian)
//   3-node:  S Phi = Lg n / (D P),  D = q + G2,
//            P = q (q + B) + C,  n = q (q + Bn) + Cn,
// the 3-node Gauss-Hermite sum (weights 2/3, 1/6, 1/6 of the Lorentzians at
// nu0 and nu0 -+ sqrt(3/2) alpha) over one common denominator, expanded in
// q: with GH = G2 + 1.5 alpha^2, P = (q + GH)^2 - 6 alpha^2 q is the product
// of the two shifted Lorentzians' denominators and 3n = 2P + D (q + GH).
// Coefficients: B = 2 G2 - 3 alpha^2, C = GH^2, Bn = 2 G2 - 1.5 alpha^2,
// Cn = GH (2 GH + G2) / 3.  The record holds the denominator as one cubic,
// D P = ((q + M2) q + M1) q + M0 with M2 = G2 + B = 3 (G2 - alpha^2),
// M1 = C + G2 B = 3 G2^2 + 2.25 alpha^4 (no cancellation) and M0 = G2 C.
// Where a^2 + u^2 >= 100, q + G2 >= 100 alpha^2, so the negative parts of
// M2 and Bn never cancel q's terms.
// The grid-index intervals (closed; empty when lo > hi) sit in WingIdx: the
// cutoff window and the points whose a^2+u^2 lies below 1e6 and below 100.
struct alignas(16) WingRec {
    double nu0;  // pressure-shifted line centre
    double Lg;   // S(T) Gamma_L / pi
    double G2;   // Gamma_L^2
    double M2, M1, M0;  // the 3-node denominator's cubic
    double Bn, Cn;      // the 3-node numerator's quadratic
};
static_assert(sizeof(WingRec) == 64, "WingRec layout");
struct alignas(16) WingIdx {
    int32_t wlo, whi;
    int32_t g3lo, g3hi;
    int32_t clo, chi;
    int32_t flags;  // kGroupSafe
    int32_t jc;     // nearest grid index to the centre (binary32 path)
};
static_assert(sizeof(WingIdx) == 32, "WingIdx layout");
// Products of four denominators stay in binary64 range: alpha^2 >= 1e-22 and
// dv^2 + Gamma_L^2 <= 1e20 at every grid point (every physical line and
// grid) put each 3-node denominator m = D P within about 1e-60 .. 1e60 (D >=
// 100 alpha^2 outside the core region).  Otherwise points are not grouped.
constexpr int32_t kGroupSafe = 1;

// Per-line record of the core-region series, read only for lines whose
// a^2+u^2 < 100 interval meets a wavefront's points.
struct alignas(16) CoreRec {
    double invA;  // 1 / alpha
    double y;     // Gamma_L / alpha  (the paper's damping parameter a)
    double y2;    // y * y
    double ex;    // erfcx(y)
    double norm;  // S(T) / (alpha sqrt(pi))
    double T1;    // sum_{n>=1} e^{-n^2/4} / (n^2/4 + y^2)
    double pad0, pad1;
};
static_assert(sizeof(CoreRec) == 64, "CoreRec layout");

// Binary32 records of one line and state, derived from the binary64 ones
// (so both precisions share S(T), widths, windows and region intervals).
// Lengths are in units of lambda = alpha when the line has 3-node or core
// points (y^2 < 1e6), else lambda = Gamma_L, which keeps every denominator
// and product in binary32 range; strengths carry the state's scale 2^s.
// For point j: dv/lambda = (j - jc) du - fu, with jc the nearest grid point
// to the centre (WingIdx.jc), du = dnu/lambda, fu = (nu0 - nu_jc)/lambda.
//   1-node:  Lg / (q + G2),  3-node:  Lg n / m  with q = (dv/lambda)^2,
// m = ((q + M2) q + M1) q + M0 and n = q (q + Bn) + Cn, the coefficients of
// WingRec scaled by powers of 1/lambda.  A line with 3-node points has
// lambda = alpha, where Bn = 2 G2 - 1.5 exactly: it is formed in the kernel
// (lines with lambda = Gamma_L never use the 3-node rule).
struct alignas(16) WingRec32 {
    float du, fu, Lg, G2, M2, M1, M0, Cn;
};
static_assert(sizeof(WingRec32) == 32, "WingRec32 layout");
// Core series in x units: x = |(j - jc) dx - fx|, dx = dnu/alpha,
// fx = (nu0 - nu_jc)/alpha; norm = 2^s S/(alpha sqrt(pi)).
struct alignas(16) CoreRec32 {
    float dx, fx, y, y2, ex, norm, T1, pad;
};
static_assert(sizeof(CoreRec32) == 32, "CoreRec32 layout");

// Sorted line list on the device (structure of arrays, ascending nu).
struct LinesDev {
    const double* nu;
    const double* S_ref;
    const double* E_lower;
    const double* gamma_air;
    const double* n_air;
    const double* gamma_self;
    const double* delta;
    const double* A21;
    int64_t n;
};

// Per-workgroup result of the device-side check of a line list (the rules
// of hk_load_lines): the first line index that breaks a rule and the first
// whose nu is below its predecessor's (n if none), and the bounds of the
// valid lines that size the launches.
struct CheckPart {
    int64_t first_bad, first_unordered;
    double max_abs_delta, max_gamma_air, max_gamma_self, max_A21, min_n_air, max_n_air, nu_max;
};

// State-dependent constants of the line preparation, computed on the host.
struct PrepParams {
    double T, T_ref, P, P_self, q_ratio;
    double dop;       // alpha / nu = sqrt(2 k_B T / m) / c
    double nat;       // 1 / (4 pi c): natural width per unit A21
    double tscale;    // T / T_ref
    double nu_min, dnu, cutoff;
    double cutoff_lorentz;  // > 0: each line's cutoff is this many Gamma_L
    int32_t n_points;
};

// Rules that read k(g) off a sorted bin: step, midpoint-linear.
constexpr int32_t kRuleStep = 0;
constexpr int32_t kRuleLinear = 1;

struct GValues {
    double g[64];
    int32_t n;
    int32_t rule;  // kRuleStep or kRuleLinear
};

// ---- work items of the wing kernels (work_plan.hip) ----
// A tile's lines are summed by one workgroup, unless the lines crowd into
// few tiles or unevenly (a wavenumber-ordered piece of a list, a dense band):
// then every tile's line range is cut where it crosses a multiple of a
// segment length Lseg (a power of two, per state, from statistics of 512-point
// reference tiles, so the same for every tile shape), and each
// piece is an item of its own that writes partial sums; a reduction adds a
// cut tile's partials in segment order.  A point's value is then the ordered
// sum over segments of the ordered sum of its lines in each segment -- the
// same for every tile shape, since a tile is cut exactly where the lines
// reaching its points span segments (other segments add exact zeros).
// Items: every (state, tile) pair in chunks of kPlanChunk tiles (dearest
// first), each chunk holding every state's run of those tiles, a pair's
// segments consecutive; workgroups take items in XCD-dealt chunks.  16
// tiles of 1024 binary64 points keep the lines of the tiles an XCD runs at
// once closer to its 4 MB L2 than 32 (measured 4% faster; 8 is no better).
constexpr int32_t kRefTilePoints = 512;
constexpr int64_t kNoSplit = (int64_t)1 << 62;
constexpr int32_t kPlanChunk = 16;
struct WorkPlan {
    const int64_t* seg;    // [n_states] segment length (kNoSplit: not cut)
    const int64_t* first;  // [n_pairs] first item of each pair, in pair order
    const int64_t* slot;   // [n_pairs] first partial slot of each cut pair
    const int64_t* total;  // [2] items, partial slots
    int64_t n_pairs;
    int64_t launch_items;  // host: workgroups to launch (the item count, or its bound)
};
// Upper bounds, for sizing without reading the plan back: items <= 6 n_tiles
// + 2 per state (launches of n_pairs = n_tiles n_states pairs), partial
// points <= 6 n_points + 2 tile_points per state.
inline int64_t plan_items_bound(int64_t n_pairs, int32_t n_states) { return 6 * n_pairs + 2 * (int64_t)n_states; }
inline int64_t plan_partial_points_bound(int64_t n_points, int32_t tile_points)
{
    return 6 * n_points + 2 * (int64_t)tile_points;
}
int64_t plan_scratch_count(int64_t n_pairs);  // int64 values of the plan's block sums
// seg[s] from the reference ranges (tiles of kRefTilePoints points, 2 n_ref
// values per state) of n_states states; min_seg: the shortest segment, a
// power of two (256 for the binary32 wing, whose compensated sums run over
// 256-line blocks aligned to global line indices).
hipError_t launch_seg_length(const int64_t* ref_ranges, int64_t n_ref, int32_t n_states, int64_t n_points,
                             int64_t n_lines, int64_t min_seg, int64_t* seg, hipStream_t s);
// first, slot and total from the tile ranges (2 n_tiles per state) and seg.
hipError_t launch_work_plan(const int64_t* ranges, int64_t n_tiles, int32_t n_states, const int64_t* seg,
                            int64_t* first, int64_t* slot, int64_t* block_sums, int64_t* total, hipStream_t s);
// Workgroups for `items` items: padded to whole XCD chunks (xcd_rank is a
// bijection on each multiple of 8 kPlanChunk).
inline int64_t plan_blocks(int64_t items) { return (items + 8 * kPlanChunk - 1) / (8 * kPlanChunk) * (8 * kPlanChunk); }

// Rank of workgroup b: XCD b % 8 takes chunks of kPlanChunk consecutive
// ranks, so neighbouring tiles, which read mostly the same lines, share an
// L2 (a bijection on every multiple of 8 kPlanChunk).
__device__ inline int64_t xcd_rank(int64_t b)
{
    const int64_t x = b & 7, k = b >> 3;
    return ((k / kPlanChunk) * 8 + x) * kPlanChunk + (k % kPlanChunk);
}
// (state, tile rank) of pair p.
__device__ inline void pair_decode(int64_t p, int64_t n_tiles, int32_t n_states, int64_t& st, int64_t& k)
{
    const int64_t per_chunk = (int64_t)kPlanChunk * n_states;
    const int64_t c = p / per_chunk;
    const int64_t sz = min((int64_t)kPlanChunk, n_tiles - c * kPlanChunk);
    const int64_t rem = p - c * per_chunk;
    st = rem / sz;
    k = c * kPlanChunk + rem % sz;
}
struct WorkItem {
    int64_t st, tile;  // state, grid tile
    int64_t lo, hi;    // lines [lo, hi)
    int64_t slot;      // partial slot, or -1: the item writes the output
};
// Item r of the plan (false past the last item).  Every thread of a
// workgroup calls it with the same r.
__device__ inline bool work_item(int64_t r, const WorkPlan& wp, const int64_t* ranges, int64_t n_tiles,
                                 int32_t n_states, WorkItem& it)
{
    const int64_t total = wp.total[0];
    if (r >= total) return false;
    int64_t p = r;  // nothing cut: item r is pair r
    if (total != wp.n_pairs) {
        int64_t a = 0, b = wp.n_pairs;  // last pair whose first item <= r
        while (b - a > 1) {
            const int64_t m = a + ((b - a) >> 1);
            if (wp.first[m] <= r) a = m;
            else b = m;
        }
        p = a;
    }
    const int64_t nseg = (p + 1 < wp.n_pairs ? wp.first[p + 1] : total) - wp.first[p];
    int64_t k;
    pair_decode(p, n_tiles, n_states, it.st, k);
    it.tile = n_tiles - 1 - k;
    const int64_t* rg = ranges + it.st * 2 * n_tiles;
    it.lo = rg[2 * it.tile];
    it.hi = rg[2 * it.tile + 1];
    it.slot = -1;
    if (nseg > 1) {
        const int64_t L = wp.seg[it.st];
        const int64_t s = r - wp.first[p];
        const int64_t g = it.lo / L + s;
        it.lo = max(it.lo, g * L);
        it.hi = min(it.hi, (g + 1) * L);
        it.slot = wp.slot[p] + s;
    }
    return true;
}

// ---- launches (stream-ordered, no synchronisation) ----
hipError_t launch_line_prep_f64(const LinesDev& L, const PrepParams& pp, WingRec* wing,
                                WingIdx* idx, CoreRec* core, hipStream_t s);
// Every state of a batch in one launch: pps [device] n_states constants,
// records L.n apart per state.
hipError_t launch_line_prep_f64_batch(const LinesDev& L, const PrepParams* pps, int32_t n_states, WingRec* wing,
                                      WingIdx* idx, CoreRec* core, hipStream_t s);
// Tile line ranges for `reach`; or, with reach_of ([device] n_states values),
// the ranges of n_states states in one launch, 2 n_tiles apart.
hipError_t launch_tile_ranges(const double* nu_sorted, int64_t n_lines, int64_t n_tiles,
                              int32_t tile_points, double nu_min, double dnu, int32_t n_points,
                              double reach, int64_t* ranges, hipStream_t s, const double* reach_of = nullptr,
                              int32_t n_states = 1);
// Binary64 opacity: the wing kernel writes kappa (points_per_lane 2, 4 or
// 8), the core kernel then adds the series terms.
int32_t opacity_f64_tile_points(int points_per_lane);
int32_t core_f64_tile_points();
int32_t core_f32_tile_points();  // points per work item of the binary32 series
// The wing items of n_states states (records n_lines apart, ranges 2 n_tiles
// apart, kappa n_points apart); items cut by the plan write partial (binary64,
// tile_points per slot), which the reduction then adds into kappa.  With
// accumulate, kappa += the wing sum (single state).  One workgroup per item
// (wp.launch_items workgroups).
hipError_t launch_wing_f64(int points_per_lane, const WingRec* wing, const WingIdx* idx, const int64_t* ranges,
                           int64_t n_lines, int64_t n_tiles, int32_t n_states, const WorkPlan& wp, double nu_min,
                           double dnu, int32_t n_points, double* kappa, double* partial, int accumulate,
                           int edge_paths, hipStream_t s);
// The series items of n_states states (tiles of core_f64_tile_points(),
// their own plan): series = the series sums, every point written (a grid of
// its own, n_points per state, added to the wing's afterwards, so that the
// two kernels can run at the same time); cut items write partial.
hipError_t launch_core_f64(const WingRec* wing, const WingIdx* idx, const CoreRec* core, const int64_t* ranges,
                           int64_t n_lines, int64_t n_tiles, int32_t n_states, const WorkPlan& wp, double nu_min,
                           double dnu, int32_t n_points, double* series, double* partial, hipStream_t s);
// Zero `bytes` (a multiple of 4) at p with a kernel (unlike hipMemsetAsync,
// safe to record into a captured graph).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// a[j] += b[j], j < n.
hipError_t launch_add_f64(double* a, const double* b, int64_t n, hipStream_t s);
// n_blocks partial triples per state; n_states states (records n_lines
// apart, partials 3 n_blocks apart) in one launch.
hipError_t launch_eval_counts(const WingIdx* idx, int64_t n_lines, int64_t* partial,
                              int32_t n_blocks, hipStream_t s, int32_t n_states = 1);

// Binary32 path: the state's scale exponent from the lines' peak heights
// (two reductions into scale[0]), the record conversion, and the kernels.
// With n_states > 1, the states of a batch in one launch each (records
// n_lines apart, partial n_blocks apart, one scale per state).
hipError_t launch_f32_scale(const WingRec* wing, const CoreRec* core, int64_t n_lines,
                            double* partial, int32_t n_blocks, int32_t* scale, hipStream_t s,
                            int32_t n_states = 1);
// Binary32 tables straight from the line list, every state of a batch in
// one launch each (state blockIdx.y, constants pps[state]): the peak bound's
// per-block maxima (n_blocks per state) and the scale of each state; then
// the index records and the binary32 records (n_lines apart per state),
// equal to those of launch_line_prep_f64 + launch_f32_scale +
// launch_line_prep_f32.
hipError_t launch_f32_scale_lines(const LinesDev& L, const PrepParams* pps, double* partial, int32_t n_blocks,
                                  int32_t* scale, hipStream_t s, int32_t n_states);
hipError_t launch_line_prep_f32_direct(const LinesDev& L, const PrepParams* pps, int32_t n_states, double nu_min,
                                       double dnu, const int32_t* scale, WingIdx* idx, WingRec32* w32,
                                       CoreRec32* c32, hipStream_t s);
hipError_t launch_line_prep_f32(const WingRec* wing, WingIdx* idx, const CoreRec* core,
                                int64_t n_lines, double nu_min, double dnu, const int32_t* scale,
                                WingRec32* w32, CoreRec32* c32, hipStream_t s, int32_t n_states = 1);
int32_t opacity_f32_tile_points(int points_per_lane);
// As launch_wing_f64: the Kahan pairs (sum, comp) of n_states states; cut
// items write (sum, comp) pairs to partial (tile_points float2 per slot).
hipError_t launch_wing_f32(int points_per_lane, const WingRec32* wing, const WingIdx* idx, const int64_t* ranges,
                           int64_t n_lines, int64_t n_tiles, int32_t n_states, const WorkPlan& wp, int32_t n_points,
                           float* sum, float* comp, float2* partial, int edge_paths, hipStream_t s);
// The series items (tiles of opacity_f32_tile_points(4)): series = the
// binary32 series sums, every point written (added to the wing's Kahan pairs
// by launch_f32_finish); surrogate (the bfloat16 parameter copy, single
// state): the learned surrogate in the cells `mask` certifies.
hipError_t launch_core_f32(const WingIdx* idx, const CoreRec32* core, const int64_t* ranges, int64_t n_lines,
                           int64_t n_tiles, int32_t n_states, const WorkPlan& wp, int32_t n_points, float* series,
                           float* partial, const void* surrogate, const uint8_t* mask, int64_t* used,
                           int64_t used_cap, hipStream_t s);
// line_sort.hip: the (nu, index) order of a list on the device, and the
// check of a list in device memory.
size_t line_sort_scratch_bytes(int64_t n);
// perm_out: points into scratch, the input indices in (nu, index) order
hipError_t launch_line_order(const double* nu, int64_t n, void* scratch, const uint32_t** perm_out, hipStream_t s);
hipError_t launch_gather(const double* src, const uint32_t* perm, int64_t n, double* dst, hipStream_t s);
int32_t check_lines_blocks(int64_t n);  // CheckPart results launch_check_lines writes
hipError_t launch_check_lines(const LinesDev& L, void* part, hipStream_t s);

// total[0] = (add ? total[0] : 0) + used[0] + ... + used[n-1]
hipError_t launch_sum_counts(const int64_t* used, int64_t n, int64_t* total, int add, hipStream_t s);


// kappa (binary64) = (the Kahan pair (sum, comp) with the series sum, when
// not zero, Kahan-added) * 2^-s, or += when accumulating; series may be NULL.
// n_states grids of n_points each (one scale per state) in one launch.
hipError_t launch_f32_finish(const float* sum, const float* comp, const float* series, const int32_t* scale,
                             int32_t n_points, double* kappa, int accumulate, hipStream_t s,
                             int32_t n_states = 1);

// k-distribution.  elem_bytes 8 (binary64 keys) or 4 (binary32 keys).
int64_t kdist_lds_max_points(int elem_bytes, int64_t lds_bytes);
// LDS per sort workgroup: 32 KB (4096 binary64 or 8192 binary32 keys);
// larger bins are sorted in chunks of that size and merged.  Measured: 300
// bins of 1e4 binary64 keys take 0.18 ms in 32 KB chunks, 0.19 in 16 KB,
// 0.22 in 64 KB and 0.30 ms in one 128 KB sort each (more, smaller sorts
// share the CUs; the merges are cheap).
constexpr int64_t kSortLdsBytes = 32768;
// Bins of up to kdist_radix_max_keys(lds_max) keys (16384 on gfx950's
// 160 KB of LDS per workgroup) are sorted by an LDS radix sort, one
// workgroup per bin, the bins of n_states contiguous grids (each n_points)
// in one launch; larger bins (one grid per call) by the chunks below.
int64_t kdist_radix_max_keys(int elem_bytes, int64_t lds_max);
hipError_t launch_kdist(const void* kappa, int elem_bytes, int64_t n_points, int64_t ppb,
                        const GValues& g, double* k_out, void* sorted_out, void* scratch,
                        int64_t lds_bytes, int64_t lds_max, int32_t n_states, hipStream_t s);
size_t kdist_scratch_bytes(int elem_bytes, int64_t n_points, int64_t ppb, int64_t lds_bytes, int64_t lds_max);
// The fixed device array of hk_kdist_noalloc (HK_KDIST_NOALLOC_SCRATCH_BYTES),
// its address on the current device (call with that device current).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
hipError_t noalloc_scratch_address(void** ptr);

// Learned K(x, y) surrogate (surrogate.hip): sizes, labels, the compute
// copy of the parameters, one training step and its Adam update, a plain
// gradient, evaluation and per-cell certification errors.
size_t surrogate_params_bytes();
int32_t surrogate_n_params();
int32_t surrogate_cells();
hipError_t launch_surrogate_labels(const float* x, const float* y, int64_t n, float* z, hipStream_t s);
hipError_t launch_surrogate_pack(const float* theta, void* P, hipStream_t s);
hipError_t launch_surrogate_train_step(const void* P, const float* x, const float* y, const float* z, int64_t n,
                                       int64_t base, int32_t batch, float wscale, float* part_grad,
                                       float* part_loss, hipStream_t s);
hipError_t launch_surrogate_adam(float* theta, float* m, float* v, const float* part_grad, int32_t batch,
                                 float lr, float beta1, float beta2, float eps, float c1, float c2, void* P,
                                 const float* part_loss, float* loss_out, hipStream_t s);
hipError_t launch_surrogate_reduce(const float* part_grad, int32_t batch, float* grad, const float* part_loss,
                                   float* loss_out, hipStream_t s);
hipError_t launch_surrogate_eval(const void* P, const float* x, const float* y, int64_t n, float* z, float* K,
                                 hipStream_t s);
hipError_t launch_surrogate_certify(const void* P, double* err, hipStream_t s);

// Resampling and transmission (resample.hip).
constexpr int kMaxCoef = 32;   // Chebyshev coefficients per bin
constexpr int kMaxQuad = 128;  // quadrature nodes of the fitted transmission
hipError_t launch_resample(const void* sorted, int key_bytes, int64_t n_points, int64_t ppb, int nc,
                           const double* Q, const double* R, const double* Ql, const double* Rl, double* coef,
                           hipStream_t s);
hipError_t launch_transmission_fit(const double* coef, int64_t n_bins, int nc, const double* yq, const double* wq,
                                   int nq, const double* m, int n_m, double* T, hipStream_t s);
hipError_t launch_transmission_direct(const void* sorted, int key_bytes, int64_t n_points, int64_t ppb,
                                      const double* m, int n_m, double* T, hipStream_t s);

// Sets the message hk_last_error(NULL) returns on this thread (host code
// outside hk_api.cpp that fails without a context).
void set_thread_error(const char* msg);

}  // namespace hk
