// line_prep.hip -- the per-line stage ("Line" in the paper's Fig. 5):
// temperature/pressure scaling of every line (§2.3) into the records the
// opacity kernels read, the line range of each grid tile, and the
// evaluation counts by region.
#include <algorithm>

#include "hk_internal.h"

#include <climits>

namespace hk {
namespace {

// e^{-k^2/4}, k = 1 .. 16: the weights of the series' line constant T1
// (needed for lines with series points, y < 10).  Later terms change no bit
// of the sum: each is below e^{-72.25} / 72.25 < 4e-34, and the sum is at
// least its first term, e^{-1/4} / (1/4 + y^2) > 7.7e-3.
__constant__ double kGaussT1[16] = {
    0.77880078307140488,
    0.36787944117144233,
    0.10539922456186433,
    0.018315638888734179,
    0.0019304541362277093,
    0.00012340980408667956,
    4.7851173921290088e-06,
    1.1253517471925912e-07,
    1.6052280551856116e-09,
    1.3887943864964021e-11,
    7.2877240958196922e-14,
    2.3195228302435696e-16,
    4.4777324417183015e-19,
    5.2428856633634639e-22,
    3.7233631217505106e-25,
    1.6038108905486379e-28,
};

// a^2 + u^2 at grid point j for a line (u = (nu_j - nu0) / alpha, a = y).
__device__ inline double r2_at(int64_t j, double nu_min, double dnu, double nu0, double invA,
                               double y2)
{
    double nuj = fma((double)j, dnu, nu_min);
    double x = fabs(nuj - nu0) * invA;
    return fma(x, x, y2);
}

// Closed interval [lo, hi] of grid indices with a^2+u^2 < R, clipped to the
// sentinels -1 and n (so "j < lo" / "j > hi" tests stay exact for every grid
// point).  a^2+u^2 computed as in r2_at is monotone in |nu_j - nu0| (every
// rounding step is monotone), so the set is an interval; the analytic
// half-width gives a start within a point or two, and the bounded searches
// settle the exact edges.  Empty: lo = INT_MAX, hi = INT_MIN.
__device__ void region_interval(double R, double nu_min, double dnu, int32_t n, double nu0,
                                double invA, double y2, int32_t* lo_out, int32_t* hi_out)
{
    if (!(y2 < R)) {
        *lo_out = INT_MAX;
        *hi_out = INT_MIN;
        return;
    }
    double half = sqrt(R - y2) / invA;  // cm^-1
    double c = (nu0 - nu_min) / dnu;
    double fhi = floor(c + half / dnu), flo = ceil(c - half / dnu);
    fhi = fmin(fmax(fhi, -1.0), (double)n);
    flo = fmin(fmax(flo, -1.0), (double)n);
    int64_t hi = (int64_t)fhi, lo = (int64_t)flo;
    for (int it = 0; it < 64 && hi < n && r2_at(hi + 1, nu_min, dnu, nu0, invA, y2) < R; ++it) ++hi;
    for (int it = 0; it < 64 && hi >= 0 && r2_at(hi, nu_min, dnu, nu0, invA, y2) >= R; ++it) --hi;
    for (int it = 0; it < 64 && lo > -1 && r2_at(lo - 1, nu_min, dnu, nu0, invA, y2) < R; ++it) --lo;
    for (int it = 0; it < 64 && lo < n && r2_at(lo, nu_min, dnu, nu0, invA, y2) >= R; ++it) ++lo;
    if (lo > hi) {
        *lo_out = INT_MAX;
        *hi_out = INT_MIN;
        return;
    }
    *lo_out = (int32_t)lo;
    *hi_out = (int32_t)hi;
}

// Line i scaled to one state (constants pp): strength, widths, centre.
struct LineScaled {
    double S, alpha, GL, nu0;
};
__device__ __forceinline__ LineScaled line_scaled(const LinesDev& L, const PrepParams& pp, int64_t i)
{
    const double nu = L.nu[i];
    const double E = L.E_lower[i];
    const double g_air = L.gamma_air[i];
    const double g_self = L.gamma_self ? L.gamma_self[i] : g_air;
    const double delta = L.delta ? L.delta[i] : 0.0;
    const double A21 = L.A21 ? L.A21[i] : 0.0;

    LineScaled r;
    // eq. (18), with E'' for Delta E and 1 - exp(-z) = -expm1(-z)
    const double boltz = exp(-kC2 * E / pp.T + kC2 * E / pp.T_ref);
    const double stim = expm1(-kC2 * nu / pp.T) / expm1(-kC2 * nu / pp.T_ref);
    r.S = L.S_ref[i] * pp.q_ratio * boltz * stim;
    // eq. (19): alpha = Gamma_D / sqrt(ln 2) = nu sqrt(2 k_B T / m) / c
    r.alpha = nu * pp.dop;
    // eq. (20), P0 = 1 atm
    r.GL = A21 * pp.nat + pow(pp.tscale, -L.n_air[i]) * (g_air * (pp.P - pp.P_self) + g_self * pp.P_self);
    // eq. (21); kept free of contraction so the window bounds below are the
    // exact binary64 expressions of the definition
    r.nu0 = __dadd_rn(nu, __dmul_rn(delta, pp.P));
    return r;
}

// S Phi bounded above by the smaller of the Doppler and the Lorentz peak
// heights, S / (alpha sqrt(pi)) and S / (pi Gamma_L): the same products
// as the records' norm and Lg / G2.
__device__ __forceinline__ double line_peak(const LineScaled& ls)
{
    const double doppler = ls.S * (1.0 / ls.alpha) * kInvSqrtPi;
    const double G2 = ls.GL * ls.GL;
    const double lorentz = G2 > 0.0 ? (ls.S * ls.GL * kInvPi) / G2 : doppler;
    return fmin(doppler, lorentz);
}

// The records of line i for one state (constants pp), in registers.
__device__ __forceinline__ void line_prep_vals(const LinesDev& L, const PrepParams& pp, int64_t i, WingRec& w,
                                               WingIdx& x, CoreRec& c)
{
    const LineScaled ls = line_scaled(L, pp, i);
    const double S = ls.S, alpha = ls.alpha, GL = ls.GL, nu0 = ls.nu0;
    w.nu0 = nu0;
    w.Lg = S * GL * kInvPi;
    w.G2 = GL * GL;
    {
        const double a2 = alpha * alpha;
        const double GH = w.G2 + 1.5 * a2;
        w.M2 = 3.0 * (w.G2 - a2);
        w.M1 = 3.0 * (w.G2 * w.G2) + 2.25 * (a2 * a2);
        w.M0 = w.G2 * (GH * GH);
        w.Bn = 2.0 * w.G2 - 1.5 * a2;
        w.Cn = GH * (2.0 * GH + w.G2) * (1.0 / 3.0);
        x.jc = 0;
    }
    const int32_t n = pp.n_points;
    {
        const double span = fmax(fabs(nu0 - pp.nu_min), fabs(fma((double)(n - 1), pp.dnu, pp.nu_min) - nu0));
        x.flags = (alpha * alpha >= 1e-22 && fma(span, span, w.G2) <= 1e20) ? kGroupSafe : 0;
    }
    {
        // the cutoff: absolute, or a multiple of the line's Lorentz HWHM
        const double cut = pp.cutoff_lorentz > 0.0 ? pp.cutoff_lorentz * GL : pp.cutoff;
        double flo = ceil((nu0 - cut - pp.nu_min) / pp.dnu);
        double fhi = floor((nu0 + cut - pp.nu_min) / pp.dnu);
        flo = fmax(flo, 0.0);
        fhi = fmin(fhi, (double)(n - 1));
        if (!(flo <= fhi)) {
            x.wlo = 1;
            x.whi = 0;
        } else {
            x.wlo = (int32_t)flo;
            x.whi = (int32_t)fhi;
        }
    }
    const double invA = 1.0 / alpha;
    const double y = GL * invA;
    const double y2 = y * y;
    region_interval(kGH1R2, pp.nu_min, pp.dnu, n, nu0, invA, y2, &x.g3lo, &x.g3hi);
    region_interval(kCoreR2, pp.nu_min, pp.dnu, n, nu0, invA, y2, &x.clo, &x.chi);

    c.invA = invA;
    c.y = y;
    c.y2 = y2;
    c.norm = S * invA * kInvSqrtPi;
    if (x.clo <= x.chi) {
        c.ex = erfcx(y);
        double t1 = 0.0;
        for (int k = 1; k <= 16; ++k) {
            double hk2 = 0.25 * (double)(k * k);
            t1 += kGaussT1[k - 1] / (hk2 + y2);
        }
        c.T1 = t1;
    } else {
        c.ex = 0.0;
        c.T1 = 0.0;
    }
    c.pad0 = 0.0;
    c.pad1 = 0.0;
}

// The records of line i for one state, to memory.
__device__ __forceinline__ void line_prep_one(const LinesDev& L, const PrepParams& pp, int64_t i,
                                              WingRec* __restrict__ wing, WingIdx* __restrict__ idx,
                                              CoreRec* __restrict__ core)
{
    WingRec w;
    WingIdx x;
    CoreRec c;
    line_prep_vals(L, pp, i, w, x, c);
    wing[i] = w;
    idx[i] = x;
    core[i] = c;
}

__global__ __launch_bounds__(256) void line_prep_f64_kernel(LinesDev L, PrepParams pp,
                                                            WingRec* __restrict__ wing,
                                                            WingIdx* __restrict__ idx,
                                                            CoreRec* __restrict__ core)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < L.n) line_prep_one(L, pp, i, wing, idx, core);
}

// Every state of a batch in one launch: state blockIdx.y, constants pps[st],
// records n_lines apart per state.
__global__ __launch_bounds__(256) void line_prep_f64_batch_kernel(LinesDev L, const PrepParams* __restrict__ pps,
                                                                  WingRec* __restrict__ wing,
                                                                  WingIdx* __restrict__ idx,
                                                                  CoreRec* __restrict__ core)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t o = (int64_t)blockIdx.y * L.n;
    if (i < L.n) line_prep_one(L, pps[blockIdx.y], i, wing + o, idx + o, core + o);
}

// Line index range [first, last) of every grid tile: the lines whose
// unshifted centre lies within `reach` of the tile's points.  Each line in
// the range is still tested against its exact window by the opacity kernel.
// reach_of: NULL, or one reach per state (state blockIdx.y, ranges
// 2 n_tiles apart per state).
__global__ __launch_bounds__(256) void tile_ranges_kernel(const double* __restrict__ nu, int64_t n,
                                                          int64_t n_tiles, int32_t tile_points,
                                                          double nu_min, double dnu,
                                                          int32_t n_points, double reach,
                                                          const double* __restrict__ reach_of,
                                                          int64_t* __restrict__ ranges)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    if (reach_of) {
        reach = reach_of[blockIdx.y];
        ranges += (int64_t)blockIdx.y * 2 * n_tiles;
    }
    int64_t j0 = t * tile_points;
    int64_t j1 = j0 + tile_points;
    if (j1 > n_points) j1 = n_points;
    double lo_nu = fma((double)j0, dnu, nu_min) - reach;
    double hi_nu = fma((double)(j1 - 1), dnu, nu_min) + reach;
    int64_t a = 0, b = n;  // first nu >= lo_nu
    while (a < b) {
        int64_t m = a + ((b - a) >> 1);
        if (nu[m] < lo_nu) a = m + 1;
        else b = m;
    }
    int64_t first = a;
    b = n;  // first nu > hi_nu
    while (a < b) {
        int64_t m = a + ((b - a) >> 1);
        if (nu[m] <= hi_nu) a = m + 1;
        else b = m;
    }
    ranges[2 * t] = first;
    ranges[2 * t + 1] = a;
}

__device__ inline int64_t overlap(int64_t alo, int64_t ahi, int64_t blo, int64_t bhi)
{
    int64_t lo = alo > blo ? alo : blo;
    int64_t hi = ahi < bhi ? ahi : bhi;
    return hi >= lo ? hi - lo + 1 : 0;
}

// Per-block partial sums of (evals, core, below 1e6) over lines.
__global__ __launch_bounds__(256) void eval_counts_kernel(const WingIdx* __restrict__ idx,
                                                          int64_t n, int64_t* __restrict__ partial)
{
    // state blockIdx.y of a batch: records n apart, partials 3 gridDim.x apart
    idx += (int64_t)blockIdx.y * n;
    partial += (int64_t)blockIdx.y * 3 * gridDim.x;
    __shared__ int64_t red[3][256];
    int64_t e = 0, c = 0, g = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const WingIdx w = idx[i];
        if (w.wlo > w.whi) continue;
        e += w.whi - w.wlo + 1;
        c += overlap(w.wlo, w.whi, w.clo, w.chi);
        g += overlap(w.wlo, w.whi, w.g3lo, w.g3hi);
    }
    red[0][threadIdx.x] = e;
    red[1][threadIdx.x] = c;
    red[2][threadIdx.x] = g;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) partial[3 * blockIdx.x + k] = red[k][0];
    }
}

// Peak height of a line's profile times S: S min(1/(alpha sqrt(pi)),
// 1/(pi Gamma_L)) bounds S Phi everywhere; per-block maxima.
__global__ __launch_bounds__(256) void f32_peak_kernel(const WingRec* __restrict__ wing,
                                                       const CoreRec* __restrict__ core, int64_t n,
                                                       double* __restrict__ partial)
{
    __shared__ double red[256];
    // state blockIdx.y of a batch: records n apart, partials gridDim.x apart
    wing += (int64_t)blockIdx.y * n;
    core += (int64_t)blockIdx.y * n;
    partial += (int64_t)blockIdx.y * gridDim.x;
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double doppler = core[i].norm;                     // S / (alpha sqrt(pi))
        const double lorentz = wing[i].G2 > 0.0 ? wing[i].Lg / wing[i].G2 : doppler;  // S/(pi G)
        m = fmax(m, fmin(doppler, lorentz));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// s = 100 - exponent(max peak): peaks land at or below 2^101, so sums of up
// to 2^26 of them stay below binary32's 2^128.
__global__ void f32_scale_kernel(const double* __restrict__ partial, int32_t n_blocks,
                                 int32_t* __restrict__ scale)
{
    if (threadIdx.x != 0) return;
    partial += (int64_t)blockIdx.x * n_blocks;  // state blockIdx.x of a batch
    scale += blockIdx.x;
    double m = 0.0;
    for (int32_t b = 0; b < n_blocks; ++b) m = fmax(m, partial[b]);
    scale[0] = m > 0.0 ? 100 - ilogb(m) : 0;
}

// The binary32 records of one line from its binary64 ones (scale s: peaks
// times 2^s), and its nearest grid point jc.
__device__ __forceinline__ void to_f32(const WingRec& w, const CoreRec& c, double nu_min, double dnu, int s,
                                       WingRec32& r, CoreRec32& k, int32_t& jc_out)
{
    const double alpha = 1.0 / c.invA;
    const double G = sqrt(w.G2);
    const bool use_alpha = c.y2 < kGH1R2;  // the line has 3-node or core points
    const double lam = use_alpha ? alpha : (G > 0.0 ? G : alpha);
    const double il = 1.0 / lam;
    // nearest grid point to the centre, clamped to int32 range
    double fjc = rint((w.nu0 - nu_min) / dnu);
    fjc = fmin(fmax(fjc, -1.0e9), 1.0e9);
    const int32_t jc = (int32_t)fjc;
    const double f = w.nu0 - fma((double)jc, dnu, nu_min);  // |f| <~ dnu/2
    r.du = (float)(dnu * il);
    r.fu = (float)(f * il);
    r.Lg = (float)ldexp(w.Lg * il * il, s);
    r.G2 = (float)(w.G2 * il * il);
    const double il2 = il * il;
    r.M2 = (float)(w.M2 * il2);
    r.M1 = (float)(w.M1 * il2 * il2);
    r.M0 = (float)(w.M0 * il2 * il2 * il2);
    r.Cn = (float)(w.Cn * il2 * il2);
    jc_out = jc;
    k.dx = (float)(dnu * c.invA);
    k.fx = (float)(f * c.invA);
    k.y = (float)c.y;
    k.y2 = (float)c.y2;
    k.ex = (float)c.ex;
    k.norm = (float)ldexp(c.norm, s);
    k.T1 = (float)c.T1;
    k.pad = 0.0f;
}

__global__ __launch_bounds__(256) void line_prep_f32_kernel(
    const WingRec* __restrict__ wing, WingIdx* __restrict__ idx, const CoreRec* __restrict__ core,
    int64_t n, double nu_min, double dnu, const int32_t* __restrict__ scale,
    WingRec32* __restrict__ w32, CoreRec32* __restrict__ c32)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    {  // state blockIdx.y of a batch: records n apart
        const int64_t o = (int64_t)blockIdx.y * n;
        wing += o;
        idx += o;
        core += o;
        w32 += o;
        c32 += o;
        scale += blockIdx.y;
    }
    WingRec32 r;
    CoreRec32 k;
    to_f32(wing[i], core[i], nu_min, dnu, scale[0], r, k, idx[i].jc);
    w32[i] = r;
    c32[i] = k;
}

// Line prep straight to the binary32 records: the binary64 records of line
// i for state blockIdx.y (constants pps[blockIdx.y]) in registers, the
// index record with its centre to idx, the binary32 records to w32 and c32
// (records n_lines apart per state).  The same values as the binary64 prep
// followed by line_prep_f32_kernel.
__global__ __launch_bounds__(256) void line_prep_f32_direct_kernel(LinesDev L, const PrepParams* __restrict__ pps,
                                                                   double nu_min, double dnu,
                                                                   const int32_t* __restrict__ scale,
                                                                   WingIdx* __restrict__ idx,
                                                                   WingRec32* __restrict__ w32,
                                                                   CoreRec32* __restrict__ c32)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.n) return;
    const int64_t o = (int64_t)blockIdx.y * L.n;
    WingRec w;
    WingIdx x;
    CoreRec c;
    line_prep_vals(L, pps[blockIdx.y], i, w, x, c);
    WingRec32 r;
    CoreRec32 k;
    to_f32(w, c, nu_min, dnu, scale[blockIdx.y], r, k, x.jc);
    idx[o + i] = x;
    w32[o + i] = r;
    c32[o + i] = k;
}

// Per-block maxima of the peak bound over the lines of state blockIdx.y,
// from the line list (the values f32_peak_kernel takes from the records).
__global__ __launch_bounds__(256) void f32_peak_lines_kernel(LinesDev L, const PrepParams* __restrict__ pps,
                                                             double* __restrict__ partial)
{
    __shared__ double red[256];
    const PrepParams& pp = pps[blockIdx.y];
    partial += (int64_t)blockIdx.y * gridDim.x;
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, line_peak(line_scaled(L, pp, i)));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}



// The wing's Kahan pair (sum, comp) of each point; the series sum, when not
// zero, Kahan-added to it (value = s - c, c the running correction); then
// scaled back into binary64.
__global__ __launch_bounds__(256) void f32_finish_kernel(const float* __restrict__ sum,
                                                         const float* __restrict__ comp,
                                                         const float* __restrict__ series,
                                                         const int32_t* __restrict__ scale,
                                                         int32_t n, double* __restrict__ kappa,
                                                         int accumulate)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    {  // state blockIdx.y of a batch: grids n apart
        const int64_t o = (int64_t)blockIdx.y * n;
        sum += o;
        comp += o;
        if (series) series += o;
        kappa += o;
        scale += blockIdx.y;
    }
    float s = sum[j], c = -comp[j];
    const float x = series ? series[j] : 0.0f;
    if (x != 0.0f) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    const double v = ldexp((double)s - (double)c, -scale[0]);
    kappa[j] = accumulate ? kappa[j] + v : v;
}

}  // namespace

hipError_t launch_f32_scale(const WingRec* wing, const CoreRec* core, int64_t n_lines,
                            double* partial, int32_t n_blocks, int32_t* scale, hipStream_t s, int32_t n_states)
{
    if (n_states <= 0) return hipSuccess;
    f32_peak_kernel<<<dim3(n_blocks, n_states), dim3(256), 0, s>>>(wing, core, n_lines, partial);
    f32_scale_kernel<<<dim3(n_states), dim3(64), 0, s>>>(partial, n_blocks, scale);
    return hipGetLastError();
}

hipError_t launch_f32_scale_lines(const LinesDev& L, const PrepParams* pps, double* partial, int32_t n_blocks,
                                  int32_t* scale, hipStream_t s, int32_t n_states)
{
    if (n_states <= 0) return hipSuccess;
    f32_peak_lines_kernel<<<dim3(n_blocks, n_states), dim3(256), 0, s>>>(L, pps, partial);
    f32_scale_kernel<<<dim3(n_states), dim3(64), 0, s>>>(partial, n_blocks, scale);
    return hipGetLastError();
}

hipError_t launch_line_prep_f32_direct(const LinesDev& L, const PrepParams* pps, int32_t n_states, double nu_min,
                                       double dnu, const int32_t* scale, WingIdx* idx, WingRec32* w32,
                                       CoreRec32* c32, hipStream_t s)
{
    if (L.n == 0 || n_states <= 0) return hipSuccess;
    const int64_t blocks = (L.n + 255) / 256;
    line_prep_f32_direct_kernel<<<dim3((unsigned)blocks, n_states), dim3(256), 0, s>>>(L, pps, nu_min, dnu, scale,
                                                                                        idx, w32, c32);
    return hipGetLastError();
}

hipError_t launch_line_prep_f32(const WingRec* wing, WingIdx* idx, const CoreRec* core,
                                int64_t n_lines, double nu_min, double dnu, const int32_t* scale,
                                WingRec32* w32, CoreRec32* c32, hipStream_t s, int32_t n_states)
{
    if (n_lines == 0 || n_states <= 0) return hipSuccess;
    const int64_t blocks = (n_lines + 255) / 256;
    line_prep_f32_kernel<<<dim3((unsigned)blocks, n_states), dim3(256), 0, s>>>(wing, idx, core, n_lines, nu_min,
                                                                                 dnu, scale, w32, c32);
    return hipGetLastError();
}

hipError_t launch_f32_finish(const float* sum, const float* comp, const float* series, const int32_t* scale,
                             int32_t n_points, double* kappa, int accumulate, hipStream_t s, int32_t n_states)
{
    if (n_points == 0 || n_states <= 0) return hipSuccess;
    const int64_t blocks = ((int64_t)n_points + 255) / 256;
    f32_finish_kernel<<<dim3((unsigned)blocks, n_states), dim3(256), 0, s>>>(sum, comp, series, scale, n_points,
                                                                              kappa, accumulate);
    return hipGetLastError();
}

hipError_t launch_line_prep_f64(const LinesDev& L, const PrepParams& pp, WingRec* wing,
                                WingIdx* idx, CoreRec* core, hipStream_t s)
{
    if (L.n == 0) return hipSuccess;
    int64_t blocks = (L.n + 255) / 256;
    line_prep_f64_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(L, pp, wing, idx, core);
    return hipGetLastError();
}

hipError_t launch_line_prep_f64_batch(const LinesDev& L, const PrepParams* pps, int32_t n_states, WingRec* wing,
                                      WingIdx* idx, CoreRec* core, hipStream_t s)
{
    if (L.n == 0 || n_states <= 0) return hipSuccess;
    int64_t blocks = (L.n + 255) / 256;
    line_prep_f64_batch_kernel<<<dim3((unsigned)blocks, n_states), dim3(256), 0, s>>>(L, pps, wing, idx, core);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const double* nu_sorted, int64_t n_lines, int64_t n_tiles,
                              int32_t tile_points, double nu_min, double dnu, int32_t n_points,
                              double reach, int64_t* ranges, hipStream_t s, const double* reach_of,
                              int32_t n_states)
{
    if (n_tiles == 0 || n_states <= 0) return hipSuccess;
    int64_t blocks = (n_tiles + 255) / 256;
    tile_ranges_kernel<<<dim3((unsigned)blocks, reach_of ? n_states : 1), dim3(256), 0, s>>>(
        nu_sorted, n_lines, n_tiles, tile_points, nu_min, dnu, n_points, reach, reach_of, ranges);
    return hipGetLastError();
}

hipError_t launch_eval_counts(const WingIdx* idx, int64_t n_lines, int64_t* partial,
                              int32_t n_blocks, hipStream_t s, int32_t n_states)
{
    if (n_states <= 0) return hipSuccess;
    eval_counts_kernel<<<dim3(n_blocks, n_states), dim3(256), 0, s>>>(idx, n_lines, partial);
    return hipGetLastError();
}

namespace {

__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

}  // namespace

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 4);
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    zero_words_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(static_cast<uint32_t*>(p), n);
    return hipGetLastError();
}

}  // namespace hk
