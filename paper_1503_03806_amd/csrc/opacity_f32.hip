// opacity_f32.hip -- the "kappa(nu)" stage with binary32 profile evaluation
// and compensated binary32 accumulation (§2.4, §2.5); line strengths, widths
// and windows come from the binary64 line preparation.
//
// Same decomposition as the binary64 kernels (wavefront per run of 64*P
// points, LDS-staged sorted lines, per-(line, wavefront) path decided once
// per tile, series in its own kernel).  Differences:
//  * offsets: dv/lambda = (j - jc) du - fu with an exact small-integer
//    j - jc, so no large magnitudes cancel in binary32;
//  * units: per line lambda = alpha or Gamma_L and a per-state power-of-two
//    scale of the strengths keep every value in binary32 range;
//  * reciprocals: the hardware v_rcp_f32 (< 2^-23 relative); two 3-node
//    points j and j + 64 (floor(j / 64) even) share one, 1/m_a = m_b/(m_a m_b)
//    (3-node denominators lie within 1e5 .. 1e18 in alpha units, so their
//    products stay in binary32 range), 1-node points take their own;
//  * accumulation: each point sums the lines of one 256-line block (blocks
//    aligned to global line indices) in binary32, then adds the block sum to
//    a Kahan pair (sum, comp).  With at most 256 positive terms per block the
//    block sum is within 256 * 2^-24 = 1.5e-5 of exact in the worst case,
//    the Kahan sum of blocks within ~2^-23 -- and the result does not depend
//    on the tile shape.
#include <algorithm>

#include "hk_internal.h"
#include "surrogate_dev.h"

namespace hk {
namespace {

constexpr int kWaves = 4;
constexpr int kTL = 64 * kWaves;  // 256 lines per LDS block, one per thread
constexpr int kMaxTerms = 2 * 10 + 14;
// Entries of a line's table 1/(n^2/4 + y^2) that voigt_core_f32 reads:
// n - 1 <= st + 17 with st <= 12 (x < 10.75; series points have x < 10).
constexpr int kTermsF32 = 30;
static_assert(2 * kTermsF32 <= 64, "two pieces' tables per 64 lanes");
// (kGH1Edge, kGH3Edge: a run wholly in one rule's region that the line's
// window covers in part; kGH3Core: a run wholly in the 3-node region and the
// window that holds series points)
enum : uint32_t { kSkip = 0, kGH1 = 1, kGH3 = 2, kGeneral = 3, kGH1Edge = 4, kGH3Edge = 5, kGH3Core = 6 };

// The path of one line for the points [run0, run1] of a wavefront; run_end
// is the run's nominal last point.  A run cut short by the grid end takes
// the general path, which leaves 3-node points whose pair partner lies
// beyond the grid unpaired (so a point's bits do not depend on the tile
// shape).  A run in the window and the 3-node region that holds series
// points takes the 3-node path with those points masked (kGH3Core).
// edges == false sends runs the window covers in part, and those, down the
// general path too (a check of the other paths, which give the same bits).
__device__ inline uint32_t classify(const WingIdx& r, int32_t run0, int32_t run1, int32_t run_end, bool edges)
{
    if (run0 > run1 || r.whi < run0 || r.wlo > run1) return kSkip;
    if (run1 < run_end) return kGeneral;
    const bool full = r.wlo <= run0 && r.whi >= run1;
    const bool nocore = run1 < r.clo || run0 > r.chi;
    const bool in3 = r.g3lo <= run0 && r.g3hi >= run1;
    if (!nocore) return (edges && full && in3) ? kGH3Core : kGeneral;
    if (!full && !edges) return kGeneral;
    if (run1 < r.g3lo || run0 > r.g3hi) return full ? kGH1 : kGH1Edge;
    if (in3) return full ? kGH3 : kGH3Edge;
    return kGeneral;
}

__device__ inline float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// Kahan step: (s, c) += x, with c the running correction (value = s - c).
__device__ inline void kahan_add(float& s, float& c, float x)
{
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Lines [L0, L1) at the points of grid tile t of one state (record
// pointers already offset to the state).  direct: the Kahan pair of each
// point, normalised through binary64 (sum = its value rounded to binary32,
// comp = the rest), to sum_out / comp_out; else the raw pair (sum, comp) to
// partial[j - obase].
template <int kP>
__device__ __forceinline__ void wing_f32_tile(int64_t t, int64_t L0, int64_t L1, const WingRec32* __restrict__ wing,
                                              const WingIdx* __restrict__ idx, int32_t n, float* __restrict__ sum_out,
                                              float* __restrict__ comp_out, float2* __restrict__ partial,
                                              int64_t obase, bool direct, bool edges)
{
    static_assert(kP % 2 == 0, "3-node points pair up within a lane");
    constexpr int kTilePoints = 64 * kP * kWaves;
    __shared__ WingRec32 tile[kTL];
    __shared__ WingIdx tidx[kTL];
    __shared__ uint32_t code[kTL];
    __shared__ float fjct[kTL];  // line centre index relative to the tile, exact
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int32_t tile0 = (int32_t)(t * kTilePoints);
    const int32_t run0 = tile0 + wave * 64 * kP;

    float fj[kP], s[kP], c[kP], part[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        fj[p] = (float)(run0 - tile0 + lane + 64 * p);  // exact: < 2^12
        s[p] = 0.0f;
        c[p] = 0.0f;
        part[p] = 0.0f;
    }

    for (int64_t base = L0 & ~(int64_t)(kTL - 1); base < L1; base += kTL) {
        const int cnt = (int)min((int64_t)kTL, L1 - base);
        if ((int)threadIdx.x < cnt) {
            tile[threadIdx.x] = wing[base + threadIdx.x];
            const WingIdx r = idx[base + threadIdx.x];
            tidx[threadIdx.x] = r;
            fjct[threadIdx.x] = (float)(r.jc - tile0);  // exact: |.| < 2^24
            uint32_t cw = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const int32_t r0 = tile0 + w * 64 * kP;
                const int32_t r1 = min(r0 + 64 * kP, n) - 1;
                cw |= classify(r, r0, r1, r0 + 64 * kP - 1, edges) << (8 * w);
            }
            code[threadIdx.x] = cw;
        }
        __syncthreads();
        // Maximal runs of consecutive lines on one path: a run's end is found
        // once, 64 codes at a time by a wavefront ballot, and the 1-node and
        // 3-node runs are looped over with nothing but a counter (the
        // partial sums stay in place)
        int k = 0;
        while (k < cnt) {
            const uint32_t path = ((uint32_t)__builtin_amdgcn_readfirstlane((int)code[k]) >> (8 * wave)) & 0xffu;
            int kend = k + 1;
            for (;;) {
                const int kk = kend + lane;
                const uint32_t ck = (code[min(kk, kTL - 1)] >> (8 * wave)) & 0xffu;
                const uint64_t m = __ballot(kk >= cnt || ck != path);
                if (m) {
                    kend += (int)__builtin_ctzll(m);
                    break;
                }
                kend += 64;
            }
            if (path == kSkip) {
                k = kend;
                continue;
            }
            if (path == kGH1) {
                do {
                    const float fjc = fjct[k];
                    const float du = tile[k].du, fu = tile[k].fu, Lg = tile[k].Lg, G2 = tile[k].G2;
#pragma unroll
                    for (int p = 0; p < kP; ++p) {
                        const float dv = fmaf(fj[p] - fjc, du, -fu);
                        part[p] = fmaf(Lg, rcpf(fmaf(dv, dv, G2)), part[p]);
                    }
                    ++k;
                } while (k < kend);
                continue;
            }
            if (path == kGH3) {
                do {
                    const float fjc = fjct[k];
                    const float du = tile[k].du, fu = tile[k].fu, Lg = tile[k].Lg;
                    const float M2 = tile[k].M2, M1 = tile[k].M1, M0 = tile[k].M0, Cn = tile[k].Cn;
                    const float Bn = fmaf(2.0f, tile[k].G2, -1.5f);
#pragma unroll
                    for (int p = 0; p < kP; p += 2) {
                        float nn[2], mm[2];
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            const float dv = fmaf(fj[p + e] - fjc, du, -fu);
                            const float q = dv * dv;
                            nn[e] = fmaf(q, q + Bn, Cn);
                            mm[e] = fmaf(fmaf(q + M2, q, M1), q, M0);
                        }
                        const float cp = rcpf(mm[0] * mm[1]) * Lg;
                        part[p] = fmaf(cp * mm[1], nn[0], part[p]);
                        part[p + 1] = fmaf(cp * mm[0], nn[1], part[p + 1]);
                    }
                    ++k;
                } while (k < kend);
                continue;
            }
            if (path == kGH1Edge || path == kGH3Edge) {
                do {
                    // the rule's own sequence, points outside the window left as
                    // they are: the general path's sequence for these points, bit
                    // for bit, without evaluating the other rule
                    const float fjc = fjct[k];
                    const float du = tile[k].du, fu = tile[k].fu, Lg = tile[k].Lg, G2 = tile[k].G2;
                    const int32_t wlo = tidx[k].wlo, whi = tidx[k].whi;
                    if (path == kGH1Edge) {
#pragma unroll
                        for (int p = 0; p < kP; ++p) {
                            const int32_t j = run0 + lane + 64 * p;
                            const float dv = fmaf(fj[p] - fjc, du, -fu);
                            const float acc = fmaf(Lg, rcpf(fmaf(dv, dv, G2)), part[p]);
                            part[p] = (j >= wlo && j <= whi) ? acc : part[p];
                        }
                    } else {
                        const float M2 = tile[k].M2, M1 = tile[k].M1, M0 = tile[k].M0, Cn = tile[k].Cn;
                        const float Bn = fmaf(2.0f, G2, -1.5f);
#pragma unroll
                        for (int p = 0; p < kP; p += 2) {
                            float nn[2], mm[2];
#pragma unroll
                            for (int e = 0; e < 2; ++e) {
                                const float dv = fmaf(fj[p + e] - fjc, du, -fu);
                                const float q = dv * dv;
                                nn[e] = fmaf(q, q + Bn, Cn);
                                mm[e] = fmaf(fmaf(q + M2, q, M1), q, M0);
                            }
                            const float cp = rcpf(mm[0] * mm[1]) * Lg;
#pragma unroll
                            for (int e = 0; e < 2; ++e) {
                                const int32_t j = run0 + lane + 64 * (p + e);
                                const float acc = fmaf(cp * mm[1 - e], nn[e], part[p + e]);
                                part[p + e] = (j >= wlo && j <= whi) ? acc : part[p + e];
                            }
                        }
                    }
                    ++k;
                } while (k < kend);
                continue;
            }
            if (path == kGH3Core) {
                do {
                    // the general path's sequence for these points: pairs without
                    // series points as on the 3-node path, the others one by one,
                    // the series points left as they are
                    const float fjc = fjct[k];
                    const float du = tile[k].du, fu = tile[k].fu, Lg = tile[k].Lg;
                    const float M2 = tile[k].M2, M1 = tile[k].M1, M0 = tile[k].M0, Cn = tile[k].Cn;
                    const float Bn = fmaf(2.0f, tile[k].G2, -1.5f);
                    const int32_t clo = tidx[k].clo, chi = tidx[k].chi;
#pragma unroll
                    for (int p = 0; p < kP; p += 2) {
                        float nn[2], mm[2];
                        bool cpt[2];
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            const int32_t j = run0 + lane + 64 * (p + e);
                            cpt[e] = j >= clo && j <= chi;
                            const float dv = fmaf(fj[p + e] - fjc, du, -fu);
                            const float q = dv * dv;
                            nn[e] = fmaf(q, q + Bn, Cn);
                            mm[e] = fmaf(fmaf(q + M2, q, M1), q, M0);
                        }
                        const bool paired = !cpt[0] && !cpt[1];
                        const float cp = rcpf(mm[0] * mm[1]) * Lg;
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            const float acc = paired ? fmaf(cp * mm[1 - e], nn[e], part[p + e])
                                                     : fmaf(Lg, nn[e] * rcpf(mm[e]), part[p + e]);
                            part[p + e] = cpt[e] ? part[p + e] : acc;
                        }
                    }
                    ++k;
                } while (k < kend);
                continue;
            }
            do {
                const float fjc = fjct[k];
                const float du = tile[k].du, fu = tile[k].fu, Lg = tile[k].Lg, G2 = tile[k].G2;
                const float M2 = tile[k].M2, M1 = tile[k].M1, M0 = tile[k].M0, Cn = tile[k].Cn;
                const float Bn = fmaf(2.0f, G2, -1.5f);
                const int32_t wlo = tidx[k].wlo, whi = tidx[k].whi;
                const int32_t g3lo = tidx[k].g3lo, g3hi = tidx[k].g3hi;
                const int32_t clo = tidx[k].clo, chi = tidx[k].chi;
#pragma unroll
                for (int p = 0; p < kP; p += 2) {
                    float nn[2], mm[2], v1[2];
                    bool take[2], one[2], core_pt[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int32_t j = run0 + lane + 64 * (p + e);
                        core_pt[e] = j >= clo && j <= chi;
                        take[e] = j >= wlo && j <= whi && !core_pt[e];
                        one[e] = j < g3lo || j > g3hi;
                        const float dv = fmaf(fj[p + e] - fjc, du, -fu);
                        const float q = dv * dv;
                        v1[e] = rcpf(fmaf(dv, dv, G2));
                        nn[e] = fmaf(q, q + Bn, Cn);
                        mm[e] = fmaf(fmaf(q + M2, q, M1), q, M0);
                    }
                    // two 3-node points outside the core, both on the grid: the
                    // sequence of the 3-node path above
                    const bool paired = !one[0] && !one[1] && !core_pt[0] && !core_pt[1] &&
                                        run0 + lane + 64 * (p + 1) < n;
                    const float cp = rcpf(mm[0] * mm[1]) * Lg;
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const float acc = paired ? fmaf(cp * mm[1 - e], nn[e], part[p + e])
                                                 : fmaf(Lg, one[e] ? v1[e] : nn[e] * rcpf(mm[e]), part[p + e]);
                        part[p + e] = take[e] ? acc : part[p + e];
                    }
                }
                ++k;
            } while (k < kend);
        }
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            kahan_add(s[p], c[p], part[p]);
            part[p] = 0.0f;
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        const int32_t j = run0 + lane + 64 * p;
        if (j < n) {
            if (direct) {
                const double v = (double)s[p] - (double)c[p];
                const float hi = (float)v;
                sum_out[j] = hi;
                comp_out[j] = (float)(v - (double)hi);
            } else {
                partial[j - obase] = make_float2(s[p], -c[p]);
            }
        }
    }
}

// One workgroup per work item (a grid tile of a state, or its lines in one
// segment); the layout of the binary64 kernel.
template <int kP>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kP == 4 ? 7 : 1))) void wing_f32_kernel(
    const WingRec32* __restrict__ wing, const WingIdx* __restrict__ idx, const int64_t* __restrict__ ranges,
    int64_t n_lines, int64_t n_tiles, int32_t n_states, WorkPlan wp, int32_t n, float* __restrict__ sum,
    float* __restrict__ comp, float2* __restrict__ partial, int edges)
{
    constexpr int64_t kTilePoints = 64 * kP * kWaves;
    WorkItem it;
    if (work_item(xcd_rank(blockIdx.x), wp, ranges, n_tiles, n_states, it)) {
        const int64_t o = it.st * n_lines, so = it.st * (int64_t)n;
        const bool direct = it.slot < 0;
        wing_f32_tile<kP>(it.tile, it.lo, it.hi, wing + o, idx + o, n, sum + so, comp + so,
                          partial + (direct ? 0 : it.slot * kTilePoints), it.tile * kTilePoints, direct, edges != 0);
    }
}

// The cut tiles: each point's value is the binary64 sum of its partial
// pairs in segment order, stored normalised as by a direct item.
__global__ __launch_bounds__(256) void wing_f32_reduce_kernel(WorkPlan wp, int64_t n_tiles, int32_t n_states,
                                                             int32_t tp, int32_t n, const float2* __restrict__ partial,
                                                             float* __restrict__ sum, float* __restrict__ comp)
{
    const int64_t total = wp.total[0];
    if (total == wp.n_pairs) return;  // nothing cut
    for (int64_t p = blockIdx.x; p < wp.n_pairs; p += gridDim.x) {
        const int64_t nseg = (p + 1 < wp.n_pairs ? wp.first[p + 1] : total) - wp.first[p];
        if (nseg < 2) continue;
        int64_t st, k;
        pair_decode(p, n_tiles, n_states, st, k);
        const int64_t j0 = (n_tiles - 1 - k) * tp;
        const float2* src = partial + wp.slot[p] * tp;
        for (int q = threadIdx.x; q < tp; q += blockDim.x) {
            const int64_t j = j0 + q;
            if (j >= n) break;
            double v = 0.0;
            for (int64_t sg = 0; sg < nseg; ++sg) {
                const float2 e = src[sg * tp + q];
                v += (double)e.x + (double)e.y;
            }
            const float hi = (float)v;
            sum[st * (int64_t)n + j] = hi;
            comp[st * (int64_t)n + j] = (float)(v - (double)hi);
        }
    }
}

// The core series in binary32 (the formula of voigt_core in
// opacity_f64.hip).  Binary32 cannot hold e^{+-nx} (x up to 10, n up to
// 34), so the Gaussians are summed directly, each over a fixed window of
// terms that holds everything above 2e-9 of its largest term:
//   e^{-(n/2 - x)^2}: 19 terms from n = max(1, round(2x) - 9), by the ratio
//     recurrence g(n+1) = g(n) e^{x - n/2 - 1/4}, started at its largest
//     term so that nothing underflows before it matters;
//   e^{-(n/2 + x)^2}: n = 1 .. 9 (below e^{-20} of e^{-x^2} beyond).
// The trip counts are the same for every lane.  The reciprocals here and in
// the tables (inv[n-1] = 1/(n^2/4 + y^2)) are the hardware's (within 1 ulp),
// well inside the binary32 path's error budget.
__device__ float voigt_core_f32(float x, float y, float ex, float T1, const float* inv)
{
    const float d = 0.60653065971263342f;  // e^{-1/2}
    const float E = expf(-x * x);
    const int st = min(max(1, (int)rintf(2.0f * x) - 9), kTermsF32 - 18);
    float s3 = 0.0f;
    {
        const float h = 0.5f * (float)st - x;
        float g = expf(-h * h);
        float r = expf(-h - 0.25f);  // e^{x - st/2 - 1/4}
#pragma unroll
        for (int k = 0; k < 19; ++k) {
            s3 = fmaf(g, inv[st - 1 + k], s3);
            g *= r;
            r *= d;
        }
    }
    float s2 = 0.0f;
    {  // e^{-(n/2 + x)^2}, n = 1 .. 9
        const float c = 0.77880078307140487f;  // e^{-1/4}
        const float dn = expf(-x);
        float g = E * dn * c, r = dn * c * d;
#pragma unroll
        for (int n = 1; n <= 9; ++n) {
            s2 = fmaf(g, inv[n - 1], s2);
            g *= r;
            r *= d;
        }
    }
    float sn, cs;
    sincosf(x * y, &sn, &cs);
    const float cos2 = (cs - sn) * (cs + sn);
    const float sy = (y > 0.0f) ? sn * __builtin_amdgcn_rcpf(y) : x;
    const float inv_pi = 0.31830988618379067f;
    return E * fmaf(ex, cos2, sn * sy * inv_pi) + (y * inv_pi) * fmaf(-cos2 * E, T1, 0.5f * (s2 + s3));
}

// Core-region terms: as core_f64_kernel (each wavefront owns a run of
// kCoreRun points; the series pieces of the lines that meet it are packed
// into 64-lane chunks, at most kChunkPieces per chunk; each lane adds its
// point's value to the run's sums in LDS, pieces in line order); the run's
// ordered binary32 series sums go to a grid of their own, which the finish
// adds to the wing's Kahan pairs (so the two kernels can run at the same
// time).  Lines [L0, L1) of tile t; direct: series_j = the run's sum (every
// point, 0 where no line reaches); else every point's sum to
// partial[j - obase].
constexpr int kCoreRun = 256;
constexpr int kCoreTilePoints = kCoreRun * kWaves;
constexpr int kCoreBatch = 32;
constexpr int kChunkPieces = 16;

struct alignas(16) CorePiece32 {  // one line's series points within a run
    float dx, fx, y, y2, ex, norm, T1;
    int32_t jc;     // the line's nearest grid point
    int32_t a;      // its first point in the run
    int32_t start;  // where its points begin in the batch's flattened list
};

__device__ inline int32_t wave_incl_scan(int32_t v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

__device__ __forceinline__ void core_f32_tile(int64_t t, int64_t L0, int64_t L1, const WingIdx* __restrict__ idx,
                                              const CoreRec32* __restrict__ core, int32_t n, float* __restrict__ series,
                                              float* __restrict__ partial, int64_t obase, bool direct)
{
    __shared__ float acc_tab[kWaves][kCoreRun];
    __shared__ CorePiece32 piece_tab[kWaves][kCoreBatch];
    __shared__ float w_tab[kWaves][kChunkPieces * kTermsF32];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t run0 = (int32_t)(t * kCoreTilePoints) + wave * kCoreRun;
    const int32_t run1 = min(run0 + kCoreRun, n) - 1;
    if (run0 > run1) return;
    float* acc = acc_tab[wave];
    CorePiece32* pc = piece_tab[wave];
    float* wt = w_tab[wave];
    for (int q = lane; q < kCoreRun; q += 64) acc[q] = 0.0f;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // two pieces' tables at a time: lane l < 2 kTermsF32 builds entry nn of
    // the first (l < kTermsF32) or the second piece
    const int half = lane >= kTermsF32 ? 1 : 0;
    const int nn_lane = lane - half * kTermsF32;
    const float m_lane = 0.5f * (float)(nn_lane + 1);

    for (int64_t base = L0; base < L1; base += kCoreBatch) {
        const int64_t i = base + lane;
        int32_t a = 1, b = 0, jc = 0;
        if (lane < kCoreBatch && i < L1) {
            const WingIdx r = idx[i];
            a = max(max(r.clo, r.wlo), run0);
            b = min(min(r.chi, r.whi), run1);
            jc = r.jc;
        }
        const bool has = a <= b;
        const uint64_t m = __ballot(has);
        if (m == 0) continue;
        const int np = __builtin_popcountll(m);
        const int32_t cnt = has ? b - a + 1 : 0;
        const int32_t incl = wave_incl_scan(cnt, lane);
        const int32_t total = __shfl(incl, 63, 64);
        if (has) {
            const CoreRec32 cr = core[i];
            CorePiece32 pp;
            pp.dx = cr.dx;
            pp.fx = cr.fx;
            pp.y = cr.y;
            pp.y2 = cr.y2;
            pp.ex = cr.ex;
            pp.norm = cr.norm;
            pp.T1 = cr.T1;
            pp.jc = jc;
            pp.a = a;
            pp.start = incl - cnt;
            pc[__builtin_popcountll(m & below)] = pp;
        }
        __builtin_amdgcn_wave_barrier();
        const int32_t st_k = lane < np ? pc[lane].start : total;
        int s_lo = 0;
        for (int32_t f0 = 0; f0 < total;) {
            // (s_lo, s_end: the same in every lane, kept in scalar registers)
            s_lo = __builtin_amdgcn_readfirstlane(s_lo);
            int s_end = __builtin_popcountll(__ballot(lane < np && st_k < f0 + 64));
            s_end = __builtin_amdgcn_readfirstlane(min(s_end, s_lo + kChunkPieces));
            const int32_t next_start = __builtin_amdgcn_readlane(st_k, min(s_end, 63));
            const int32_t f_end = s_end < np ? min(next_start, f0 + 64) : min(total, f0 + 64);
            for (int k = s_lo; k < s_end; k += 2) {
                const int kk = k + half;
                if (lane < 2 * kTermsF32 && kk < s_end)
                    wt[(kk - s_lo) * kTermsF32 + nn_lane] = __builtin_amdgcn_rcpf(fmaf(m_lane, m_lane, pc[kk].y2));
            }
            __builtin_amdgcn_wave_barrier();
            const int32_t f = f0 + lane;
            const bool act = f < f_end;
            int my = s_lo;
            for (int s = s_lo + 1; s < s_end; ++s) my = __builtin_amdgcn_readlane(st_k, s) <= f ? s : my;
            const CorePiece32& pp = pc[my];
            const int32_t j = pp.a + (f - pp.start);
            const int32_t jr = act ? j - run0 : 0;
            const float x = act ? fabsf(fmaf((float)(j - pp.jc), pp.dx, -pp.fx)) : 0.0f;
            const float* w = wt + (my - s_lo) * kTermsF32;
            float v = 0.0f;
            if (act) v = pp.norm * voigt_core_f32(x, pp.y, pp.ex, pp.T1, w);
            // add in line order: lanes of one piece hold distinct points, and
            // the pieces' read-add-writes stay in order (volatile, and the
            // fence: neither merged nor reordered by the compiler; a
            // wavefront's LDS operations are carried out in issue order).
            // (The LDS atomic add that core_f64_tile uses measured slower
            // here.)
            lds_volatile<float>* vacc = (lds_volatile<float>*)acc;
            for (int s = s_lo; s < s_end; ++s) {
                if (act && my == s) vacc[jr] = vacc[jr] + v;
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            }
            s_lo = (s_end < np && f_end >= next_start) ? s_end : s_end - 1;
            f0 = f_end;
        }
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();
    for (int q = lane; q < kCoreRun; q += 64) {
        const int32_t jj = run0 + q;
        if (jj <= run1) {
            if (direct)
                series[jj] = acc[q];
            else
                partial[jj - obase] = acc[q];
        }
    }
}

// The series-region terms with the learned surrogate (HK_F32_SURROGATE): the
// pieces of a wavefront's run are flattened as in core_f32_tile, and every
// window of kSurrWin flattened points is taken in four passes, so that the
// network and the series each run on full 64-lane batches and never both for
// one batch: (A) each point's cell is looked up and the point's index goes to
// the list of certified points or to that of the others (order kept);
// (B) the series for the others, 64 at a time; (C) the network for the
// certified ones, 64 at a time, its bfloat16 weights staged in LDS once per
// workgroup; (D) the values, kept per point in LDS, are added to the run's
// sums in line order as in core_f32_tile.  Returns the points the network
// evaluated.  (The values are those core_f32_tile<true> computes: the same
// per-point arithmetic, only grouped differently.)
constexpr int kSurrWin = 256;

__device__ __forceinline__ int64_t core_f32_surr_tile(int64_t t, int64_t L0, int64_t L1,
                                                      const WingIdx* __restrict__ idx,
                                                      const CoreRec32* __restrict__ core, int32_t n,
                                                      float* __restrict__ series, float* __restrict__ partial,
                                                      int64_t obase, bool direct, const surr::MlpBf16* P,
                                                      const uint8_t* __restrict__ mask)
{
    __shared__ __align__(16) uint16_t mlp_tab[kWaves][64 * surr::kLd];
    __shared__ float acc_tab[kWaves][kCoreRun];
    __shared__ CorePiece32 piece_tab[kWaves][kCoreBatch];
    __shared__ float w_tab[kWaves][kCoreBatch * kMaxTerms];
    __shared__ float val_tab[kWaves][kSurrWin];
    __shared__ uint8_t own_tab[kWaves][kSurrWin];
    __shared__ uint16_t list_tab[kWaves][2][kSurrWin];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t run0 = (int32_t)(t * kCoreTilePoints) + wave * kCoreRun;
    const int32_t run1 = min(run0 + kCoreRun, n) - 1;
    if (run0 > run1) return 0;
    float* acc = acc_tab[wave];
    CorePiece32* pc = piece_tab[wave];
    float* wt = w_tab[wave];
    float* val = val_tab[wave];
    uint8_t* own = own_tab[wave];
    uint16_t* cert = list_tab[wave][0];
    uint16_t* plain = list_tab[wave][1];
    for (int q = lane; q < kCoreRun; q += 64) acc[q] = 0.0f;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int64_t n_used = 0;

    for (int64_t base = L0; base < L1; base += kCoreBatch) {
        const int64_t i = base + lane;
        int32_t a = 1, b = 0, jc = 0;
        if (lane < kCoreBatch && i < L1) {
            const WingIdx r = idx[i];
            a = max(max(r.clo, r.wlo), run0);
            b = min(min(r.chi, r.whi), run1);
            jc = r.jc;
        }
        const bool has = a <= b;
        const uint64_t m = __ballot(has);
        if (m == 0) continue;
        const int np = __builtin_popcountll(m);
        const int32_t cnt = has ? b - a + 1 : 0;
        const int32_t incl = wave_incl_scan(cnt, lane);
        const int32_t total = __shfl(incl, 63, 64);
        if (has) {
            const CoreRec32 cr = core[i];
            CorePiece32 pp;
            pp.dx = cr.dx;
            pp.fx = cr.fx;
            pp.y = cr.y;
            pp.y2 = cr.y2;
            pp.ex = cr.ex;
            pp.norm = cr.norm;
            pp.T1 = cr.T1;
            pp.jc = jc;
            pp.a = a;
            pp.start = incl - cnt;
            pc[__builtin_popcountll(m & below)] = pp;
        }
        __builtin_amdgcn_wave_barrier();
        // the series tables of every piece of the batch
        for (int e = lane; e < np * kMaxTerms; e += 64) {
            const int k = e / kMaxTerms, nn = e - k * kMaxTerms;
            const float mm = 0.5f * (float)(nn + 1);
            wt[e] = __builtin_amdgcn_rcpf(fmaf(mm, mm, pc[k].y2));
        }
        const int32_t st_k = lane < np ? pc[lane].start : total;
        __builtin_amdgcn_wave_barrier();
        int s_lo = 0;  // the piece holding point f0
        for (int32_t f0 = 0; f0 < total; f0 += kSurrWin) {
            const int32_t f1 = min(total, f0 + kSurrWin);
            // (A) each point's piece and cell; the two lists
            int n_cert = 0, n_plain = 0;
            int s_at = s_lo;
            for (int32_t c0 = f0; c0 < f1; c0 += 64) {
                const int32_t f = c0 + lane;
                const bool act = f < f1;
                while (s_at + 1 < np && __shfl(st_k, s_at + 1, 64) <= c0) ++s_at;
                int my = s_at;
                for (int s = s_at + 1; s < np && __shfl(st_k, s, 64) < c0 + 64; ++s)
                    my = __shfl(st_k, s, 64) <= f ? s : my;
                const CorePiece32& pp = pc[my];
                const int32_t j = pp.a + (f - pp.start);
                const float x = act ? fabsf(fmaf((float)(j - pp.jc), pp.dx, -pp.fx)) : 0.0f;
                const bool use = act && surr::certified(mask, x, pp.y);
                const uint64_t um = __ballot(use), pm = __ballot(act && !use);
                if (act) own[f - f0] = (uint8_t)my;
                if (use) cert[n_cert + __builtin_popcountll(um & below)] = (uint16_t)(f - f0);
                if (act && !use) plain[n_plain + __builtin_popcountll(pm & below)] = (uint16_t)(f - f0);
                n_cert += __builtin_popcountll(um);
                n_plain += __builtin_popcountll(pm);
            }
            n_used += n_cert;
            __builtin_amdgcn_wave_barrier();
            // (B) the series, full batches of the other points
            for (int c = 0; c < n_plain; c += 64) {
                if (c + lane < n_plain) {
                    const int q = plain[c + lane];
                    const int my = own[q];
                    const CorePiece32& pp = pc[my];
                    const int32_t j = pp.a + (f0 + q - pp.start);
                    const float x = fabsf(fmaf((float)(j - pp.jc), pp.dx, -pp.fx));
                    val[q] = pp.norm * voigt_core_f32(x, pp.y, pp.ex, pp.T1, wt + my * kMaxTerms);
                }
            }
            // (C) the network, full batches of the certified points
            for (int c = 0; c < n_cert; c += 64) {
                const bool act = c + lane < n_cert;
                const int q = act ? cert[c + lane] : 0;
                const CorePiece32& pp = pc[own[q]];
                const int32_t j = pp.a + (f0 + q - pp.start);
                const float x = act ? fabsf(fmaf((float)(j - pp.jc), pp.dx, -pp.fx)) : 0.0f;
                const float z = surr::mlp_forward<false>(P, mlp_tab[wave], surr::feature_x(x),
                                                         surr::feature_y(act ? pp.y : 1.0f));
                if (act) val[q] = pp.norm * surr::surrogate_K(x, pp.y, z);
            }
            __builtin_amdgcn_wave_barrier();
            // (D) add in line order (see core_f64_tile)
            for (int32_t c0 = f0; c0 < f1; c0 += 64) {
                const int32_t f = c0 + lane;
                const bool act = f < f1;
                const int my = act ? own[f - f0] : 0;
                const int s_first = __shfl(my, 0, 64);
                const int s_last = __shfl(my, min(f1 - c0, 64) - 1, 64);
                const CorePiece32& pp = pc[my];
                const int32_t jr = act ? pp.a + (f - pp.start) - run0 : 0;
                const float v = act ? val[f - f0] : 0.0f;
                lds_volatile<float>* vacc = (lds_volatile<float>*)acc;
                for (int s = s_first; s <= s_last; ++s) {
                    if (act && my == s) vacc[jr] = vacc[jr] + v;
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                }
            }
            s_lo = s_at;
            __builtin_amdgcn_wave_barrier();
        }
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();
    for (int q = lane; q < kCoreRun; q += 64) {
        const int32_t jj = run0 + q;
        if (jj <= run1) {
            if (direct)
                series[jj] = acc[q];
            else
                partial[jj - obase] = acc[q];
        }
    }
    return n_used;
}

// One workgroup per work item of the series (the layout of wing_f32_kernel),
// in plan order as in the binary64 series kernel;
// kSurr: the learned surrogate where certified (single state), and
// used[blockIdx.x] = the points of the item the network evaluated (every
// launched workgroup writes its slot, so the counts need no clearing).
template <bool kSurr>
__global__ __launch_bounds__(64 * kWaves) void core_f32_kernel(
    const WingIdx* __restrict__ idx, const CoreRec32* __restrict__ core, const int64_t* __restrict__ ranges,
    int64_t n_lines, int64_t n_tiles, int32_t n_states, WorkPlan wp, int32_t n, float* __restrict__ series,
    float* __restrict__ partial, const surr::MlpBf16* __restrict__ P, const uint8_t* __restrict__ mask,
    int64_t* __restrict__ used)
{
    WorkItem it;
    int64_t n_used = 0;
    if (work_item(blockIdx.x, wp, ranges, n_tiles, n_states, it)) {
        const int64_t o = it.st * n_lines, so = it.st * (int64_t)n;
        const bool direct = it.slot < 0;
        if constexpr (kSurr)
            n_used = core_f32_surr_tile(it.tile, it.lo, it.hi, idx + o, core + o, n, series + so,
                                        partial + (direct ? 0 : it.slot * kCoreTilePoints),
                                        it.tile * kCoreTilePoints, direct, P, mask);
        else
            core_f32_tile(it.tile, it.lo, it.hi, idx + o, core + o, n, series + so,
                          partial + (direct ? 0 : it.slot * kCoreTilePoints), it.tile * kCoreTilePoints, direct);
    }
    if constexpr (kSurr) {
        __shared__ int64_t wave_used[kWaves];
        if ((threadIdx.x & 63) == 0) wave_used[threadIdx.x >> 6] = n_used;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t t = 0;
            for (int w = 0; w < kWaves; ++w) t += wave_used[w];
            used[blockIdx.x] = t;
        }
    }
}

// Cut series tiles: series_j = the partials summed in segment order in
// binary32.
__global__ __launch_bounds__(256) void core_f32_reduce_kernel(WorkPlan wp, int64_t n_tiles, int32_t n_states,
                                                             int32_t tp, int32_t n, const float* __restrict__ partial,
                                                             float* __restrict__ series)
{
    const int64_t total = wp.total[0];
    if (total == wp.n_pairs) return;  // nothing cut
    for (int64_t p = blockIdx.x; p < wp.n_pairs; p += gridDim.x) {
        const int64_t nseg = (p + 1 < wp.n_pairs ? wp.first[p + 1] : total) - wp.first[p];
        if (nseg < 2) continue;
        int64_t st, k;
        pair_decode(p, n_tiles, n_states, st, k);
        const int64_t j0 = (n_tiles - 1 - k) * tp;
        const float* src = partial + wp.slot[p] * tp;
        for (int q = threadIdx.x; q < tp; q += blockDim.x) {
            const int64_t j = j0 + q;
            if (j >= n) break;
            float v = 0.0f;
            for (int64_t sg = 0; sg < nseg; ++sg) v += src[sg * tp + q];
            series[st * (int64_t)n + j] = v;
        }
    }
}

// total[0] (+)= used[0] + ... + used[n-1], one workgroup (the surrogate's
// per-workgroup counts of a launch).
__global__ __launch_bounds__(256) void sum_counts_kernel(const int64_t* __restrict__ used, int64_t n,
                                                         int64_t* __restrict__ total, int add)
{
    __shared__ int64_t part[256];
    int64_t t = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) t += used[i];
    part[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) total[0] = add ? total[0] + part[0] : part[0];
}

template <int kP>
hipError_t launch_wing(const WingRec32* wing, const WingIdx* idx, const int64_t* ranges, int64_t n_lines,
                       int64_t n_tiles, int32_t n_states, const WorkPlan& wp, int32_t n, float* sum, float* comp,
                       float2* partial, int edges, hipStream_t s)
{
    const int64_t nb = plan_blocks(wp.launch_items);
    if (nb > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    wing_f32_kernel<kP><<<dim3((unsigned)nb), dim3(64 * kWaves), 0, s>>>(wing, idx, ranges, n_lines, n_tiles,
                                                                        n_states, wp, n, sum, comp, partial, edges);
    const int64_t nr = std::min<int64_t>(wp.n_pairs, 8192);
    wing_f32_reduce_kernel<<<dim3((unsigned)nr), dim3(256), 0, s>>>(wp, n_tiles, n_states, 64 * kP * kWaves, n,
                                                                    partial, sum, comp);
    return hipGetLastError();
}

}  // namespace

int32_t opacity_f32_tile_points(int points_per_lane) { return 64 * points_per_lane * kWaves; }
int32_t core_f32_tile_points() { return kCoreTilePoints; }

hipError_t launch_wing_f32(int points_per_lane, const WingRec32* wing, const WingIdx* idx, const int64_t* ranges,
                           int64_t n_lines, int64_t n_tiles, int32_t n_states, const WorkPlan& wp, int32_t n_points,
                           float* sum, float* comp, float2* partial, int edges, hipStream_t s)
{
    if (n_tiles == 0 || n_states == 0) return hipSuccess;
    switch (points_per_lane) {
    case 2:
        return launch_wing<2>(wing, idx, ranges, n_lines, n_tiles, n_states, wp, n_points, sum, comp, partial, edges, s);
    case 4:
        return launch_wing<4>(wing, idx, ranges, n_lines, n_tiles, n_states, wp, n_points, sum, comp, partial, edges, s);
    case 8:
        return launch_wing<8>(wing, idx, ranges, n_lines, n_tiles, n_states, wp, n_points, sum, comp, partial, edges, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_core_f32(const WingIdx* idx, const CoreRec32* core, const int64_t* ranges, int64_t n_lines,
                           int64_t n_tiles, int32_t n_states, const WorkPlan& wp, int32_t n_points, float* series,
                           float* partial, const void* surrogate, const uint8_t* mask, int64_t* used,
                           int64_t used_cap, hipStream_t s)
{
    if (n_tiles == 0 || n_states == 0) return hipSuccess;
    if (surrogate && n_states != 1) return hipErrorInvalidValue;
    const int64_t nb = plan_blocks(wp.launch_items);
    if (nb > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    if (surrogate && (!used || nb > used_cap)) return hipErrorInvalidValue;
    const auto* P = static_cast<const surr::MlpBf16*>(surrogate);
    if (surrogate)
        core_f32_kernel<true><<<dim3((unsigned)nb), dim3(64 * kWaves), 0, s>>>(
            idx, core, ranges, n_lines, n_tiles, n_states, wp, n_points, series, partial, P, mask, used);
    else
        core_f32_kernel<false><<<dim3((unsigned)nb), dim3(64 * kWaves), 0, s>>>(
            idx, core, ranges, n_lines, n_tiles, n_states, wp, n_points, series, partial, nullptr, nullptr,
            nullptr);
    const int64_t nr = std::min<int64_t>(wp.n_pairs, 8192);
    core_f32_reduce_kernel<<<dim3((unsigned)nr), dim3(256), 0, s>>>(wp, n_tiles, n_states, kCoreTilePoints,
                                                                    n_points, partial, series);
    return hipGetLastError();
}

hipError_t launch_sum_counts(const int64_t* used, int64_t n, int64_t* total, int add, hipStream_t s)
{
    sum_counts_kernel<<<dim3(1), dim3(256), 0, s>>>(used, n, total, add);
    return hipGetLastError();
}

}  // namespace hk
