// opacity_f64.hip -- the "kappa(nu)" stage in binary64 (§2.4, §2.5).
//
// The paper's GPU scheme is a serial loop over lines with the grid spread
// over threads, kappa held in a register (§2.5).  Here each wavefront owns a
// contiguous run of 64*P grid points (lane l holds points run0 + l + 64 p),
// a workgroup's waves share an LDS tile of line records (lines sorted by
// wavenumber, §2.5's global-to-shared staging), and every wavefront walks the
// lines of its tile in order, so each point sums its lines in ascending
// (nu, index) order without atomics.
//
// Two kernels per call:
//  wing: the 3-node and 1-node Gauss-Hermite rules (a^2+u^2 >= 100) for
//        every line and point; it writes kappa (over the work items of
//        work_plan.hip: a tile, or the part of its lines in one segment,
//        whose partial sums a reduction adds in segment order).
//  core: the series for a^2+u^2 < 100, a few hundred times rarer but ~30
//        times dearer per point and heavy in registers; it writes its own
//        ordered sums into a grid of their own (so the two kernels can run
//        at the same time, on two streams), added to kappa afterwards.
// So kappa_j = sum_wing + sum_core, each in line order: reproducible bit for
// bit, independent of the tile shape.
#include <algorithm>

#include "hk_internal.h"

namespace hk {
namespace {

constexpr int kWaves = 4;            // wavefronts per workgroup
constexpr int kTL = 64 * kWaves;     // line records per LDS tile: one per thread
constexpr int kMaxTerms = 2 * 10 + 14;  // series terms: n = 1 .. 2 ceil(x) + 14, x < 10
static_assert(kMaxTerms <= 64, "one lane per series term builds the tables");

// Per-(line, wavefront) path, decided once per LDS tile.
// (kGH1Edge, kGH3Edge: a run wholly in one rule's region that the line's
// window covers in part; kGH3Core: a run wholly in the 3-node region and the
// window that holds series points)
enum : uint32_t { kSkip = 0, kGH1 = 1, kGH3 = 2, kGeneral = 3, kGH1Edge = 4, kGH3Edge = 5, kGH3Core = 6 };

// num / den to about 2^-48 relative: the hardware reciprocal (relative
// error below 2^-24 on gfx950) and one Newton correction of the quotient.
// Callers discard the result (by select) wherever den may be 0.
__device__ inline double qdiv(double num, double den)
{
    const double r = __builtin_amdgcn_rcp(den);
    const double q = num * r;
    const double e = fma(-den, q, num);
    return fma(e, r, q);
}

// 1 / den to about 2^-48 relative (one Newton step on the reciprocal).
__device__ inline double qrcp(double den)
{
    const double r = __builtin_amdgcn_rcp(den);
    return fma(r, fma(-den, r, 1.0), r);
}

// Work items run dearest tile first (high wavenumber: wider Doppler cores,
// more 3-node points), so cheap tiles fill the launch's tail, and are dealt
// to the 8 XCDs (each with its own L2) in chunks of consecutive tiles
// (xcd_rank), so an XCD's neighbouring tiles, which read mostly the same
// lines, share its L2 while every XCD gets a mix of dear and cheap chunks.

// The path of one line for the points [run0, run1] of a wavefront; run_end
// is the run's nominal last point.  A run cut short by the grid end takes
// the general path, which evaluates points whose group reaches beyond the
// grid one by one, and so do lines outside the grouping range.  A run
// wholly in one rule's region that the line's window covers only in part
// takes the rule's own path with a window mask (kGH1Edge, kGH3Edge); a run
// in the window and the 3-node region that holds series points takes the
// 3-node path with the series points masked (kGH3Core).  edges == false
// sends these down the general path instead (a check: both give the same
// bits).
__device__ inline uint32_t classify(const WingIdx& r, int32_t run0, int32_t run1, int32_t run_end, bool edges)
{
    if (run0 > run1 || r.whi < run0 || r.wlo > run1) return kSkip;
    if (run1 < run_end || !(r.flags & kGroupSafe)) return kGeneral;
    const bool full = r.wlo <= run0 && r.whi >= run1;
    const bool nocore = run1 < r.clo || run0 > r.chi;
    const bool out3 = run1 < r.g3lo || run0 > r.g3hi;  // wholly 1-node
    const bool in3 = r.g3lo <= run0 && r.g3hi >= run1;  // wholly 3-node
    if (!edges) {
        if (!full || !nocore) return kGeneral;
        return out3 ? kGH1 : in3 ? kGH3 : kGeneral;
    }
    if (!nocore) return (full && in3) ? kGH3Core : kGeneral;
    if (out3) return full ? kGH1 : kGH1Edge;
    if (in3) return full ? kGH3 : kGH3Edge;
    return kGeneral;
}

// An index interval [lo, hi] relative to a tile's first point t0, each end
// clipped to [-1, tp] (tp = the tile's points), packed as two int16: for the
// tile's points 0 .. tp-1 every comparison with an end comes out as with the
// unclipped interval.
__device__ inline uint32_t bnd_pack(int32_t lo, int32_t hi, int32_t t0, int32_t tp)
{
    const int64_t l = min<int64_t>(max<int64_t>((int64_t)lo - t0, -1), tp);
    const int64_t h = min<int64_t>(max<int64_t>((int64_t)hi - t0, -1), tp);
    return ((uint32_t)l & 0xffffu) | ((uint32_t)h << 16);
}
__device__ inline int32_t bnd_lo(uint32_t w) { return (int32_t)(int16_t)(w & 0xffffu); }
__device__ inline int32_t bnd_hi(uint32_t w) { return (int32_t)w >> 16; }

// 3-node rule of one point: S Phi = Lg n / m with q = dv^2,
// n = q (q + Bn) + Cn, m = (q + G2)(q (q + B) + C) = ((q + M2) q + M1) q + M0.
__device__ inline void gh3_nm(double dv, double M2, double M1, double M0, double Bn, double Cn,
                              double& n, double& m)
{
    const double q = dv * dv;
    n = fma(q, q + Bn, Cn);
    m = fma(fma(q + M2, q, M1), q, M0);
}

// Points form groups of four that share one reciprocal (the binary64
// reciprocal issues at a quarter of the FMA rate): with d_0 .. d_3 the
// group's denominators, P01 = d_0 d_1, P23 = d_2 d_3, c = rcp(P01 P23) Lg,
// 1/d_0 = (c P23) d_1 / Lg and so on.  Point j groups with j + 64, j + 128
// and j + 192 when floor(j / 64) is a multiple of 4 (runs start at multiples
// of 256), and each group type has one fixed sequence of operations, so a
// point's value has the same bits whichever path or tile shape computes it:
//   all 1-node:  acc_0 += (c P23) * d_1   (one fma; likewise for the others)
//   otherwise:   acc_0 += ((c P23) d_1) * num_0
// (num = 1 for a 1-node point, n of the 3-node rule otherwise).
// Lines [L0, L1) at the points of grid tile t of one state (record
// pointers already offset to the state): out[j - obase] = the ordered sum,
// or += it with accumulate.
template <int kP>
__device__ __forceinline__ void wing_f64_tile(int64_t t, int64_t L0, int64_t L1, const WingRec* __restrict__ wing,
                                              const WingIdx* __restrict__ idx, double nu_min, double dnu, int32_t n,
                                              double* __restrict__ out, int64_t obase, int accumulate, bool edges)
{
    static_assert(kP % 4 == 0, "points are processed in groups of four");
    constexpr int kTilePoints = 64 * kP * kWaves;
    __shared__ WingRec tile[kTL];
    __shared__ uint8_t code[kWaves][kTL];  // path of each staged line, per wavefront
    // each staged line's window, 3-node and series intervals and flags,
    // relative to the tile (bnd_pack), for the window-edge and general paths
    __shared__ uint4 bnd[kTL];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int32_t tile0 = (int32_t)(t * kTilePoints);
    const int32_t run0 = tile0 + wave * 64 * kP;
    const int32_t rel0 = wave * 64 * kP;  // run0 relative to the tile

    double nuj[kP], acc[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        const int32_t j = run0 + lane + 64 * p;
        nuj[p] = fma((double)j, dnu, nu_min);
        acc[p] = 0.0;
    }

    for (int64_t base = L0; base < L1; base += kTL) {
        const int cnt = (int)min((int64_t)kTL, L1 - base);
        // stage one record per thread and decide its path for each wavefront
        if ((int)threadIdx.x < cnt) {
            tile[threadIdx.x] = wing[base + threadIdx.x];
            const WingIdx r = idx[base + threadIdx.x];
            bnd[threadIdx.x] = make_uint4(bnd_pack(r.wlo, r.whi, tile0, kTilePoints),
                                          bnd_pack(r.g3lo, r.g3hi, tile0, kTilePoints),
                                          bnd_pack(r.clo, r.chi, tile0, kTilePoints), (uint32_t)r.flags);
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const int32_t r0 = tile0 + w * 64 * kP;
                const int32_t r1 = min(r0 + 64 * kP, n) - 1;
                code[w][threadIdx.x] = (uint8_t)classify(r, r0, r1, r0 + 64 * kP - 1, edges);
            }
        }
        __syncthreads();
        // Maximal runs of consecutive lines on one path: a run's end is found
        // once, 64 codes at a time by a wavefront ballot, and the 1-node and
        // 3-node runs are looped over with nothing but a counter (few scalar
        // instructions per line beside the path's own work; the accumulators
        // stay in place)
        const uint8_t* cw = code[wave];
        // The 1-node and 3-node loops read each record by uniform (scalar)
        // loads, its values then scalar operands of the VALU work, from the
        // caches that the staging loads above have just filled: no LDS reads
        // and no VGPRs for them (binary64 step 7.62 -> 7.20 ms; reading the
        // records only that way, without the staging, measured slower: the
        // scalar loads then miss).  The rarer paths read the LDS copy.
        const WingRec* grec = wing + base;
        int k = 0;
        while (k < cnt) {
            const uint32_t path = (uint32_t)__builtin_amdgcn_readfirstlane((int)cw[k]);
            int kend = k + 1;
            for (;;) {
                const int kk = kend + lane;
                const uint64_t m = __ballot(kk >= cnt || cw[min(kk, kTL - 1)] != path);
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
                    const double nu0 = grec[k].nu0, Lg = grec[k].Lg, G2 = grec[k].G2;
#pragma unroll
                    for (int p = 0; p < kP; p += 4) {
                        double D[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const double dv = nuj[p + e] - nu0;
                            D[e] = fma(dv, dv, G2);
                        }
                        const double P01 = D[0] * D[1], P23 = D[2] * D[3];
                        const double c = qrcp(P01 * P23) * Lg;
                        const double c01 = c * P23, c23 = c * P01;
                        acc[p] = fma(c01, D[1], acc[p]);
                        acc[p + 1] = fma(c01, D[0], acc[p + 1]);
                        acc[p + 2] = fma(c23, D[3], acc[p + 2]);
                        acc[p + 3] = fma(c23, D[2], acc[p + 3]);
                    }
                    ++k;
                } while (k < kend);
                continue;
            }
            if (path == kGH3) {
                do {
                    const double nu0 = grec[k].nu0, Lg = grec[k].Lg;
                    const double M2 = grec[k].M2, M1 = grec[k].M1, M0 = grec[k].M0, Bn = grec[k].Bn, Cn = grec[k].Cn;
#pragma unroll
                    for (int p = 0; p < kP; p += 4) {
                        double nn[4], mm[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) gh3_nm(nuj[p + e] - nu0, M2, M1, M0, Bn, Cn, nn[e], mm[e]);
                        const double P01 = mm[0] * mm[1], P23 = mm[2] * mm[3];
                        const double c = qrcp(P01 * P23) * Lg;
                        const double c01 = c * P23, c23 = c * P01;
                        acc[p] = fma(c01 * mm[1], nn[0], acc[p]);
                        acc[p + 1] = fma(c01 * mm[0], nn[1], acc[p + 1]);
                        acc[p + 2] = fma(c23 * mm[3], nn[2], acc[p + 2]);
                        acc[p + 3] = fma(c23 * mm[2], nn[3], acc[p + 3]);
                    }
                    ++k;
                } while (k < kend);
                continue;
            }
            if (path == kGH1Edge || path == kGH3Edge) {
                do {
                    // the rule's own sequence, points outside the window adding
                    // zero: the general path's sequence for these groups, bit
                    // for bit, without evaluating the other rule
                    const uint32_t wb = (uint32_t)__builtin_amdgcn_readfirstlane((int)bnd[k].x);
                    const int32_t wlo = bnd_lo(wb), whi = bnd_hi(wb);
                    const double nu0 = tile[k].nu0, Lg = tile[k].Lg;
                    bool take[kP];
#pragma unroll
                    for (int p = 0; p < kP; ++p) {
                        const int32_t jr = rel0 + lane + 64 * p;
                        take[p] = jr >= wlo && jr <= whi;
                    }
                    if (path == kGH1Edge) {
                        const double G2 = tile[k].G2;
#pragma unroll
                        for (int p = 0; p < kP; p += 4) {
                            double D[4];
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const double dv = nuj[p + e] - nu0;
                                D[e] = fma(dv, dv, G2);
                            }
                            const double P01 = D[0] * D[1], P23 = D[2] * D[3];
                            const double c = qrcp(P01 * P23) * Lg;
                            const double c01 = c * P23, c23 = c * P01;
                            acc[p] = fma(take[p] ? c01 : 0.0, D[1], acc[p]);
                            acc[p + 1] = fma(take[p + 1] ? c01 : 0.0, D[0], acc[p + 1]);
                            acc[p + 2] = fma(take[p + 2] ? c23 : 0.0, D[3], acc[p + 2]);
                            acc[p + 3] = fma(take[p + 3] ? c23 : 0.0, D[2], acc[p + 3]);
                        }
                    } else {
                        const double M2 = tile[k].M2, M1 = tile[k].M1, M0 = tile[k].M0, Bn = tile[k].Bn,
                                     Cn = tile[k].Cn;
#pragma unroll
                        for (int p = 0; p < kP; p += 4) {
                            double nn[4], mm[4];
#pragma unroll
                            for (int e = 0; e < 4; ++e) gh3_nm(nuj[p + e] - nu0, M2, M1, M0, Bn, Cn, nn[e], mm[e]);
                            const double P01 = mm[0] * mm[1], P23 = mm[2] * mm[3];
                            const double c = qrcp(P01 * P23) * Lg;
                            const double c01 = c * P23, c23 = c * P01;
                            const double x0 = c01 * mm[1], x1 = c01 * mm[0], x2 = c23 * mm[3], x3 = c23 * mm[2];
                            acc[p] = fma(take[p] ? x0 : 0.0, nn[0], acc[p]);
                            acc[p + 1] = fma(take[p + 1] ? x1 : 0.0, nn[1], acc[p + 1]);
                            acc[p + 2] = fma(take[p + 2] ? x2 : 0.0, nn[2], acc[p + 2]);
                            acc[p + 3] = fma(take[p + 3] ? x3 : 0.0, nn[3], acc[p + 3]);
                        }
                    }
                    ++k;
                } while (k < kend);
                continue;
            }
            if (path == kGH3Core) {
                do {
                    // the general path's sequences for these groups: a group
                    // without series points the 3-node path's, one with them a
                    // division per point, the series points adding zero
                    const uint32_t cb = (uint32_t)__builtin_amdgcn_readfirstlane((int)bnd[k].z);
                    const int32_t clo = bnd_lo(cb), chi = bnd_hi(cb);
                    const double nu0 = tile[k].nu0, Lg = tile[k].Lg;
                    const double M2 = tile[k].M2, M1 = tile[k].M1, M0 = tile[k].M0, Bn = tile[k].Bn, Cn = tile[k].Cn;
#pragma unroll
                    for (int p = 0; p < kP; p += 4) {
                        double nn[4], mm[4];
                        bool cp[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            gh3_nm(nuj[p + e] - nu0, M2, M1, M0, Bn, Cn, nn[e], mm[e]);
                            const int32_t jr = rel0 + lane + 64 * (p + e);
                            cp[e] = jr >= clo && jr <= chi;
                        }
                        if (!cp[0] && !cp[1] && !cp[2] && !cp[3]) {
                            const double P01 = mm[0] * mm[1], P23 = mm[2] * mm[3];
                            const double c = qrcp(P01 * P23) * Lg;
                            const double c01 = c * P23, c23 = c * P01;
                            acc[p] = fma(c01 * mm[1], nn[0], acc[p]);
                            acc[p + 1] = fma(c01 * mm[0], nn[1], acc[p + 1]);
                            acc[p + 2] = fma(c23 * mm[3], nn[2], acc[p + 2]);
                            acc[p + 3] = fma(c23 * mm[2], nn[3], acc[p + 3]);
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const double v = qdiv(Lg * nn[e], mm[e]);
                                acc[p + e] += cp[e] ? 0.0 : v;
                            }
                        }
                    }
                    ++k;
                } while (k < kend);
                continue;
            }
            do {
                const double nu0 = tile[k].nu0, Lg = tile[k].Lg, G2 = tile[k].G2;
                const double M2 = tile[k].M2, M1 = tile[k].M1, M0 = tile[k].M0, Bn = tile[k].Bn, Cn = tile[k].Cn;
                // general path: window edges (with edges == false), region edges,
                // core points (left to the core kernel), the grid end, lines
                // outside the grouping range (rare)
                const uint4 b4 = bnd[k];
                const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b4.x);
                const uint32_t b1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b4.y);
                const uint32_t b2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b4.z);
                const uint32_t b3 = (uint32_t)__builtin_amdgcn_readfirstlane((int)b4.w);
                const int32_t wlo = bnd_lo(b0), whi = bnd_hi(b0);
                const int32_t g3lo = bnd_lo(b1), g3hi = bnd_hi(b1);
                const int32_t clo = bnd_lo(b2), chi = bnd_hi(b2);
                const bool safe = (b3 & kGroupSafe) != 0;
#pragma unroll
                for (int p = 0; p < kP; p += 4) {
                    double num[4], den[4];
                    bool take[4], one[4], core_pt[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int32_t jr = rel0 + lane + 64 * (p + e);
                        const double dv = nuj[p + e] - nu0;
                        double n3, m3;
                        gh3_nm(dv, M2, M1, M0, Bn, Cn, n3, m3);
                        one[e] = jr < g3lo || jr > g3hi;
                        core_pt[e] = jr >= clo && jr <= chi;
                        take[e] = jr >= wlo && jr <= whi && !core_pt[e];
                        num[e] = one[e] ? 1.0 : n3;
                        den[e] = one[e] ? fma(dv, dv, G2) : m3;
                    }
                    if (safe && !core_pt[0] && !core_pt[1] && !core_pt[2] && !core_pt[3] &&
                        run0 + lane + 64 * (p + 3) < n) {
                        const double P01 = den[0] * den[1], P23 = den[2] * den[3];
                        const double c = qrcp(P01 * P23) * Lg;
                        const double c01 = c * P23, c23 = c * P01;
                        double xs[4], ys[4];
                        if (one[0] && one[1] && one[2] && one[3]) {
                            xs[0] = c01; ys[0] = den[1];
                            xs[1] = c01; ys[1] = den[0];
                            xs[2] = c23; ys[2] = den[3];
                            xs[3] = c23; ys[3] = den[2];
                        } else {
                            xs[0] = c01 * den[1]; ys[0] = num[0];
                            xs[1] = c01 * den[0]; ys[1] = num[1];
                            xs[2] = c23 * den[3]; ys[2] = num[2];
                            xs[3] = c23 * den[2]; ys[3] = num[3];
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[p + e] = fma(take[e] ? xs[e] : 0.0, ys[e], acc[p + e]);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const double v = qdiv(Lg * num[e], den[e]);
                            acc[p + e] += take[e] ? v : 0.0;
                        }
                    }
                }
                ++k;
            } while (k < kend);
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        const int32_t j = run0 + lane + 64 * p;
        if (j < n) out[j - obase] = accumulate ? out[j - obase] + acc[p] : acc[p];
    }
}

// One workgroup per work item (a grid tile of a state, or its lines in one
// segment), wp.launch_items of them (the plan's item count or its bound:
// workgroups past the last item exit at once; a loop over several items per
// workgroup measured slower, it costs registers).  Per-state arrays lie n_lines records, 2 n_tiles ranges
// and n points apart; a cut item writes its slot of partial (kTilePoints
// values).
template <int kP>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(kP == 4 ? 7 : 1))) void wing_f64_kernel(
    const WingRec* __restrict__ wing, const WingIdx* __restrict__ idx, const int64_t* __restrict__ ranges,
    int64_t n_lines, int64_t n_tiles, int32_t n_states, WorkPlan wp, double nu_min, double dnu, int32_t n,
    double* __restrict__ kappa, double* __restrict__ partial, int accumulate, int edges)
{
    constexpr int64_t kTilePoints = 64 * kP * kWaves;
    WorkItem it;
    if (work_item(xcd_rank(blockIdx.x), wp, ranges, n_tiles, n_states, it)) {
        const int64_t o = it.st * n_lines;
        const bool direct = it.slot < 0;
        double* out = direct ? kappa + it.st * (int64_t)n : partial + it.slot * kTilePoints;
        wing_f64_tile<kP>(it.tile, it.lo, it.hi, wing + o, idx + o, nu_min, dnu, n, out,
                          direct ? 0 : it.tile * kTilePoints, direct ? accumulate : 0, edges != 0);
    }
}

// The cut tiles: kappa_j (+)= the ordered sum of the tile's partials,
// segment by segment.  Workgroups stride over the (state, tile) pairs.
__global__ __launch_bounds__(256) void wing_f64_reduce_kernel(WorkPlan wp, int64_t n_tiles, int32_t n_states,
                                                             int32_t tp, int32_t n, const double* __restrict__ partial,
                                                             double* __restrict__ kappa, int accumulate)
{
    const int64_t total = wp.total[0];
    if (total == wp.n_pairs) return;  // nothing cut
    for (int64_t p = blockIdx.x; p < wp.n_pairs; p += gridDim.x) {
        const int64_t nseg = (p + 1 < wp.n_pairs ? wp.first[p + 1] : total) - wp.first[p];
        if (nseg < 2) continue;
        int64_t st, k;
        pair_decode(p, n_tiles, n_states, st, k);
        const int64_t j0 = (n_tiles - 1 - k) * tp;
        const double* src = partial + wp.slot[p] * tp;
        double* dst = kappa + st * (int64_t)n;
        for (int q = threadIdx.x; q < tp; q += blockDim.x) {
            const int64_t j = j0 + q;
            if (j >= n) break;
            double v = 0.0;
            for (int64_t sg = 0; sg < nseg; ++sg) v += src[sg * tp + q];
            dst[j] = accumulate ? dst[j] + v : v;
        }
    }
}

// H_V(a, u) for a^2 + u^2 < 100 by the series form of the Faddeeva function
// (Abramowitz & Stegun 7.1.29 applied to w(z) = e^{-z^2} erfc(-iz), step
// 1/2), the three exponential series summed in one loop (§2.4):
//   H = e^{-x^2} [erfcx(y) cos 2xy + sin(xy) (sin(xy)/y) / pi]
//     + (y/pi) [ -cos(2xy) e^{-x^2} T1 + (S2 + S3)/2 ],
// x = |u|, y = a, T1 = sum_n e^{-n^2/4}/(n^2/4+y^2) (per line), and
// S2 + S3 = sum_n (e^{-(n/2+x)^2} + e^{-(n/2-x)^2}) / (n^2/4 + y^2)
//         = 2 e^{-x^2} sum_n w_n cosh(n x),  w_n = e^{-n^2/4} / (n^2/4 + y^2),
// so that H = e^{-x^2} [erfcx(y) cos 2xy + sin^2(xy)/(pi y)
//                        + (y/pi) (sum_n w_n cosh(nx) - cos(2xy) T1)].
// cosh(nx) comes from a three-term recurrence in n (at most e^{340}/2,
// x < 10, n <= 34); w[n-1] is the line's table (same y for all its points),
// read from LDS.
// e^{-n^2/4}, n = 1 .. kMaxTerms
__constant__ double kGauss[kMaxTerms] = {
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
    4.1900931944943974e-32,
    6.6396771995807348e-36,
    6.3815034480607908e-40,
    3.7200759760208361e-44,
    1.3153258948574645e-48,
    2.8207700884601352e-53,
    3.6690596154291634e-58,
    2.8946403116483003e-63,
    1.3851193699226017e-68,
    4.0200602157433552e-74,
    7.0766981754295491e-80,
    7.5558190197119609e-86,
    4.8931122620973616e-92,
    1.9219477278238491e-98,
    4.5787899692915775e-105,
    6.6162610567094853e-112,
    5.7986554185640377e-119,
    3.0824406969490981e-126,
};

__device__ double voigt_core(double x, double y, double ex, double T1, const double* w)
{
    const double E = exp(-x * x);
    const double up = exp(x);
    const double c1 = up + qrcp(up);  // 2 cosh x
    // all kMaxTerms terms for every point (x < 10, so at least the
    // 2 ceil(x) + 14 terms the series needs; the rest are below 1e-20 of the
    // sum): a fixed trip count, the same for every lane.  2 cosh(n x) by the
    // three-term recurrence c_{n+1} = c_1 c_n - c_{n-1}, c_0 = 2, which
    // follows the growing solution e^{nx} stably (relative error ~n eps).
    // (w is read a pair of terms at a time, each pair one pair ahead of its
    // use, so that a read is in flight while the previous pair is summed;
    // the loop is unrolled twice, which saves the register moves of the
    // pairs' hand-over: binary64 step 7.30 -> 7.20 ms, the same box)
    static_assert(kMaxTerms % 4 == 2, "8 double pairs in the loop, one after it");
    const double2* w2 = reinterpret_cast<const double2*>(w);
    double cm = 2.0, cc = c1, sc = 0.0;
    auto term = [&](double wn) {
        sc = fma(wn, cc, sc);
        const double cn = fma(c1, cc, -cm);
        cm = cc;
        cc = cn;
    };
    double2 wa = w2[0];
#pragma unroll 2
    for (int h = 0; h < kMaxTerms / 2 - 1; h += 2) {
        const double2 wb = w2[h + 1];
        term(wa.x);
        term(wa.y);
        wa = w2[h + 2];
        term(wb.x);
        term(wb.y);
    }
    term(wa.x);
    term(wa.y);
    double s, co;
    sincos(x * y, &s, &co);
    const double cos2 = (co - s) * (co + s);
    const double sy = (y > 0.0) ? qdiv(s, y) : x;
    return E * (fma(ex, cos2, s * sy * kInvPi) + (y * kInvPi) * fma(-cos2, T1, 0.5 * sc));
}

// Core-region contributions.  Each wavefront owns a run of kCoreRun
// consecutive points and walks, in line order, the lines whose a^2+u^2 < 100
// points meet its run; a line's such points form one interval (a piece).
// Pieces are packed into 64-lane chunks: the lines are examined kCoreBatch
// at a time, their pieces' points laid end to end, and each chunk takes the
// next 64 of them (at most kChunkPieces pieces per chunk), so lanes stay
// full when pieces are short.  A lane evaluates the series for its point and
// adds it to the run's sums in LDS; lanes of one chunk that share a point
// (two lines covering it) add in line order, piece by piece.  So each point
// still sums its lines in ascending (nu, index) order, with the same values:
// the result does not depend on how pieces fall into chunks.
// Lines [L0, L1) of tile t; direct: series_j = the run's sum (every point,
// 0 where no line reaches); else every point's sum to partial[j - obase].
// The series has a grid of its own, added to the wing's afterwards (the two
// kernels can then run at the same time).
constexpr int kCoreRun = 256;                        // points per wavefront
constexpr int kCoreTilePoints = kCoreRun * kWaves;   // points per work item
constexpr int kCoreBatch = 32;                       // lines examined at once
constexpr int kChunkPieces = 16;                     // pieces per 64-lane chunk

struct alignas(16) CorePiece {  // one line's series points within a run
    double nu0, invA, y, y2, ex, norm, T1;
    int32_t a;      // its first grid point
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

__device__ __forceinline__ void core_f64_tile(int64_t t, int64_t L0, int64_t L1, const WingRec* __restrict__ wing,
                                              const WingIdx* __restrict__ idx, const CoreRec* __restrict__ core,
                                              double nu_min, double dnu, int32_t n, double* __restrict__ series,
                                              double* __restrict__ partial, int64_t obase, bool direct)
{
    __shared__ double acc_tab[kWaves][kCoreRun];
    __shared__ CorePiece piece_tab[kWaves][kCoreBatch];
    __shared__ __align__(16) double w_tab[kWaves][kChunkPieces * kMaxTerms];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    // lane nn < kMaxTerms builds term nn + 1 of each piece's table
    const double g_lane = kGauss[min(lane, kMaxTerms - 1)];
    const double m_lane = 0.5 * (double)(lane + 1);
    const int32_t run0 = (int32_t)(t * kCoreTilePoints) + wave * kCoreRun;
    const int32_t run1 = min(run0 + kCoreRun, n) - 1;
    if (run0 > run1) return;
    double* acc = acc_tab[wave];
    CorePiece* pc = piece_tab[wave];
    double* wt = w_tab[wave];
    for (int q = lane; q < kCoreRun; q += 64) acc[q] = 0.0;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));

    for (int64_t base = L0; base < L1; base += kCoreBatch) {
        // lanes below kCoreBatch examine one line each
        const int64_t i = base + lane;
        int32_t a = 1, b = 0;
        if (lane < kCoreBatch && i < L1) {
            const WingIdx r = idx[i];
            a = max(max(r.clo, r.wlo), run0);
            b = min(min(r.chi, r.whi), run1);
        }
        const bool has = a <= b;
        const uint64_t m = __ballot(has);
        if (m == 0) continue;
        const int np = __builtin_popcountll(m);
        const int32_t cnt = has ? b - a + 1 : 0;
        const int32_t incl = wave_incl_scan(cnt, lane);
        const int32_t total = __shfl(incl, 63, 64);
        if (has) {
            const CoreRec cr = core[i];
            CorePiece pp;
            pp.nu0 = wing[i].nu0;
            pp.invA = cr.invA;
            pp.y = cr.y;
            pp.y2 = cr.y2;
            pp.ex = cr.ex;
            pp.norm = cr.norm;
            pp.T1 = cr.T1;
            pp.a = a;
            pp.start = incl - cnt;
            pc[__builtin_popcountll(m & below)] = pp;
        }
        __builtin_amdgcn_wave_barrier();
        // lane k holds piece k's start (pieces in line order, starts rising)
        const int32_t st_k = lane < np ? pc[lane].start : total;
        int s_lo = 0;  // the piece holding point f0 of the flattened list
        for (int32_t f0 = 0; f0 < total;) {
            // (s_lo, s_end: the same in every lane, kept in scalar registers)
            s_lo = __builtin_amdgcn_readfirstlane(s_lo);
            int s_end = __builtin_popcountll(__ballot(lane < np && st_k < f0 + 64));
            s_end = __builtin_amdgcn_readfirstlane(min(s_end, s_lo + kChunkPieces));
            const int32_t next_start = __builtin_amdgcn_readlane(st_k, min(s_end, 63));
            const int32_t f_end = s_end < np ? min(next_start, f0 + 64) : min(total, f0 + 64);
            // the 1 / (n^2/4 + y^2) e^{-n^2/4} tables of pieces s_lo .. s_end-1
            for (int k = s_lo; k < s_end; ++k) {
                const double y2 = pc[k].y2;
                if (lane < kMaxTerms) wt[(k - s_lo) * kMaxTerms + lane] = g_lane * qrcp(fma(m_lane, m_lane, y2));
            }
            __builtin_amdgcn_wave_barrier();
            // this lane's point f and its piece
            const int32_t f = f0 + lane;
            const bool act = f < f_end;
            int my = s_lo;
            for (int s = s_lo + 1; s < s_end; ++s) my = __builtin_amdgcn_readlane(st_k, s) <= f ? s : my;
            double v = 0.0;
            int32_t jr = 0;  // the point, relative to run0
            if (act) {
                const CorePiece& pp = pc[my];
                const int32_t j = pp.a + (f - pp.start);
                jr = j - run0;
                const double dv = fma((double)j, dnu, nu_min) - pp.nu0;
                v = pp.norm * voigt_core(fabs(dv) * pp.invA, pp.y, pp.ex, pp.T1, wt + (my - s_lo) * kMaxTerms);
            }
            // add in line order: one LDS add instruction per piece, whose
            // lanes hold distinct points; a wavefront's LDS operations are
            // carried out in the order they are issued, and the fence keeps
            // the compiler from merging or reordering the pieces' adds
            for (int s = s_lo; s < s_end; ++s) {
                if (act && my == s)
                    __hip_atomic_fetch_add(&acc[jr], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            }
            s_lo = (s_end < np && f_end >= next_start) ? s_end : s_end - 1;
            f0 = f_end;
        }
        __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();
    for (int q = lane; q < kCoreRun; q += 64) {
        const int32_t j = run0 + q;
        if (j <= run1) {
            if (direct)
                series[j] = acc[q];
            else
                partial[j - obase] = acc[q];
        }
    }
}

// One workgroup per work item of the series (the layout of wing_f64_kernel),
// taken in plan order: a series tile reads few lines, so dealing neighbouring
// tiles to one XCD does not pay here (measured: it costs ~5%).
__global__ __launch_bounds__(64 * kWaves) void core_f64_kernel(
    const WingRec* __restrict__ wing, const WingIdx* __restrict__ idx, const CoreRec* __restrict__ core,
    const int64_t* __restrict__ ranges, int64_t n_lines, int64_t n_tiles, int32_t n_states, WorkPlan wp,
    double nu_min, double dnu, int32_t n, double* __restrict__ series, double* __restrict__ partial)
{
    WorkItem it;
    if (work_item(blockIdx.x, wp, ranges, n_tiles, n_states, it)) {
        const int64_t o = it.st * n_lines;
        const bool direct = it.slot < 0;
        core_f64_tile(it.tile, it.lo, it.hi, wing + o, idx + o, core + o, nu_min, dnu, n,
                      series + it.st * (int64_t)n, partial + (direct ? 0 : it.slot * kCoreTilePoints),
                      it.tile * kCoreTilePoints, direct);
    }
}

// Cut series tiles: series_j = the ordered sum of the tile's partials.
__global__ __launch_bounds__(256) void core_f64_reduce_kernel(WorkPlan wp, int64_t n_tiles, int32_t n_states,
                                                             int32_t tp, int32_t n, const double* __restrict__ partial,
                                                             double* __restrict__ series)
{
    const int64_t total = wp.total[0];
    if (total == wp.n_pairs) return;  // nothing cut
    for (int64_t p = blockIdx.x; p < wp.n_pairs; p += gridDim.x) {
        const int64_t nseg = (p + 1 < wp.n_pairs ? wp.first[p + 1] : total) - wp.first[p];
        if (nseg < 2) continue;
        int64_t st, k;
        pair_decode(p, n_tiles, n_states, st, k);
        const int64_t j0 = (n_tiles - 1 - k) * tp;
        const double* src = partial + wp.slot[p] * tp;
        double* dst = series + st * (int64_t)n;
        for (int q = threadIdx.x; q < tp; q += blockDim.x) {
            const int64_t j = j0 + q;
            if (j >= n) break;
            double v = 0.0;
            for (int64_t sg = 0; sg < nseg; ++sg) v += src[sg * tp + q];
            dst[j] = v;
        }
    }
}

template <int kP>
hipError_t launch_wing(const WingRec* wing, const WingIdx* idx, const int64_t* ranges, int64_t n_lines,
                       int64_t n_tiles, int32_t n_states, const WorkPlan& wp, double nu_min, double dnu, int32_t n,
                       double* kappa, double* partial, int accumulate, int edges, hipStream_t s)
{
    const int64_t nb = plan_blocks(wp.launch_items);
    if (nb > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    wing_f64_kernel<kP><<<dim3((unsigned)nb), dim3(64 * kWaves), 0, s>>>(
        wing, idx, ranges, n_lines, n_tiles, n_states, wp, nu_min, dnu, n, kappa, partial, accumulate, edges);
    const int64_t nr = std::min<int64_t>(wp.n_pairs, 8192);
    wing_f64_reduce_kernel<<<dim3((unsigned)nr), dim3(256), 0, s>>>(wp, n_tiles, n_states, 64 * kP * kWaves, n,
                                                                    partial, kappa, accumulate);
    return hipGetLastError();
}



}  // namespace

int32_t opacity_f64_tile_points(int points_per_lane) { return 64 * points_per_lane * kWaves; }
int32_t core_f64_tile_points() { return kCoreTilePoints; }

hipError_t launch_wing_f64(int points_per_lane, const WingRec* wing, const WingIdx* idx, const int64_t* ranges,
                           int64_t n_lines, int64_t n_tiles, int32_t n_states, const WorkPlan& wp, double nu_min,
                           double dnu, int32_t n_points, double* kappa, double* partial, int accumulate, int edges,
                           hipStream_t s)
{
    if (n_tiles == 0 || n_states == 0) return hipSuccess;
    switch (points_per_lane) {
    case 4: return launch_wing<4>(wing, idx, ranges, n_lines, n_tiles, n_states, wp, nu_min, dnu, n_points, kappa,
                                  partial, accumulate, edges, s);
    case 8: return launch_wing<8>(wing, idx, ranges, n_lines, n_tiles, n_states, wp, nu_min, dnu, n_points, kappa,
                                  partial, accumulate, edges, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_core_f64(const WingRec* wing, const WingIdx* idx, const CoreRec* core, const int64_t* ranges,
                           int64_t n_lines, int64_t n_tiles, int32_t n_states, const WorkPlan& wp, double nu_min,
                           double dnu, int32_t n_points, double* series, double* partial, hipStream_t s)
{
    if (n_tiles == 0 || n_states == 0) return hipSuccess;
    const int64_t nb = plan_blocks(wp.launch_items);
    if (nb > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    core_f64_kernel<<<dim3((unsigned)nb), dim3(64 * kWaves), 0, s>>>(wing, idx, core, ranges, n_lines, n_tiles,
                                                                    n_states, wp, nu_min, dnu, n_points, series,
                                                                    partial);
    const int64_t nr = std::min<int64_t>(wp.n_pairs, 8192);
    core_f64_reduce_kernel<<<dim3((unsigned)nr), dim3(256), 0, s>>>(wp, n_tiles, n_states, core_f64_tile_points(),
                                                                    n_points, partial, series);
    return hipGetLastError();
}

namespace {

__global__ __launch_bounds__(256) void add_f64_kernel(double* __restrict__ a, const double* __restrict__ b, int64_t n)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) a[j] += b[j];
}

}  // namespace

hipError_t launch_add_f64(double* a, const double* b, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if ((n + 255) / 256 > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    add_f64_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(a, b, n);
    return hipGetLastError();
}

}  // namespace hk
