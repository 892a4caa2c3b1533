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
// Per (wavefront, line) a uniform test against the line's precomputed index
// intervals picks one of three paths: all points in the 1-node region, all
// in the 3-node region, or the general path (window edges, region edges,
// core series).  Only the general path evaluates the series, per lane, for
// the points with a^2+u^2 < 100.
#include "hk_internal.h"

namespace hk {
namespace {

constexpr int kP = 4;       // grid points per lane
constexpr int kWaves = 4;   // wavefronts per workgroup
constexpr int kTL = 256;    // line records per LDS tile
constexpr int kTilePoints = 64 * kP * kWaves;

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so neighbouring tiles, which read mostly the same
// lines, share that XCD's L2.
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb)
{
    int64_t q = nb >> 3, r = nb & 7;
    int64_t x = b & 7, k = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// H_V(a, u) for a^2 + u^2 < 100 by the series form of the Faddeeva function
// (Abramowitz & Stegun 7.1.29 applied to w(z) = e^{-z^2} erfc(-iz), step
// 1/2), the three exponential series summed in one loop (§2.4).  x = |u|,
// y = a, ex = erfcx(y), T1 = sum_n e^{-n^2/4}/(n^2/4+y^2).  The Gaussians
// e^{-(n/2 -+ x)^2} come from two geometric-ratio recurrences instead of an
// exp() per term.
__device__ double voigt_core(double x, double y, double y2, double ex, double T1)
{
    const double c = 0.77880078307140486825;  // e^{-1/4}
    const double d = 0.60653065971263342360;  // e^{-1/2}
    const double E = exp(-x * x);
    const double up = exp(x);
    const double dn = 1.0 / up;
    double g3 = E * up * c;  // e^{-(1/2 - x)^2}
    double g2 = E * dn * c;  // e^{-(1/2 + x)^2}
    double r3 = up * (c * d);
    double r2 = dn * (c * d);
    const int N = 2 * (int)ceil(x) + 14;
    double s23 = 0.0;
    for (int n = 1; n <= N; ++n) {
        const double den = fma(0.25 * (double)n, (double)n, y2);
        s23 += (g2 + g3) / den;
        g3 *= r3;
        r3 *= d;
        g2 *= r2;
        r2 *= d;
    }
    double s, co;
    sincos(x * y, &s, &co);
    const double cos2 = (co - s) * (co + s);
    const double sy = (y > 0.0) ? s / y : x;
    return E * fma(ex, cos2, s * sy * kInvPi) + (y * kInvPi) * fma(-cos2 * E, T1, 0.5 * s23);
}

__global__ __launch_bounds__(64 * kWaves) void opacity_f64_kernel(
    const WingRec* __restrict__ wing, const CoreRec* __restrict__ core,
    const int64_t* __restrict__ ranges, int64_t n_tiles, double nu_min, double dnu, int32_t n,
    double* __restrict__ kappa, int accumulate)
{
    __shared__ WingRec tile[kTL];
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t run0 = (int32_t)(t * kTilePoints) + wave * 64 * kP;
    const int32_t run1 = min(run0 + 64 * kP, n) - 1;  // last point of the run (inclusive)
    const bool active = run0 < n;

    double nuj[kP], acc[kP];
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        const int32_t j = run0 + lane + 64 * p;
        nuj[p] = fma((double)j, dnu, nu_min);
        acc[p] = (accumulate && j < n) ? kappa[j] : 0.0;
    }

    const int64_t L0 = ranges[2 * t], L1 = ranges[2 * t + 1];
    for (int64_t base = L0; base < L1; base += kTL) {
        const int cnt = (int)min((int64_t)kTL, L1 - base);
        {
            const uint4* src = reinterpret_cast<const uint4*>(wing + base);
            uint4* dst = reinterpret_cast<uint4*>(tile);
            for (int k = threadIdx.x; k < cnt * 4; k += 64 * kWaves) dst[k] = src[k];
        }
        __syncthreads();
        if (active) {
            for (int k = 0; k < cnt; ++k) {
                const int32_t wlo = tile[k].wlo, whi = tile[k].whi;
                if (whi < run0 || wlo > run1) continue;
                const int32_t g3lo = tile[k].g3lo, g3hi = tile[k].g3hi;
                const int32_t clo = tile[k].clo, chi = tile[k].chi;
                const double nu0 = tile[k].nu0, Lg = tile[k].Lg, G2 = tile[k].G2;
                const bool full = wlo <= run0 && whi >= run1;
                const bool all1 = run1 < g3lo || run0 > g3hi;
                const bool nocore = run1 < clo || run0 > chi;
                if (full && all1) {
#pragma unroll
                    for (int p = 0; p < kP; ++p) {
                        const double dv = nuj[p] - nu0;
                        acc[p] += Lg / fma(dv, dv, G2);
                    }
                    continue;
                }
                const double h = tile[k].h, c6 = tile[k].c6;
                const double Lg3 = Lg * (1.0 / 3.0);
                if (full && nocore && g3lo <= run0 && g3hi >= run1) {
#pragma unroll
                    for (int p = 0; p < kP; ++p) {
                        const double dv = nuj[p] - nu0;
                        const double q = dv * dv;
                        const double D0 = q + G2;
                        const double E = D0 + h;
                        const double P = fma(E, E, -c6 * q);
                        acc[p] += (Lg3 * fma(D0, E, 2.0 * P)) / (D0 * P);
                    }
                    continue;
                }
                // general path
#pragma unroll
                for (int p = 0; p < kP; ++p) {
                    const int32_t j = run0 + lane + 64 * p;
                    const bool inw = j >= wlo && j <= whi;
                    const bool one = j < g3lo || j > g3hi;
                    const double dv = nuj[p] - nu0;
                    const double q = dv * dv;
                    const double D0 = q + G2;
                    const double E = D0 + h;
                    const double P = fma(E, E, -c6 * q);
                    const double num = one ? Lg : Lg3 * fma(D0, E, 2.0 * P);
                    const double den = one ? D0 : D0 * P;
                    double v = num / den;
                    if (!nocore) {
                        if (inw && j >= clo && j <= chi) {
                            const CoreRec& cr = core[base + k];
                            const double x = fabs(dv) * cr.invA;
                            v = cr.norm * voigt_core(x, cr.y, cr.y2, cr.ex, cr.T1);
                        }
                    }
                    acc[p] += inw ? v : 0.0;
                }
            }
        }
        __syncthreads();
    }
    if (active) {
#pragma unroll
        for (int p = 0; p < kP; ++p) {
            const int32_t j = run0 + lane + 64 * p;
            if (j < n) kappa[j] = acc[p];
        }
    }
}

}  // namespace

int32_t opacity_f64_tile_points() { return kTilePoints; }

hipError_t launch_opacity_f64(const WingRec* wing, const CoreRec* core, const int64_t* ranges,
                              int64_t n_tiles, double nu_min, double dnu, int32_t n_points,
                              double* kappa, int accumulate, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    opacity_f64_kernel<<<dim3((unsigned)n_tiles), dim3(64 * kWaves), 0, s>>>(
        wing, core, ranges, n_tiles, nu_min, dnu, n_points, kappa, accumulate);
    return hipGetLastError();
}

}  // namespace hk
