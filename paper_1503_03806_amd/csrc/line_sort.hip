// line_sort.hip -- ordering and checking a line list on the device.
//
// The opacity kernels walk the lines in ascending (nu, input index) order
// (lines sorted by wavenumber, staged through LDS, §2.5).  A list handed over
// in device memory, or an unordered host list once copied, is put in that
// order here: a stable least-significant-digit radix sort of the keys' bit
// patterns (nu > 0, so the binary64 bits order like the values) carrying the
// input index, eight passes of 8-bit digits; then every field is gathered
// through the permutation.  Each pass: a per-tile digit histogram, an
// exclusive scan of the histograms (digit-major, so a digit's tiles follow
// each other), and a stable scatter in which each wavefront ranks its keys
// among equal digits with ballots (eight ballots give each lane the mask of
// lanes holding its digit) and the workgroup's waves and rounds are chained
// through LDS counters in input order.  No global atomics.
//
// The same file holds the device-side check of a list's values (the rules of
// hk_load_lines) and the bounds the launches need (largest shift, widths).
#include <algorithm>
#include <utility>

#include "hk_internal.h"

namespace hk {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;  // keys per thread per tile
constexpr int64_t kSortTile = (int64_t)kSortThreads * kSortRounds;
constexpr int kDigits = 256;

__global__ __launch_bounds__(256) void line_keys_kernel(const double* __restrict__ nu, int64_t n,
                                                         uint64_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        keys[i] = (uint64_t)__double_as_longlong(nu[i]);
        vals[i] = (uint32_t)i;
    }
}

// hist[d * n_tiles + t] = keys of tile t whose digit (bits shift .. shift+7) is d
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint64_t* __restrict__ keys, int64_t n,
                                                                  int shift, int64_t n_tiles,
                                                                  uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[kDigits];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t t = blockIdx.x;
    const int64_t base = t * kSortTile;
#pragma unroll 4
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + t] = h[threadIdx.x];
}

// Exclusive scan of m counts in three launches: per-block sums, a scan of
// the block sums in one workgroup, then each block's scan plus its offset.
constexpr int kScanBlock = 1024;  // counts per scan block (256 threads x 4)

__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total)
{
    // 256 threads: inclusive scan in LDS (Hillis-Steele), then exclusive
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t a = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0u;
        __syncthreads();
        sh[threadIdx.x] += a;
        __syncthreads();
    }
    const uint32_t incl = sh[threadIdx.x];
    if (total) *total = sh[255];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void scan_sums_kernel(const uint32_t* __restrict__ a, int64_t m,
                                                        uint32_t* __restrict__ sums)
{
    __shared__ uint32_t sh[256];
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    uint32_t s = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b0 + threadIdx.x * 4 + k;
        if (i < m) s += a[i];
    }
    uint32_t tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void scan_top_kernel(uint32_t* __restrict__ sums, int64_t nb)
{
    __shared__ uint32_t sh[256];
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += 256) {
        const int64_t i = c0 + threadIdx.x;
        const uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, sh, &tot);
        if (i < nb) sums[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(256) void scan_apply_kernel(uint32_t* __restrict__ a, int64_t m,
                                                         const uint32_t* __restrict__ sums)
{
    __shared__ uint32_t sh[256];
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    uint32_t v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b0 + threadIdx.x * 4 + k;
        v[k] = i < m ? a[i] : 0u;
        s += v[k];
    }
    uint32_t run = block_excl_scan(s, sh, nullptr) + sums[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        const int64_t i = b0 + threadIdx.x * 4 + k;
        if (i < m) a[i] = run;
        run += v[k];
    }
}

// Stable scatter of one pass.  Tile t's keys go, in input order, to
// off[d * n_tiles + t] + (rank among the tile's earlier keys of digit d).
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t n, int shift, int64_t n_tiles,
    const uint32_t* __restrict__ off, uint64_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out)
{
    constexpr int kW = kSortThreads / 64;
    __shared__ uint32_t run[kDigits];        // keys of each digit placed so far in this tile
    __shared__ uint32_t wcnt[kW][kDigits];   // this round: keys of each digit per wavefront
    const int64_t t = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    run[threadIdx.x] = off[(int64_t)threadIdx.x * n_tiles + t];
    for (int w = 0; w < kW; ++w) wcnt[w][threadIdx.x] = 0u;
    __syncthreads();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));  // lanes below this one
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = t * kSortTile + (int64_t)r * kSortThreads + threadIdx.x;
        const bool valid = i < n;
        const uint64_t k = valid ? keys[i] : 0ull;
        const uint32_t v = valid ? vals[i] : 0u;
        const uint32_t d = (uint32_t)(k >> shift) & 0xffu;
        // lanes holding the same digit: the AND over the digit's bits of the
        // ballot of that bit (or of its complement)
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__builtin_popcountll(peers & below);
        // the lowest lane of each digit group records the group's size
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__builtin_popcountll(peers);
        __syncthreads();
        // digit threadIdx.x: the waves' starts, in wave order, after what
        // earlier rounds placed
        {
            uint32_t s = run[threadIdx.x];
            for (int w = 0; w < kW; ++w) {
                const uint32_t c = wcnt[w][threadIdx.x];
                wcnt[w][threadIdx.x] = s;  // now the wave's start for this digit
                s += c;
            }
            run[threadIdx.x] = s;
        }
        __syncthreads();
        const uint32_t pos = wcnt[wave][d] + rank;
        if (valid && pos < n) {  // pos < n always; the test keeps a wrong plan in bounds
            keys_out[pos] = k;
            vals_out[pos] = v;
        }
        __syncthreads();
        for (int w = 0; w < kW; ++w) wcnt[w][threadIdx.x] = 0u;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void gather_kernel(const double* __restrict__ src, const uint32_t* __restrict__ perm,
                                                     int64_t n, double* __restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = perm[i] < n ? src[perm[i]] : 0.0;  // perm is a permutation of 0 .. n-1
}

__global__ __launch_bounds__(256) void check_lines_kernel(LinesDev L, CheckPart* __restrict__ part)
{
    __shared__ CheckPart sh[256];
    CheckPart c;
    c.first_bad = L.n;
    c.first_unordered = L.n;
    c.max_abs_delta = 0.0;
    c.max_gamma_air = 0.0;
    c.max_gamma_self = 0.0;
    c.max_A21 = 0.0;
    c.min_n_air = __builtin_inf();
    c.max_n_air = -__builtin_inf();
    c.nu_max = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < L.n; i += (int64_t)gridDim.x * 256) {
        const double nu = L.nu[i], S = L.S_ref[i], E = L.E_lower[i], ga = L.gamma_air[i], na = L.n_air[i];
        const double gs = L.gamma_self ? L.gamma_self[i] : ga;
        const double de = L.delta ? L.delta[i] : 0.0;
        const double A = L.A21 ? L.A21[i] : 0.0;
        const bool bad = !isfinite(nu) || !(nu > 0.0) || !isfinite(S) || !(S >= 0.0) || !isfinite(E) ||
                         !isfinite(ga) || !(ga >= 0.0) || !isfinite(na) || !isfinite(gs) || !(gs >= 0.0) ||
                         !isfinite(de) || !isfinite(A) || !(A >= 0.0);
        if (i > 0 && nu < L.nu[i - 1]) c.first_unordered = min(c.first_unordered, i);
        if (bad) {
            c.first_bad = min(c.first_bad, i);
            continue;
        }
        c.max_abs_delta = fmax(c.max_abs_delta, fabs(de));
        c.max_gamma_air = fmax(c.max_gamma_air, ga);
        c.max_gamma_self = fmax(c.max_gamma_self, gs);
        c.max_A21 = fmax(c.max_A21, A);
        c.min_n_air = fmin(c.min_n_air, na);
        c.max_n_air = fmax(c.max_n_air, na);
        c.nu_max = fmax(c.nu_max, nu);
    }
    sh[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            CheckPart& a = sh[threadIdx.x];
            const CheckPart& b = sh[threadIdx.x + w];
            a.first_bad = min(a.first_bad, b.first_bad);
            a.first_unordered = min(a.first_unordered, b.first_unordered);
            a.max_abs_delta = fmax(a.max_abs_delta, b.max_abs_delta);
            a.max_gamma_air = fmax(a.max_gamma_air, b.max_gamma_air);
            a.max_gamma_self = fmax(a.max_gamma_self, b.max_gamma_self);
            a.max_A21 = fmax(a.max_A21, b.max_A21);
            a.min_n_air = fmin(a.min_n_air, b.min_n_air);
            a.max_n_air = fmax(a.max_n_air, b.max_n_air);
            a.nu_max = fmax(a.nu_max, b.nu_max);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

int64_t grid_blocks(int64_t n) { return std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 8192); }

}  // namespace

int64_t line_sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

size_t line_sort_scratch_bytes(int64_t n)
{
    const int64_t nt = std::max<int64_t>(line_sort_tiles(n), 1);
    const int64_t m = nt * kDigits;
    const int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    // keys and indices twice, the histograms, the scan's block sums
    return (size_t)n * (2 * sizeof(uint64_t) + 2 * sizeof(uint32_t)) + (size_t)m * sizeof(uint32_t) +
           (size_t)nb * sizeof(uint32_t) + 256;
}

hipError_t launch_line_order(const double* nu, int64_t n, void* scratch, const uint32_t** perm_out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (n > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    const int64_t nt = line_sort_tiles(n);
    const int64_t m = nt * kDigits;
    const int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    if (nt > (int64_t)UINT32_MAX || nb > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    char* p = static_cast<char*>(scratch);
    uint64_t* k0 = reinterpret_cast<uint64_t*>(p);
    uint64_t* k1 = k0 + n;
    uint32_t* v0 = reinterpret_cast<uint32_t*>(k1 + n);
    uint32_t* v1 = v0 + n;
    uint32_t* hist = v1 + n;
    uint32_t* sums = hist + m;
    line_keys_kernel<<<dim3((unsigned)grid_blocks(n)), dim3(256), 0, s>>>(nu, n, k0, v0);
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        radix_hist_kernel<<<dim3((unsigned)nt), dim3(kSortThreads), 0, s>>>(k0, n, shift, nt, hist);
        scan_sums_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(hist, m, sums);
        scan_top_kernel<<<dim3(1), dim3(256), 0, s>>>(sums, nb);
        scan_apply_kernel<<<dim3((unsigned)nb), dim3(256), 0, s>>>(hist, m, sums);
        radix_scatter_kernel<<<dim3((unsigned)nt), dim3(kSortThreads), 0, s>>>(k0, v0, n, shift, nt, hist, k1, v1);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    *perm_out = v0;  // eight passes: back in the first buffers
    return hipGetLastError();
}

hipError_t launch_gather(const double* src, const uint32_t* perm, int64_t n, double* dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    gather_kernel<<<dim3((unsigned)grid_blocks(n)), dim3(256), 0, s>>>(src, perm, n, dst);
    return hipGetLastError();
}

int32_t check_lines_blocks(int64_t n) { return (int32_t)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 1024); }

hipError_t launch_check_lines(const LinesDev& L, void* part, hipStream_t s)
{
    check_lines_kernel<<<dim3((unsigned)check_lines_blocks(L.n)), dim3(256), 0, s>>>(L, static_cast<CheckPart*>(part));
    return hipGetLastError();
}


}  // namespace hk
