// kdist.hip -- the "Sort" stage (§2.2, §2.6): per-bin sort of the opacity
// grid, cumulative coordinate g_i = (i+1)/M, and k(g) at the requested g by
// the step or the midpoint-linear rule.
//
// The paper sorts the whole grid at once with bin tags (Thrust, §2.6).  Here
// bins are independent, and keys are the opacities' bit patterns
// (non-negative IEEE values order like their unsigned integer images).  A
// bin of up to kRadixMaxKeys keys is sorted by one workgroup in registers
// and LDS, by a radix sort whose ranking uses wavefront ballots (below); a
// larger bin is cut into LDS-sized chunks, each sorted in LDS by a bitonic
// network, then merged pairwise in global memory (each element finds its
// rank in the partner run by binary search; ties keep left-before-right, so
// the merge is stable).
#include "hk_internal.h"

namespace hk {
size_t radix_lds_bytes(int elem_bytes, int64_t keys);
namespace {

// threads per chunk-sort workgroup (measured on 300 bins of 1e4 binary64
// keys sorted this way: 0.177 ms, against 0.185 ms with 1024 threads and
// 0.188 ms with 256)
constexpr int kSortThreads = 512;

template <typename K>
struct KeyMax;
template <>
struct KeyMax<uint64_t> {
    static constexpr uint64_t v = ~0ull;
};
template <>
struct KeyMax<uint32_t> {
    static constexpr uint32_t v = ~0u;
};

template <typename K>
__device__ inline double key_value(K k);
template <>
__device__ inline double key_value<uint64_t>(uint64_t k)
{
    return __longlong_as_double((long long)k);
}
template <>
__device__ inline double key_value<uint32_t>(uint32_t k)
{
    return (double)__uint_as_float(k);
}

// Sort s[0 .. npad) ascending in LDS; npad is a power of two, all threads of
// the block take part.
// Each stage has npad/2 compare-exchange pairs (i, i + j), i with bit j
// clear; thread t takes pairs t, t + blockDim, ... so that every lane works.
template <typename K>
__device__ void bitonic_lds(K* s, int npad)
{
    const int half = npad >> 1;
    for (int k = 2; k <= npad; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int q = threadIdx.x; q < half; q += blockDim.x) {
                const int i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
                const int ixj = i + j;
                const K a = s[i], b = s[ixj];
                const bool up = (i & k) == 0;
                if ((a > b) == up) {
                    s[i] = b;
                    s[ixj] = a;
                }
            }
            __syncthreads();
        }
    }
}

// k(g) read off a bin's m sorted keys s[0 .. m).  Step rule: the smallest
// rank r whose g_r = (r+1)/m reaches g.  Midpoint-linear rule: key i sits at
// (i + 1/2)/m, straight lines between neighbours, the end keys held outside;
// no contraction, so the binary64 result is that of the expression as written.
template <typename K>
__device__ inline double k_of_g(const K* s, int64_t m, double g, int rule)
{
#pragma clang fp contract(off)
    if (rule == kRuleStep) {
        int64_t r = (int64_t)ceil(g * (double)m) - 1;
        r = r < 0 ? 0 : (r > m - 1 ? m - 1 : r);
        return key_value<K>(s[r]);
    }
    const double u = g * (double)m - 0.5;
    const double fl = floor(u);
    if (u <= 0.0) return key_value<K>(s[0]);
    if (fl >= (double)(m - 1)) return key_value<K>(s[m - 1]);
    const int64_t i = (int64_t)fl;  // 0 <= i <= m - 2
    const double a = key_value<K>(s[i]), b = key_value<K>(s[i + 1]);
    return a + (u - fl) * (b - a);
}

// LDS radix sort of one bin per workgroup (bins of up to kRadixMaxKeys keys):
// kRadixThreads threads hold the bin's keys in registers -- wavefront w
// holds positions [w R 64, (w+1) R 64), lane l of it key r at position
// w R 64 + r 64 + l (R keys per thread) -- and sort them least significant
// digit first, 8 bits per pass (binary32 keys: 4 passes; binary64 keys: the
// 4 passes of the high words and a finish, below).
// Each pass is stable: a wavefront ranks its keys round by round (so in
// position order) among equal digits with eight ballots (the lanes sharing a
// lane's digit are the AND over the digit's bits of each bit's ballot or its
// complement) and keeps a running count per digit in its own LDS counters,
// with no barrier between rounds; then the counters become offsets (waves in
// order, digits by a scan), every key is written to its place in LDS and read
// back in position order.  Four barriers per pass.
constexpr int kRadixThreads = 1024;
constexpr int kRadixWaves = kRadixThreads / 64;
constexpr int kRadixMaxRounds = 16;
constexpr int64_t kRadixMaxKeys = (int64_t)kRadixThreads * kRadixMaxRounds;
static_assert(kRadixMaxKeys <= (1 << 16), "LDS positions and counters fit 32 bits with room");

// The bin sorted into buf[0, m).  Binary32 keys: four passes.  Binary64
// keys: the four passes of their high words first; keys whose high words
// are equal (values within about 2^-20 of each other: few, in short runs)
// are then put in order by one thread per run, by insertion on the whole
// key.  Should a run be longer than kRunMax, the eight passes of the whole
// key follow instead.  Either way buf ends in ascending order of the keys.
constexpr int kRunMax = 32;

__device__ inline uint32_t key_hi(uint64_t k) { return (uint32_t)(k >> 32); }

template <typename K>
__device__ inline void radix_sort_block(K (&key)[kRadixMaxRounds], int rounds, int m, K* buf, uint32_t* cnt,
                                        uint32_t* wsum)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    lds_volatile<uint32_t>* wc = (lds_volatile<uint32_t>*)(cnt + wave * 256);  // this wavefront's counters
    uint32_t rank[kRadixMaxRounds];
    constexpr bool wide = sizeof(K) == 8;
    int n_pass = 4;
    for (int it = 0; it < n_pass; ++it) {
        // binary64: the high word's bytes, then (only after a long run) all
        // eight from the lowest
        const int shift = !wide ? 8 * it : (it < 4 ? 32 + 8 * it : 8 * (it - 4));
        for (int q = lane; q < 256; q += 64) wc[q] = 0u;
#pragma unroll
        for (int r = 0; r < kRadixMaxRounds; ++r) {
            if (r < rounds) {
                const bool valid = wave * 64 * rounds + r * 64 + lane < m;
                const uint32_t d = (uint32_t)(key[r] >> shift) & 0xffu;
                // peers: the lanes whose digit equals this lane's, as two
                // 32-bit halves; bit b of the digit takes each lane's mask
                // mb = 0 where the bit is set and all ones where it is not,
                // and keeps the lanes of the ballot (bit set) XOR mb
                const uint64_t vb = __ballot(valid);
                uint32_t plo = (uint32_t)vb, phi = (uint32_t)(vb >> 32);
                const uint32_t nd = ~d;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const uint32_t mb = (uint32_t)((int32_t)(nd << (31 - b)) >> 31);
                    const uint64_t bal = __ballot(mb == 0u);
                    plo &= (uint32_t)bal ^ mb;
                    phi &= (uint32_t)(bal >> 32) ^ mb;
                }
                const uint32_t rk = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
                const uint32_t old = wc[d];
                rank[r] = old + rk;
                if (valid && rk == 0) wc[d] = old + (uint32_t)(__builtin_popcount(plo) + __builtin_popcount(phi));
            }
        }
        __syncthreads();
        // digit t (threads 0 .. 255): the waves' starts in wave order, then
        // the digits' starts by an exclusive scan of their totals
        uint32_t tot = 0;
        uint32_t pre[kRadixWaves];  // digit t's count in the waves before each
        if (t < 256) {
#pragma unroll
            for (int w = 0; w < kRadixWaves; ++w) pre[w] = cnt[w * 256 + t];
#pragma unroll
            for (int w = 0; w < kRadixWaves; ++w) {
                const uint32_t c = pre[w];
                pre[w] = tot;
                tot += c;
            }
        }
        uint32_t incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (t < 256 && lane == 63) wsum[wave] = incl;
        __syncthreads();
        if (t < 256) {
            uint32_t base = incl - tot;
            for (int w = 0; w < wave; ++w) base += wsum[w];
#pragma unroll
            for (int w = 0; w < kRadixWaves; ++w) cnt[w * 256 + t] = base + pre[w];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRadixMaxRounds; ++r) {
            if (r < rounds && wave * 64 * rounds + r * 64 + lane < m) {
                const uint32_t d = (uint32_t)(key[r] >> shift) & 0xffu;
                const uint32_t pos = cnt[wave * 256 + d] + rank[r];
                if (pos < (uint32_t)m) buf[pos] = key[r];  // pos < m always
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRadixMaxRounds; ++r) {
            const int p = wave * 64 * rounds + r * 64 + lane;
            if (r < rounds && p < m) key[r] = buf[p];
        }
        if (wide && it == 3) {
            bool long_run = false;
            for (int p = t; p + kRunMax < m; p += kRadixThreads)
                long_run |= key_hi((uint64_t)buf[p]) == key_hi((uint64_t)buf[p + kRunMax]);
            // (also the barrier after every thread's read-back)
            if (__syncthreads_or(long_run)) n_pass = 12;
        }
    }
    if (!wide || n_pass > 4) return;
    // (a thread reads the high words next to its run while other threads
    // reorder theirs: within a run every key has the same high word, so what
    // it reads does not depend on their progress)
    for (int p = t; p < m; p += kRadixThreads) {
        const uint32_t h = key_hi((uint64_t)buf[p]);
        if ((p > 0 && key_hi((uint64_t)buf[p - 1]) == h) || p + 1 >= m || key_hi((uint64_t)buf[p + 1]) != h)
            continue;
        int q = p + 1;  // the run [p, q] of high word h: at most kRunMax keys
        while (q + 1 < m && key_hi((uint64_t)buf[q + 1]) == h) ++q;
        for (int i = p + 1; i <= q; ++i) {
            const K v = buf[i];
            int j = i - 1;
            while (j >= p && buf[j] > v) {
                buf[j + 1] = buf[j];
                --j;
            }
            buf[j + 1] = v;
        }
    }
    __syncthreads();
}

// One workgroup per bin: bins of ppb consecutive points of n_states grids
// of n_points each (grid s at s * n_points; a grid's last bin may be short).
// Sorted keys to dst (optional, same layout) and k(g) to k_out[bin][g.n].
template <typename K>
__global__ __launch_bounds__(kRadixThreads) void radix_bin_kernel(const K* __restrict__ src, int64_t n_points,
                                                                  int64_t ppb, int64_t bins_per_grid,
                                                                  K* __restrict__ dst, GValues g,
                                                                  double* __restrict__ k_out)
{
    extern __shared__ __align__(16) unsigned char radix_lds[];
    const int64_t bin = blockIdx.x;
    const int64_t st = bin / bins_per_grid, lb = bin - st * bins_per_grid;
    const int64_t b0 = st * n_points + lb * ppb;
    const int m = (int)min(ppb, n_points - lb * ppb);
    const int rounds = (m + kRadixThreads - 1) / kRadixThreads;
    K* buf = reinterpret_cast<K*>(radix_lds);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(radix_lds + (size_t)rounds * kRadixThreads * sizeof(K));
    uint32_t* wsum = cnt + kRadixWaves * 256;
    K key[kRadixMaxRounds];
    const int base_p = (int)(threadIdx.x >> 6) * 64 * rounds + (int)(threadIdx.x & 63);
#pragma unroll
    for (int r = 0; r < kRadixMaxRounds; ++r) {
        const int p = base_p + r * 64;
        key[r] = (r < rounds && p < m) ? src[b0 + p] : KeyMax<K>::v;
    }
    radix_sort_block<K>(key, rounds, m, buf, cnt, wsum);
    if (dst) {  // the sorted bin, from LDS (coalesced)
        for (int p = (int)threadIdx.x; p < m; p += kRadixThreads) dst[b0 + p] = buf[p];
    }
    // buf holds the bin in order after the last pass
    if ((int)threadIdx.x < g.n) k_out[bin * g.n + threadIdx.x] = k_of_g<K>(buf, m, g.g[threadIdx.x], g.rule);
}

// One workgroup per bin (bins <= chunk), or per chunk of a larger bin when
// `chunk < ppb`: sort in LDS; if `final`, also emit k(g) for the bin.
template <typename K>
__global__ __launch_bounds__(kSortThreads) void sort_chunk_lds_kernel(
    const K* __restrict__ src, int64_t n_points, int64_t ppb, int64_t chunk, int npad,
    int64_t chunks_per_bin, K* __restrict__ dst, GValues g, double* __restrict__ k_out, int final)
{
    extern __shared__ unsigned char lds_raw[];
    K* s = reinterpret_cast<K*>(lds_raw);
    const int64_t bin = blockIdx.x / chunks_per_bin;
    const int64_t c = blockIdx.x - bin * chunks_per_bin;
    const int64_t b0 = bin * ppb;
    const int64_t m_bin = min(ppb, n_points - b0);
    const int64_t j0 = b0 + c * chunk;
    const int64_t m = min(chunk, b0 + m_bin - j0);
    for (int i = threadIdx.x; i < npad; i += blockDim.x) s[i] = i < m ? src[j0 + i] : KeyMax<K>::v;
    __syncthreads();
    bitonic_lds(s, npad);
    if (dst) {
        for (int i = threadIdx.x; i < m; i += blockDim.x) dst[j0 + i] = s[i];
    }
    if (final && (int)threadIdx.x < g.n) {
        k_out[bin * g.n + threadIdx.x] = k_of_g<K>(s, m, g.g[threadIdx.x], g.rule);
    }
}

// One pass of pairwise merging of sorted runs of length `run` inside each
// bin.  One thread per element.
template <typename K>
__global__ __launch_bounds__(256) void merge_pass_kernel(const K* __restrict__ src,
                                                         K* __restrict__ dst, int64_t n_points,
                                                         int64_t ppb, int64_t run)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_points) return;
    const int64_t bin = e / ppb;
    const int64_t b0 = bin * ppb;
    const int64_t m = min(ppb, n_points - b0);
    const int64_t i = e - b0;
    const int64_t r = i / run;
    const int64_t pair0 = (r & ~(int64_t)1) * run;
    const int64_t own0 = r * run;
    const K key = src[e];
    int64_t p0, p1;
    if ((r & 1) == 0) {
        p0 = own0 + run;
        p1 = min(own0 + 2 * run, m);
    } else {
        p0 = own0 - run;
        p1 = own0;
    }
    int64_t lo = p0, hi = p1 > p0 ? p1 : p0;
    if ((r & 1) == 0) {  // left run: count partner keys < key
        while (lo < hi) {
            int64_t mid = lo + ((hi - lo) >> 1);
            if (src[b0 + mid] < key) lo = mid + 1;
            else hi = mid;
        }
    } else {  // right run: count partner keys <= key
        while (lo < hi) {
            int64_t mid = lo + ((hi - lo) >> 1);
            if (src[b0 + mid] <= key) lo = mid + 1;
            else hi = mid;
        }
    }
    const int64_t partner_rank = lo - p0;
    dst[b0 + pair0 + (i - own0) + partner_rank] = key;
}

template <typename K>
__global__ __launch_bounds__(64) void kdist_pick_kernel(const K* __restrict__ sorted,
                                                        int64_t n_points, int64_t ppb, GValues g,
                                                        double* __restrict__ k_out)
{
    const int64_t bin = blockIdx.x;
    const int64_t b0 = bin * ppb;
    const int64_t m = min(ppb, n_points - b0);
    if ((int)threadIdx.x < g.n)
        k_out[bin * g.n + threadIdx.x] = k_of_g<K>(sorted + b0, m, g.g[threadIdx.x], g.rule);
}

int pow2_at_least(int64_t m)
{
    int p = 1;
    while (p < m) p <<= 1;
    return p;
}

template <typename K>
hipError_t run_kdist(const K* kappa, int64_t n_points, int64_t ppb, const GValues& g,
                     double* k_out, K* sorted_out, K* scratch, int64_t lds_bytes, int64_t radix_keys,
                     int32_t n_states, hipStream_t s)
{
    const int64_t n_bins = (n_points + ppb - 1) / ppb;
    if (ppb <= radix_keys) {  // one LDS radix sort per bin, every grid in one launch
        const int rounds = (int)((ppb + kRadixThreads - 1) / kRadixThreads);
        const size_t shm = radix_lds_bytes(sizeof(K), rounds * kRadixThreads);
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&radix_bin_kernel<K>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        const int64_t nb = n_bins * n_states;
        if (nb > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
        radix_bin_kernel<K><<<dim3((unsigned)nb), dim3(kRadixThreads), shm, s>>>(kappa, n_points, ppb, n_bins,
                                                                                  sorted_out, g, k_out);
        return hipGetLastError();
    }
    if (n_states != 1) return hipErrorInvalidValue;  // bins above one LDS sort: one grid per call
    const int64_t cap = kdist_lds_max_points(sizeof(K), lds_bytes);
    if (ppb <= cap) {
        const int npad = pow2_at_least(ppb);
        const size_t shm = (size_t)npad * sizeof(K);
        hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void*>(&sort_chunk_lds_kernel<K>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        sort_chunk_lds_kernel<K><<<dim3((unsigned)n_bins), dim3(kSortThreads), shm, s>>>(
            kappa, n_points, ppb, ppb, npad, 1, sorted_out, g, k_out, 1);
        return hipGetLastError();
    }
    // chunked: sort chunks of `cap` points, then merge runs until one run
    // covers the bin.  Ping-pong between scratch halves; the last pass
    // lands in sorted_out when given.
    const int64_t chunk = cap;
    const int64_t cpb = (ppb + chunk - 1) / chunk;
    const int npad = pow2_at_least(chunk);
    const size_t shm = (size_t)npad * sizeof(K);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sort_chunk_lds_kernel<K>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    K* bufA = scratch;
    K* bufB = scratch + n_points;
    sort_chunk_lds_kernel<K><<<dim3((unsigned)(n_bins * cpb)), dim3(kSortThreads), shm, s>>>(
        kappa, n_points, ppb, chunk, npad, cpb, bufA, g, k_out, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    K* cur = bufA;
    K* nxt = bufB;
    int passes = 0;
    for (int64_t run = chunk; run < ppb; run *= 2) ++passes;
    int done = 0;
    for (int64_t run = chunk; run < ppb; run *= 2) {
        ++done;
        K* out = (done == passes && sorted_out) ? sorted_out : nxt;
        const int64_t blocks = (n_points + 255) / 256;
        merge_pass_kernel<K><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(cur, out, n_points, ppb, run);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        nxt = cur;
        cur = out;
    }
    kdist_pick_kernel<K><<<dim3((unsigned)n_bins), dim3(64), 0, s>>>(cur, n_points, ppb, g, k_out);
    return hipGetLastError();
}

}  // namespace

size_t radix_lds_bytes(int elem_bytes, int64_t keys)
{
    return (size_t)keys * elem_bytes + (size_t)kRadixWaves * 256 * 4 + 64;
}

int64_t kdist_radix_max_keys(int elem_bytes, int64_t lds_max)
{
    // whole rounds of kRadixThreads keys whose sort fits the workgroup's LDS
    int64_t r = kRadixMaxRounds;
    while (r > 0 && radix_lds_bytes(elem_bytes, r * kRadixThreads) > (size_t)lds_max) --r;
    return r * kRadixThreads;
}

int64_t kdist_lds_max_points(int elem_bytes, int64_t lds_bytes)
{
    // largest power of two whose keys fit in the workgroup's LDS
    int64_t p = 1;
    while (p * 2 * elem_bytes <= lds_bytes && p * 2 <= (1 << 16)) p *= 2;
    return p;
}

size_t kdist_scratch_bytes(int elem_bytes, int64_t n_points, int64_t ppb, int64_t lds_bytes, int64_t lds_max)
{
    if (ppb <= kdist_radix_max_keys(elem_bytes, lds_max) || ppb <= kdist_lds_max_points(elem_bytes, lds_bytes))
        return 0;
    return (size_t)2 * (size_t)n_points * (size_t)elem_bytes;
}

hipError_t launch_kdist(const void* kappa, int elem_bytes, int64_t n_points, int64_t ppb,
                        const GValues& g, double* k_out, void* sorted_out, void* scratch,
                        int64_t lds_bytes, int64_t lds_max, int32_t n_states, hipStream_t s)
{
    if (n_points == 0 || n_states == 0) return hipSuccess;
    const int64_t rk = kdist_radix_max_keys(elem_bytes, lds_max);
    if (elem_bytes == 8)
        return run_kdist<uint64_t>(static_cast<const uint64_t*>(kappa), n_points, ppb, g, k_out,
                                   static_cast<uint64_t*>(sorted_out),
                                   static_cast<uint64_t*>(scratch), lds_bytes, rk, n_states, s);
    return run_kdist<uint32_t>(static_cast<const uint32_t*>(kappa), n_points, ppb, g, k_out,
                               static_cast<uint32_t*>(sorted_out), static_cast<uint32_t*>(scratch),
                               lds_bytes, rk, n_states, s);
}

// The fixed sort scratch of hk_kdist_noalloc: one array per device, made
// when the code object is loaded and held until the process ends.  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is a host-side stand-in).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch_address(void** ptr)
{
    *ptr = nullptr;
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

}  // namespace hk
