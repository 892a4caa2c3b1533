// work_plan.hip -- the work items of the wing kernels (the scheme is stated
// beside WorkPlan in hk_internal.h): the segment length of each state, then
// each (state, tile) pair's segment count and the exclusive prefix sums that
// number the items and the partial slots, in three passes (block sums, one
// scan of the block sums, offsets).
#include <algorithm>

#include "hk_internal.h"

namespace hk {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int64_t kPerBlock = (int64_t)kThreads * kPerThread;
// A state's tiles are cut when fewer than kBusyMin reference tiles hold
// lines, or when the fullest holds more than kUneven times the mean.
constexpr int64_t kBusyMin = 4096;
constexpr int64_t kUneven = 3;

// One workgroup per state.  Segment length: the smallest power of two >=
// min_seg and >= W / (4 n_points), W = 512 sum_t c_t + 4096 n_lines (c_t:
// lines of reference tile t).  W bounds the sum over any tiles of <= 2048
// points of (lines in the tile's range) x (tile points): a line's reach
// covers |A| grid points, which lie in >= |A| / 512 reference tiles and meet
// <= |A| / tp + 2 tiles of tp points.  So the items stay <= sum_t (c_t / L
// + 2) <= 6 n_tiles and the partial points <= 6 n_points + 2 tile points.
__global__ __launch_bounds__(kThreads) void seg_length_kernel(const int64_t* __restrict__ ref, int64_t n_ref,
                                                              int64_t n_points, int64_t n_lines, int64_t min_seg,
                                                              int64_t* __restrict__ seg)
{
    __shared__ int64_t red[3][kThreads];
    const int64_t* rg = ref + (int64_t)blockIdx.x * 2 * n_ref;
    int64_t busy = 0, mx = 0, sum = 0;
    for (int64_t t = threadIdx.x; t < n_ref; t += kThreads) {
        const int64_t c = rg[2 * t + 1] - rg[2 * t];
        busy += c > 0;
        mx = max(mx, c);
        sum += c;
    }
    red[0][threadIdx.x] = busy;
    red[1][threadIdx.x] = mx;
    red[2][threadIdx.x] = sum;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] = max(red[1][threadIdx.x], red[1][threadIdx.x + h]);
            red[2][threadIdx.x] += red[2][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        busy = red[0][0];
        mx = red[1][0];
        sum = red[2][0];
        int64_t L = kNoSplit;
        if (sum > 0 && (busy < kBusyMin || mx * busy > kUneven * sum)) {
            const double W = 512.0 * (double)sum + 4096.0 * (double)n_lines;
            const double need = W / (4.0 * (double)n_points);
            L = min_seg;
            while ((double)L < need && L < kNoSplit) L <<= 1;  // kNoSplit: not cut after all
        }
        seg[blockIdx.x] = L;
    }
}

__device__ inline void pair_counts(int64_t p, int64_t n_pairs, const int64_t* __restrict__ ranges,
                                   int64_t n_tiles, int32_t n_states, const int64_t* __restrict__ seg,
                                   int64_t& items, int64_t& slots)
{
    items = 0;
    slots = 0;
    if (p >= n_pairs) return;
    int64_t st, k;
    pair_decode(p, n_tiles, n_states, st, k);
    const int64_t t = n_tiles - 1 - k;
    const int64_t* rg = ranges + st * 2 * n_tiles;
    const int64_t lo = rg[2 * t], hi = rg[2 * t + 1];
    const int64_t L = seg[st];
    items = hi > lo ? (hi - 1) / L - lo / L + 1 : 1;
    slots = items > 1 ? items : 0;
}

// Exclusive scan of (a, b) over the workgroup; returns the totals.
__device__ inline void block_scan(int64_t& a, int64_t& b, int64_t& ta, int64_t& tb)
{
    __shared__ int64_t sa[kThreads], sb[kThreads];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int o = 1; o < kThreads; o <<= 1) {
        const int64_t va = (int)threadIdx.x >= o ? sa[threadIdx.x - o] : 0;
        const int64_t vb = (int)threadIdx.x >= o ? sb[threadIdx.x - o] : 0;
        __syncthreads();
        sa[threadIdx.x] += va;
        sb[threadIdx.x] += vb;
        __syncthreads();
    }
    ta = sa[kThreads - 1];
    tb = sb[kThreads - 1];
    a = sa[threadIdx.x] - a;
    b = sb[threadIdx.x] - b;
    __syncthreads();
}

// Pass 1: per-pair counts, block-local exclusive prefixes, block totals.
__global__ __launch_bounds__(kThreads) void plan_count_kernel(const int64_t* __restrict__ ranges, int64_t n_tiles,
                                                              int32_t n_states, const int64_t* __restrict__ seg,
                                                              int64_t n_pairs, int64_t* __restrict__ first,
                                                              int64_t* __restrict__ slot,
                                                              int64_t* __restrict__ bsum)
{
    const int64_t p0 = (int64_t)blockIdx.x * kPerBlock + (int64_t)threadIdx.x * kPerThread;
    int64_t it[kPerThread], sl[kPerThread];
    int64_t a = 0, b = 0;
    for (int i = 0; i < kPerThread; ++i) {
        pair_counts(p0 + i, n_pairs, ranges, n_tiles, n_states, seg, it[i], sl[i]);
        a += it[i];
        b += sl[i];
    }
    int64_t ta, tb;
    block_scan(a, b, ta, tb);
    for (int i = 0; i < kPerThread; ++i) {
        if (p0 + i < n_pairs) {
            first[p0 + i] = a;
            slot[p0 + i] = b;
        }
        a += it[i];
        b += sl[i];
    }
    if (threadIdx.x == 0) {
        bsum[2 * blockIdx.x] = ta;
        bsum[2 * blockIdx.x + 1] = tb;
    }
}

// Pass 2 (one workgroup): exclusive scan of the block totals in place, and
// the grand totals.
__global__ __launch_bounds__(kThreads) void plan_scan_kernel(int64_t* __restrict__ bsum, int64_t n_blocks,
                                                             int64_t* __restrict__ total)
{
    int64_t ra = 0, rb = 0;  // running totals of earlier rounds
    for (int64_t base = 0; base < n_blocks; base += kThreads) {
        const int64_t i = base + threadIdx.x;
        int64_t a = i < n_blocks ? bsum[2 * i] : 0;
        int64_t b = i < n_blocks ? bsum[2 * i + 1] : 0;
        int64_t ta, tb;
        block_scan(a, b, ta, tb);
        if (i < n_blocks) {
            bsum[2 * i] = ra + a;
            bsum[2 * i + 1] = rb + b;
        }
        ra += ta;
        rb += tb;
    }
    if (threadIdx.x == 0) {
        total[0] = ra;
        total[1] = rb;
    }
}

// Pass 3: add each block's offset.
__global__ __launch_bounds__(kThreads) void plan_offset_kernel(int64_t n_pairs, const int64_t* __restrict__ bsum,
                                                               int64_t* __restrict__ first,
                                                               int64_t* __restrict__ slot)
{
    const int64_t oa = bsum[2 * blockIdx.x], ob = bsum[2 * blockIdx.x + 1];
    const int64_t p0 = (int64_t)blockIdx.x * kPerBlock;
    for (int64_t i = threadIdx.x; i < kPerBlock; i += kThreads) {
        const int64_t p = p0 + i;
        if (p < n_pairs) {
            first[p] += oa;
            slot[p] += ob;
        }
    }
}

}  // namespace

int64_t plan_scratch_count(int64_t n_pairs) { return 2 * std::max<int64_t>(1, (n_pairs + kPerBlock - 1) / kPerBlock); }

hipError_t launch_seg_length(const int64_t* ref_ranges, int64_t n_ref, int32_t n_states, int64_t n_points,
                             int64_t n_lines, int64_t min_seg, int64_t* seg, hipStream_t s)
{
    if (n_states <= 0) return hipSuccess;
    if (min_seg < 1 || (min_seg & (min_seg - 1)) != 0) return hipErrorInvalidValue;
    seg_length_kernel<<<dim3((unsigned)n_states), dim3(kThreads), 0, s>>>(ref_ranges, n_ref, n_points, n_lines,
                                                                         min_seg, seg);
    return hipGetLastError();
}

hipError_t launch_work_plan(const int64_t* ranges, int64_t n_tiles, int32_t n_states, const int64_t* seg,
                            int64_t* first, int64_t* slot, int64_t* block_sums, int64_t* total, hipStream_t s)
{
    const int64_t n_pairs = n_tiles * (int64_t)n_states;
    const int64_t nb = std::max<int64_t>(1, (n_pairs + kPerBlock - 1) / kPerBlock);
    plan_count_kernel<<<dim3((unsigned)nb), dim3(kThreads), 0, s>>>(ranges, n_tiles, n_states, seg, n_pairs, first,
                                                                    slot, block_sums);
    plan_scan_kernel<<<dim3(1), dim3(kThreads), 0, s>>>(block_sums, nb, total);
    plan_offset_kernel<<<dim3((unsigned)nb), dim3(kThreads), 0, s>>>(n_pairs, block_sums, first, slot);
    return hipGetLastError();
}

}  // namespace hk
