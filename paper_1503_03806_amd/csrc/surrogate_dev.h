// surrogate_dev.h -- device code of the learned K(x, y) surrogate shared by
// its training/certification kernels and the opacity kernel that deploys it.
//
// Network: features f1 = x/25 - 1, f2 = (log10 y + 1)/3; four hidden layers
// of 64 SiLU units; one linear output z_hat.  K_hat = G3(x, y) exp(tau
// sinh(z_hat)), G3 the 3-node Gauss-Hermite value, tau = 1e-5.  Weights are
// bfloat16, sums binary32; the three 64x64 layers run on the matrix cores
// (v_mfma_f32_16x16x32_bf16), one wavefront per 64 samples.
#pragma once

#include "hk_internal.h"

namespace hk {
namespace surr {

constexpr int kHid = 64;
constexpr int kLd = kHid + 8;  // LDS row stride (bf16 elements) of a 64x64 tile
constexpr float kTau = 1e-5f;
// flat parameter vector: W1[64][2] b1 W2[64][64] b2 W3 b3 W4 b4 w5[64] b5
constexpr int kOffW1 = 0, kOffB1 = 128, kOffW2 = 192, kOffB2 = 4288, kOffW3 = 4352, kOffB3 = 8448,
              kOffW4 = 8512, kOffB4 = 12608, kOffW5 = 12672, kOffB5 = 12736, kNParams = 12737;
// certification cells over the series region: x in [0, 10), log10 y in [-4, 1)
constexpr int kCellsX = 80, kCellsY = 40;
constexpr float kCellW = 10.0f / kCellsX, kCellH = 5.0f / kCellsY;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Compute copy of the parameters (written after every update).
struct MlpBf16 {
    uint16_t W[3][kHid * kHid];   // W2..W4, [out][in]
    uint16_t WT[3][kHid * kHid];  // the same, [in][out]
    uint16_t W1[kHid * 2];
    uint16_t w5[kHid];
    float b[4][kHid];  // b1..b4
    float b5;
};

// binary32 -> bfloat16, round to nearest even (finite inputs)
__device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoid(z); }
__device__ inline float dsilu(float z)
{
    const float s = sigmoid(z);
    return s * fmaf(z, 1.0f - s, 1.0f);
}

__device__ inline bf16x8 ld8(const uint16_t* p)
{
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    return __builtin_bit_cast(bf16x8, v);
}

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline float feature_x(float x) { return x / 25.0f - 1.0f; }
__device__ inline float feature_y(float y) { return (log10f(y) + 1.0f) / 3.0f; }

// One 64x64 layer on the matrix cores: acc[m][n] = A[s][i] W[o][i]^T for the
// wavefront's 64 samples, A read from act ([s][kLd]), W from Wrow ([o][i]).
// Lane l holds acc[m][n][r] = Z[s = 16m + 4(l/16) + r][o = 16n + l%16].
__device__ __forceinline__ void layer_mfma(const uint16_t* act, const uint16_t* Wrow, floatx4 (&acc)[4][4])
{
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kq = 8 * (lane >> 4);
    bf16x8 a[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        a[m][0] = ld8(act + (16 * m + row) * kLd + kq);
        a[m][1] = ld8(act + (16 * m + row) * kLd + 32 + kq);
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const bf16x8 b0 = ld8(Wrow + (16 * n + row) * kHid + kq);
        const bf16x8 b1 = ld8(Wrow + (16 * n + row) * kHid + 32 + kq);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            floatx4 c = {0.0f, 0.0f, 0.0f, 0.0f};
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][0], b0, c, 0, 0, 0);
            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][1], b1, c, 0, 0, 0);
        }
    }
}

// Forward pass of one wavefront (lane = sample): returns z_hat.  act is the
// wavefront's [64][kLd] bfloat16 scratch.  With kTrain, also keeps the
// pre-activations Z[layer][s][o] (binary32) and the bfloat16 inputs of
// layers 2-5 transposed, inT[layer-2][i][s] (row stride kLd).
template <bool kTrain>
__device__ __forceinline__ float mlp_forward(const MlpBf16* __restrict__ P, uint16_t* act, float f1, float f2,
                             float* Z = nullptr, uint16_t* inT = nullptr)
{
    const int lane = threadIdx.x & 63;
    // layer 1 (2 -> 64) on the vector units, one sample per lane
#pragma unroll 1
    for (int o = 0; o < kHid; o += 8) {
        uint16_t hv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float z = fmaf(bf2f(P->W1[2 * (o + e)]), f1, fmaf(bf2f(P->W1[2 * (o + e) + 1]), f2, P->b[0][o + e]));
            hv[e] = f2bf(silu(z));
            if (kTrain) {
                Z[lane * kHid + o + e] = z;
                inT[(o + e) * kLd + lane] = hv[e];
            }
        }
        uint4 pk;
        pk.x = hv[0] | ((uint32_t)hv[1] << 16);
        pk.y = hv[2] | ((uint32_t)hv[3] << 16);
        pk.z = hv[4] | ((uint32_t)hv[5] << 16);
        pk.w = hv[6] | ((uint32_t)hv[7] << 16);
        *reinterpret_cast<uint4*>(act + lane * kLd + o) = pk;
    }
    wave_sync();
    // layers 2-4 (64 -> 64) on the matrix cores
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        floatx4 acc[4][4];
        layer_mfma(act, P->W[k], acc);
        wave_sync();  // every lane has read act
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int s = 16 * m + 4 * (lane >> 4) + r, o = 16 * n + (lane & 15);
                    const float z = acc[m][n][r] + P->b[k + 1][o];
                    const uint16_t h = f2bf(silu(z));
                    act[s * kLd + o] = h;
                    if (kTrain) {
                        Z[((k + 1) * kHid + s) * kHid + o] = z;
                        inT[((k + 1) * kHid + o) * kLd + s] = h;
                    }
                }
        wave_sync();
    }
    // output (64 -> 1): lane s dots its row with w5
    float out = P->b5;
#pragma unroll
    for (int o = 0; o < kHid; o += 8) {
        const uint4 v = *reinterpret_cast<const uint4*>(act + lane * kLd + o);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            out = fmaf(bf2f(P->w5[o + 2 * e]), __uint_as_float(w[e] << 16), out);
            out = fmaf(bf2f(P->w5[o + 2 * e + 1]), __uint_as_float(w[e] & 0xFFFF0000u), out);
        }
    }
    return out;
}

// K_hat from the network output: G3 exp(tau sinh(z_hat)), binary32.
__device__ inline float surrogate_K(float x, float y, float zhat)
{
    const float t1 = 1.2247448713915890f;             // sqrt(3/2)
    const float w0 = 1.1816359006036774f;             // 2 sqrt(pi) / 3
    const float w1 = 0.29540897515091934f;            // sqrt(pi) / 6
    const float y2 = y * y;
    const float dm = x - t1, dp = x + t1;
    const float g3 = (y * 0.31830988618379067f) *
                     (w0 * __builtin_amdgcn_rcpf(fmaf(x, x, y2)) + w1 * __builtin_amdgcn_rcpf(fmaf(dm, dm, y2)) +
                      w1 * __builtin_amdgcn_rcpf(fmaf(dp, dp, y2)));
    const float e = __expf(zhat);
    const float sh = 0.5f * (e - __builtin_amdgcn_rcpf(e));
    return g3 * __expf(kTau * sh);
}

// Whether (x, y) lies in a certified cell (mask: [kCellsY][kCellsX] bytes).
__device__ inline bool certified(const uint8_t* mask, float x, float y)
{
    if (!(y >= 1e-4f) || !(y < 10.0f) || !(x < 10.0f)) return false;
    const int ix = min((int)(x * (1.0f / kCellW)), kCellsX - 1);
    const int iy = min((int)((log10f(y) + 4.0f) * (1.0f / kCellH)), kCellsY - 1);
    return mask[iy * kCellsX + max(ix, 0)] != 0;
}

}  // namespace surr
}  // namespace hk
