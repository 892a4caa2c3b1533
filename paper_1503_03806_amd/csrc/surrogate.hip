// surrogate.hip -- training, evaluation and certification of the learned
// K(x, y) surrogate (not part of the paper's method; the series of §2.4
// stays its fallback and the measure of its error).
//
//  * labels: the plain method's K in binary64 (series for x^2+y^2 < 100,
//    3-node rule beyond, §2.4), turned into the target
//    z = asinh(ln(K/G3)/tau);
//  * training step: one wavefront per 64 samples runs the forward pass, the
//    mean-squared-error gradient and the backward pass (the 64x64 products
//    dW = dZ^T A and dA = dZ W on the matrix cores) and writes its partial
//    gradient; the update kernel sums the partials in a fixed order and
//    applies Adam (Kingma & Ba 2015), then rewrites the bfloat16 copies.
//    No atomics: the result does not depend on scheduling;
//  * certification: one workgroup per cell of (x, log10 y) compares the
//    surrogate at a 16x16 lattice of the cell's points (edges included) with
//    the binary64 series and returns the cell's largest relative error.
#include <cmath>

#include "surrogate_dev.h"

namespace hk {
namespace {

using namespace surr;

// The plain method's K(x, y) in binary64 (x >= 0, y > 0): series of the
// Faddeeva function with step 1/2 (A&S 7.1.29) for x^2+y^2 < 100, one exp
// per term; the 3-node rule up to 1e6; the 1-node rule beyond.
__device__ __forceinline__ double plain_K(double x, double y)
{
    const double r = x * x + y * y;
    const double kPiD = 3.14159265358979323846;
    if (r >= 100.0) {
        if (r >= 1.0e6) return (y / kPiD) * (1.7724538509055160 / r);
        const double t1 = 1.2247448713915890, w0 = 1.1816359006036774, w1 = 0.29540897515091934;
        return (y / kPiD) * (w0 / r + w1 / ((x - t1) * (x - t1) + y * y) + w1 / ((x + t1) * (x + t1) + y * y));
    }
    const int N = 2 * (int)ceil(x) + 14;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int n = 1; n <= N; ++n) {
        const double hn = 0.5 * n;
        const double den = hn * hn + y * y;
        s1 += exp(-(hn * hn + x * x)) / den;
        s2 += exp(-(hn + x) * (hn + x)) / den;
        s3 += exp(-(hn - x) * (hn - x)) / den;
    }
    const double ex2 = exp(-x * x);
    const double c2 = cos(2.0 * x * y);
    const double s = sin(x * y);
    return ex2 * erfcx(y) * c2 + (ex2 * s * s / y) / kPiD + (-y * c2 * s1 + 0.5 * y * (s2 + s3)) / kPiD;
}

__device__ double gh3_K(double x, double y)
{
    const double kPiD = 3.14159265358979323846;
    const double t1 = 1.2247448713915890, w0 = 1.1816359006036774, w1 = 0.29540897515091934;
    return (y / kPiD) * (w0 / (x * x + y * y) + w1 / ((x - t1) * (x - t1) + y * y) +
                         w1 / ((x + t1) * (x + t1) + y * y));
}

__global__ __launch_bounds__(256) void label_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                   int64_t n, float* __restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xd = fabs((double)x[i]), yd = (double)y[i];
    const double t = log(plain_K(xd, yd) / gh3_K(xd, yd));
    z[i] = (float)asinh(t / 1e-5);
}

// Parameters (binary32) -> the bfloat16 compute copy; thread per parameter.
__device__ void write_copy(const float* __restrict__ theta, int p, MlpBf16* __restrict__ P)
{
    const float v = theta[p];
    if (p < kOffB1) {
        P->W1[p] = f2bf(v);
    } else if (p < kOffW2) {
        P->b[0][p - kOffB1] = v;
    } else if (p < kOffW5) {
        const int q = p - kOffW2, k = q / (kHid * kHid + kHid), e = q % (kHid * kHid + kHid);
        if (e < kHid * kHid) {
            const int o = e / kHid, i = e % kHid;
            P->W[k][o * kHid + i] = f2bf(v);
            P->WT[k][i * kHid + o] = f2bf(v);
        } else {
            P->b[k + 1][e - kHid * kHid] = v;
        }
    } else if (p < kOffB5) {
        P->w5[p - kOffW5] = f2bf(v);
    } else {
        P->b5 = v;
    }
}

__global__ __launch_bounds__(256) void pack_kernel(const float* __restrict__ theta, MlpBf16* __restrict__ P)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParams) write_copy(theta, p, P);
}

// LDS of the training step (one wavefront per workgroup)
struct alignas(16) TrainLds {
    float Z[4][kHid][kHid];         // pre-activations of layers 1-4, [s][o]
    uint16_t inT[4][kHid][kLd];   // bfloat16 inputs of layers 2-5, [i][s]
    uint16_t act[kHid][kLd];      // forward scratch [s][i]
    uint16_t dz[kHid][kLd];       // bfloat16 dZ of the current layer, [s][o]
    uint16_t dzT[kHid][kLd];      // the same, [o][s]
    float f1[kHid], f2[kHid], dout[kHid];
};

// Forward, loss and backward of 64 samples; samples j = (base + 64 w + l)
// mod n for 64 w + l < batch (other lanes are padding with zero gradient).
// Loss: mean of w(z) (z_hat - z)^2 with w(z) = 1 / (1 + (z/wscale)^2), or
// w = 1 when wscale = 0.  part_grad[w][p]; part_loss[w] = the weighted sum.
__global__ __launch_bounds__(64) void train_kernel(const MlpBf16* __restrict__ P, const float* __restrict__ xs,
                                                   const float* __restrict__ ys, const float* __restrict__ zs,
                                                   int64_t n, int64_t base, int32_t batch, float wscale,
                                                   float* __restrict__ part_grad, float* __restrict__ part_loss)
{
    __shared__ __align__(16) TrainLds L;
    const int lane = threadIdx.x;
    const int64_t b = (int64_t)blockIdx.x * kHid + lane;
    const bool active = b < batch;
    const int64_t j = (base + b) % n;
    const float x = active ? fabsf(xs[j]) : 0.0f, y = active ? ys[j] : 1.0f;
    const float f1 = feature_x(x), f2 = feature_y(y);
    L.f1[lane] = f1;
    L.f2[lane] = f2;
    const float out = mlp_forward<true>(P, &L.act[0][0], f1, f2, &L.Z[0][0][0], &L.inT[0][0][0]);
    const float zt = active ? zs[j] : 0.0f;
    const float res = active ? out - zt : 0.0f;
    const float q = wscale > 0.0f ? zt / wscale : 0.0f;
    const float wgt = 1.0f / fmaf(q, q, 1.0f);
    const float dout = 2.0f * wgt * res / (float)batch;
    L.dout[lane] = dout;
    float* G = part_grad + (int64_t)blockIdx.x * kNParams;
    // loss
    float sq = wgt * res * res;
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
    if (lane == 0) part_loss[blockIdx.x] = sq;
    float db5 = dout;
    for (int o = 32; o > 0; o >>= 1) db5 += __shfl_xor(db5, o, 64);
    wave_sync();
    // output layer: dw5[o] = sum_s dout[s] in5[s][o] (lane o), db5
    {
        float g = 0.0f;
        for (int s = 0; s < kHid; ++s) g = fmaf(L.dout[s], bf2f(L.inT[3][lane][s]), g);
        G[kOffW5 + lane] = g;
        if (lane == 0) G[kOffB5] = db5;
    }
    // dH4 in the product layout: dH[s][o] = dout[s] w5[o]
    floatx4 dh[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int nn = 0; nn < 4; ++nn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = 16 * m + 4 * (lane >> 4) + r, o = 16 * nn + (lane & 15);
                dh[m][nn][r] = L.dout[s] * bf2f(P->w5[o]);
            }
    const int row = lane & 15, kq = 8 * (lane >> 4);
    for (int k = 3; k >= 1; --k) {  // layers 4, 3, 2 (weights P->W[k-1])
        // dZ = dH * SiLU'(Z); bias gradient; bfloat16 dZ in both layouts
        float bsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int nn = 0; nn < 4; ++nn)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int s = 16 * m + 4 * (lane >> 4) + r, o = 16 * nn + (lane & 15);
                    const float dz = dh[m][nn][r] * dsilu(L.Z[k][s][o]);
                    bsum[nn] += dz;
                    const uint16_t h = f2bf(dz);
                    L.dz[s][o] = h;
                    L.dzT[o][s] = h;
                }
#pragma unroll
        for (int nn = 0; nn < 4; ++nn) {
            float v = bsum[nn];
            v += __shfl_xor(v, 16, 64);
            v += __shfl_xor(v, 32, 64);
            if (lane < 16) G[kOffB2 + (k - 1) * (kHid * kHid + kHid) + 16 * nn + lane] = v;
        }
        wave_sync();
        // dW[o][i] = sum_s dZ[s][o] in[s][i]:  A = dZ^T (rows o), B = in^T rows i
        {
            const uint16_t* inT = &L.inT[k - 1][0][0];
            bf16x8 a[4][2], bb[4][2];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                a[m][0] = ld8(&L.dzT[16 * m + row][kq]);
                a[m][1] = ld8(&L.dzT[16 * m + row][32 + kq]);
                bb[m][0] = ld8(inT + (16 * m + row) * kLd + kq);
                bb[m][1] = ld8(inT + (16 * m + row) * kLd + 32 + kq);
            }
            float* GW = G + kOffW2 + (k - 1) * (kHid * kHid + kHid);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int nn = 0; nn < 4; ++nn) {
                    floatx4 c = {0.0f, 0.0f, 0.0f, 0.0f};
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][0], bb[nn][0], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][1], bb[nn][1], c, 0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        GW[(16 * m + 4 * (lane >> 4) + r) * kHid + 16 * nn + (lane & 15)] = c[r];
                }
        }
        // dH_prev[s][i] = sum_o dZ[s][o] W[o][i]:  A = dZ (rows s), B = W^T rows i
        {
            bf16x8 a[4][2];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                a[m][0] = ld8(&L.dz[16 * m + row][kq]);
                a[m][1] = ld8(&L.dz[16 * m + row][32 + kq]);
            }
            const uint16_t* WT = P->WT[k - 1];
#pragma unroll
            for (int nn = 0; nn < 4; ++nn) {
                const bf16x8 b0 = ld8(WT + (16 * nn + row) * kHid + kq);
                const bf16x8 b1 = ld8(WT + (16 * nn + row) * kHid + 32 + kq);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    floatx4 c = {0.0f, 0.0f, 0.0f, 0.0f};
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][0], b0, c, 0, 0, 0);
                    dh[m][nn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m][1], b1, c, 0, 0, 0);
                }
            }
        }
        wave_sync();  // dz / dzT are rewritten by the next layer
    }
    // layer 1: dZ1 = dH1 SiLU'(Z1), kept in place of Z1
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int nn = 0; nn < 4; ++nn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = 16 * m + 4 * (lane >> 4) + r, o = 16 * nn + (lane & 15);
                L.Z[0][s][o] = dh[m][nn][r] * dsilu(L.Z[0][s][o]);
            }
    wave_sync();
    {
        float g0 = 0.0f, g1 = 0.0f, gb = 0.0f;
        for (int s = 0; s < kHid; ++s) {
            const float dz = L.Z[0][s][lane];
            g0 = fmaf(dz, L.f1[s], g0);
            g1 = fmaf(dz, L.f2[s], g1);
            gb += dz;
        }
        G[kOffW1 + 2 * lane] = g0;
        G[kOffW1 + 2 * lane + 1] = g1;
        G[kOffB1 + lane] = gb;
    }
}

// Sum of the per-workgroup partials in workgroup order; thread per parameter.
__device__ inline float sum_partials(const float* __restrict__ part, int32_t n_wg, int p)
{
    float g = 0.0f;
    for (int w = 0; w < n_wg; ++w) g += part[(int64_t)w * kNParams + p];
    return g;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ theta, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ part,
                                                   int32_t n_wg, float lr, float beta1, float beta2, float eps,
                                                   float c1, float c2, MlpBf16* __restrict__ P,
                                                   const float* __restrict__ part_loss, int32_t batch,
                                                   float* __restrict__ loss_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss_out) {
        float s = 0.0f;
        for (int w = 0; w < n_wg; ++w) s += part_loss[w];
        *loss_out = s / (float)batch;
    }
    if (p >= kNParams) return;
    const float g = sum_partials(part, n_wg, p);
    const float mm = beta1 * m[p] + (1.0f - beta1) * g;
    const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    theta[p] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    write_copy(theta, p, P);
}

__global__ __launch_bounds__(256) void reduce_kernel(const float* __restrict__ part, int32_t n_wg,
                                                     float* __restrict__ grad, const float* __restrict__ part_loss,
                                                     int32_t batch, float* __restrict__ loss_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss_out) {
        float s = 0.0f;
        for (int w = 0; w < n_wg; ++w) s += part_loss[w];
        *loss_out = s / (float)batch;
    }
    if (p < kNParams) grad[p] = sum_partials(part, n_wg, p);
}

// Network output and K_hat at given points; four wavefronts of 64 samples.
__global__ __launch_bounds__(256) void eval_kernel(const MlpBf16* __restrict__ P, const float* __restrict__ xs,
                                                   const float* __restrict__ ys, int64_t n,
                                                   float* __restrict__ z_out, float* __restrict__ K_out)
{
    __shared__ __align__(16) uint16_t act[4][kHid * kLd];
    const int wave = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const float x = i < n ? fabsf(xs[i]) : 0.0f, y = i < n ? ys[i] : 1.0f;
    const float z = mlp_forward<false>(P, act[wave], feature_x(x), feature_y(y));
    if (i < n) {
        z_out[i] = z;
        if (K_out) K_out[i] = surrogate_K(x, y, z);
    }
}

// One workgroup per cell c = iy * kCellsX + ix, sampling its 16x16 lattice
// (edges included): thread t takes (i, j) = (t % 16, t / 16),
// x = (ix + i/15) w, log10 y = -4 + (iy + j/15) h; err[c] = the largest
// relative error of K_hat against the binary64 series.  A dense-sampling
// check, not a bound: the network and the method are smooth on the cell's
// scale, and the deployed error is checked on whole bins against the oracle.
constexpr int kCertSide = 16;
__global__ __launch_bounds__(256) void certify_kernel(const MlpBf16* __restrict__ P, double* __restrict__ err)
{
    __shared__ __align__(16) uint16_t act[4][kHid * kLd];
    __shared__ double wmax[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int c = blockIdx.x;
    const int ix = c % kCellsX, iy = c / kCellsX;
    const int i = threadIdx.x % kCertSide, j = threadIdx.x / kCertSide;
    const float x = ((float)ix + (float)i / (float)(kCertSide - 1)) * kCellW;
    const float ly = -4.0f + ((float)iy + (float)j / (float)(kCertSide - 1)) * kCellH;
    const float y = exp10f(ly);
    const float z = mlp_forward<false>(P, act[wave], feature_x(x), feature_y(y));
    const double K = (double)surrogate_K(x, y, z);
    const double ref = plain_K((double)x, (double)y);
    double e = fabs(K / ref - 1.0);
    if (!(e == e)) e = 1e300;
    for (int o = 32; o > 0; o >>= 1) e = fmax(e, __shfl_xor(e, o, 64));
    if (lane == 0) wmax[wave] = e;
    __syncthreads();
    if (threadIdx.x == 0) err[c] = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
}
static_assert(kCertSide * kCertSide == 256, "one lattice point per thread");

}  // namespace

size_t surrogate_params_bytes() { return sizeof(MlpBf16); }
int32_t surrogate_n_params() { return kNParams; }
int32_t surrogate_cells() { return kCellsX * kCellsY; }

hipError_t launch_surrogate_labels(const float* x, const float* y, int64_t n, float* z, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    label_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(x, y, n, z);
    return hipGetLastError();
}

hipError_t launch_surrogate_pack(const float* theta, void* P, hipStream_t s)
{
    pack_kernel<<<dim3((kNParams + 255) / 256), dim3(256), 0, s>>>(theta, static_cast<MlpBf16*>(P));
    return hipGetLastError();
}

hipError_t launch_surrogate_train_step(const void* P, const float* x, const float* y, const float* z, int64_t n,
                                       int64_t base, int32_t batch, float wscale, float* part_grad,
                                       float* part_loss, hipStream_t s)
{
    const int n_wg = (batch + kHid - 1) / kHid;
    train_kernel<<<dim3(n_wg), dim3(64), 0, s>>>(static_cast<const MlpBf16*>(P), x, y, z, n, base, batch, wscale,
                                                 part_grad, part_loss);
    return hipGetLastError();
}

hipError_t launch_surrogate_adam(float* theta, float* m, float* v, const float* part_grad, int32_t batch,
                                 float lr, float beta1, float beta2, float eps, float c1, float c2, void* P,
                                 const float* part_loss, float* loss_out, hipStream_t s)
{
    const int n_wg = (batch + kHid - 1) / kHid;
    adam_kernel<<<dim3((kNParams + 255) / 256), dim3(256), 0, s>>>(theta, m, v, part_grad, n_wg, lr, beta1, beta2,
                                                                   eps, c1, c2, static_cast<MlpBf16*>(P),
                                                                   part_loss, batch, loss_out);
    return hipGetLastError();
}

hipError_t launch_surrogate_reduce(const float* part_grad, int32_t batch, float* grad, const float* part_loss,
                                   float* loss_out, hipStream_t s)
{
    const int n_wg = (batch + kHid - 1) / kHid;
    reduce_kernel<<<dim3((kNParams + 255) / 256), dim3(256), 0, s>>>(part_grad, n_wg, grad, part_loss, batch,
                                                                     loss_out);
    return hipGetLastError();
}

hipError_t launch_surrogate_eval(const void* P, const float* x, const float* y, int64_t n, float* z, float* K,
                                 hipStream_t s)
{
    if (n == 0) return hipSuccess;
    eval_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(static_cast<const MlpBf16*>(P), x, y, n, z,
                                                                        K);
    return hipGetLastError();
}

hipError_t launch_surrogate_certify(const void* P, double* err, hipStream_t s)
{
    certify_kernel<<<dim3(kCellsX * kCellsY), dim3(256), 0, s>>>(static_cast<const MlpBf16*>(P), err);
    return hipGetLastError();
}

}  // namespace hk
