// resample.hip -- the steps after the k-distribution (§2.6, eq. 5):
// least-squares Chebyshev coefficients of ln kappa(y) per bin, and the
// transmission function T(m) = int_0^1 exp(-kappa(y) m) dy.
//
// The design matrix A[i][c] = T_c(t_i), t_i = 2 (i + 1/2)/M - 1, is the same
// for every bin of M points, so its QR factors (A = QR, thin Householder,
// computed once on the host) are shared: per bin the kernel forms Q^T d
// (d_i = ln kappa_i of the sorted bin) and solves R C = Q^T d.
#include "hk_internal.h"

namespace hk {
namespace {

constexpr int kThreads = 256;

__device__ inline double key_to_double(const double* s, int64_t i) { return s[i]; }
__device__ inline double key_to_double(const float* s, int64_t i) { return (double)s[i]; }

// One workgroup per bin.  Q: row-major [M][nc]; R: row-major [nc][nc],
// upper triangular.  The last bin may use its own factors (Ql, Rl, ml).
template <typename K>
__global__ __launch_bounds__(kThreads) void resample_kernel(const K* __restrict__ sorted, int64_t n_points,
                                                            int64_t ppb, int nc, const double* __restrict__ Q,
                                                            const double* __restrict__ Rm, const double* __restrict__ Ql,
                                                            const double* __restrict__ Rl, double* __restrict__ coef)
{
    __shared__ double part[kThreads / 64][kMaxCoef];
    __shared__ double qd[kMaxCoef];
    const int64_t b = blockIdx.x;
    const int64_t b0 = b * ppb;
    const int64_t m = min(ppb, n_points - b0);
    const bool last = m != ppb;
    const double* q = last ? Ql : Q;
    const double* r = last ? Rl : Rm;
    double acc[kMaxCoef];
#pragma unroll
    for (int c = 0; c < kMaxCoef; ++c) acc[c] = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += kThreads) {
        const double d = log(fmax(key_to_double(sorted, b0 + i), 2.2250738585072014e-308));
        const double* qi = q + i * nc;
#pragma unroll
        for (int c = 0; c < kMaxCoef; ++c)
            if (c < nc) acc[c] = fma(qi[c], d, acc[c]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kMaxCoef; ++c) {
        double v = acc[c];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) part[wave][c] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
        double v = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) v += part[w][threadIdx.x];
        qd[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // back substitution R C = Q^T d
        double x[kMaxCoef];
        for (int c = nc - 1; c >= 0; --c) {
            double s = qd[c];
            for (int k = c + 1; k < nc; ++k) s -= r[c * nc + k] * x[k];
            x[c] = s / r[c * nc + c];
        }
        for (int c = 0; c < nc; ++c) coef[b * nc + c] = x[c];
    }
}

// T(m_j) = sum_q w_q exp(-exp(P(t_q)) m_j), P the bin's Chebyshev sum, at the
// quadrature nodes y_q (t_q = 2 y_q - 1).  One workgroup per bin.
__global__ __launch_bounds__(kThreads) void transmission_fit_kernel(const double* __restrict__ coef, int nc,
                                                                    const double* __restrict__ yq,
                                                                    const double* __restrict__ wq, int nq,
                                                                    const double* __restrict__ mcol, int n_m,
                                                                    double* __restrict__ T)
{
    __shared__ double kq[kMaxQuad];
    const int64_t b = blockIdx.x;
    const double* c = coef + b * nc;
    for (int q = threadIdx.x; q < nq; q += kThreads) {
        const double t = 2.0 * yq[q] - 1.0;
        double tm = 1.0, tc = t, s = c[0];
        if (nc > 1) s = fma(c[1], t, s);
        for (int k = 2; k < nc; ++k) {
            const double tn = fma(2.0 * t, tc, -tm);
            tm = tc;
            tc = tn;
            s = fma(c[k], tc, s);
        }
        kq[q] = exp(s);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n_m; j += kThreads) {
        const double mj = mcol[j];
        double s = 0.0;
        for (int q = 0; q < nq; ++q) s = fma(wq[q], exp(-kq[q] * mj), s);
        T[b * n_m + j] = s;
    }
}

// T(m_j) = (1/M) sum_i exp(-kappa_i m_j) over a bin's values.  Block
// (bin, chunk of 256 column masses); the bin's values pass through LDS.
template <typename K>
__global__ __launch_bounds__(kThreads) void transmission_direct_kernel(const K* __restrict__ sorted,
                                                                       int64_t n_points, int64_t ppb,
                                                                       const double* __restrict__ mcol, int n_m,
                                                                       double* __restrict__ T)
{
    __shared__ double kb[kThreads];
    const int64_t b = blockIdx.x;
    const int j = blockIdx.y * kThreads + threadIdx.x;
    const int64_t b0 = b * ppb;
    const int64_t m = min(ppb, n_points - b0);
    const double mj = j < n_m ? mcol[j] : 0.0;
    double s = 0.0;
    for (int64_t i0 = 0; i0 < m; i0 += kThreads) {
        const int64_t i = i0 + threadIdx.x;
        kb[threadIdx.x] = i < m ? key_to_double(sorted, b0 + i) : 0.0;
        __syncthreads();
        const int cnt = (int)min((int64_t)kThreads, m - i0);
        for (int k = 0; k < cnt; ++k) s += exp(-kb[k] * mj);
        __syncthreads();
    }
    if (j < n_m) T[b * n_m + j] = s / (double)m;
}

}  // namespace

hipError_t launch_resample(const void* sorted, int key_bytes, int64_t n_points, int64_t ppb, int nc,
                           const double* Q, const double* R, const double* Ql, const double* Rl, double* coef,
                           hipStream_t s)
{
    const int64_t n_bins = (n_points + ppb - 1) / ppb;
    if (n_bins == 0) return hipSuccess;
    if (key_bytes == 8)
        resample_kernel<double><<<dim3((unsigned)n_bins), dim3(kThreads), 0, s>>>(
            static_cast<const double*>(sorted), n_points, ppb, nc, Q, R, Ql, Rl, coef);
    else
        resample_kernel<float><<<dim3((unsigned)n_bins), dim3(kThreads), 0, s>>>(
            static_cast<const float*>(sorted), n_points, ppb, nc, Q, R, Ql, Rl, coef);
    return hipGetLastError();
}

hipError_t launch_transmission_fit(const double* coef, int64_t n_bins, int nc, const double* yq, const double* wq,
                                   int nq, const double* m, int n_m, double* T, hipStream_t s)
{
    if (n_bins == 0 || n_m == 0) return hipSuccess;
    transmission_fit_kernel<<<dim3((unsigned)n_bins), dim3(kThreads), 0, s>>>(coef, nc, yq, wq, nq, m, n_m, T);
    return hipGetLastError();
}

hipError_t launch_transmission_direct(const void* sorted, int key_bytes, int64_t n_points, int64_t ppb,
                                      const double* m, int n_m, double* T, hipStream_t s)
{
    const int64_t n_bins = (n_points + ppb - 1) / ppb;
    if (n_bins == 0 || n_m == 0) return hipSuccess;
    const dim3 grid((unsigned)n_bins, (unsigned)((n_m + kThreads - 1) / kThreads));
    if (key_bytes == 8)
        transmission_direct_kernel<double><<<grid, dim3(kThreads), 0, s>>>(static_cast<const double*>(sorted),
                                                                           n_points, ppb, m, n_m, T);
    else
        transmission_direct_kernel<float><<<grid, dim3(kThreads), 0, s>>>(static_cast<const float*>(sorted),
                                                                          n_points, ppb, m, n_m, T);
    return hipGetLastError();
}

}  // namespace hk
