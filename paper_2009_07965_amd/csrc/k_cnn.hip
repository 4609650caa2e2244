// Local-basis surrogate network: inference and training kernels.
//
// The network maps the input features of an S x S subdomain patch (the
// centred log-permeability and the log Robin parameters on the boundary
// cells) to its R local basis fields (the basis problems of Section 2.1):
// L 3x3 convolution layers with zero padding, ReLU between them, and a
// learned mean field added to the output.  Compute and accumulation are
// FP32; the convolution weights enter rounded to bfloat16 (round to
// nearest even) from FP32 master weights, which Adam updates.
//
// Layout: activations [n][channel][j][i] (row j, column i), weights
// [co][ci][3][3], parameter vector per layer W then b, then the mean field
// [R][S][S].  Every reduction runs in a fixed order (no atomics), so a
// training run is reproducible bit for bit.

#include "rmrcm_cnn.h"

namespace rmrcm {

__device__ inline float bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

// y[n][o] = b[o] + sum_c W[o][c] (*) x[n][c] (+ mean field) (ReLU); one
// workgroup per (sample, group of COB output channels), one thread per
// pixel; the zero-padded input planes and the group's weights in LDS.
template <int S, int COB>
__global__ __launch_bounds__(S * S) void k_conv_fwd(const float* __restrict__ x, int ci,
                                                    const float* __restrict__ W,
                                                    const float* __restrict__ b, int co,
                                                    const float* __restrict__ bmap, int relu,
                                                    float* __restrict__ y) {
    constexpr int P = S + 2, NT = S * S;
    extern __shared__ float sm[];
    float* xs = sm;
    float* ws = xs + ci * P * P;
    const int n = blockIdx.x, cb = blockIdx.y * COB, tid = threadIdx.x;
    const int nco = min(COB, co - cb);
    const float* xn = x + (size_t)n * ci * NT;
    for (int t = tid; t < ci * P * P; t += NT) {
        const int c = t / (P * P), r = t % (P * P), jj = r / P - 1, ii = r % P - 1;
        xs[t] = (jj >= 0 && jj < S && ii >= 0 && ii < S) ? xn[(size_t)c * NT + jj * S + ii] : 0.f;
    }
    for (int t = tid; t < COB * ci * 9; t += NT) {
        const int o = t / (ci * 9);
        ws[t] = o < nco ? W[(size_t)(cb + o) * ci * 9 + t % (ci * 9)] : 0.f;
    }
    __syncthreads();
    const int j = tid / S, i = tid % S;
    float acc[COB];
#pragma unroll
    for (int o = 0; o < COB; ++o) acc[o] = o < nco ? b[cb + o] : 0.f;
    for (int c = 0; c < ci; ++c) {
        const float* xc = xs + c * P * P + j * P + i;
        float xv[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int d = 0; d < 3; ++d) xv[a * 3 + d] = xc[a * P + d];
#pragma unroll
        for (int o = 0; o < COB; ++o) {
            const float* w = ws + (o * ci + c) * 9;
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[o] = fmaf(w[k], xv[k], acc[o]);
        }
    }
#pragma unroll
    for (int o = 0; o < COB; ++o) {
        if (o >= nco) break;
        float v = acc[o];
        if (bmap) v += bmap[(size_t)(cb + o) * NT + tid];
        if (relu) v = fmaxf(v, 0.f);
        y[((size_t)n * co + cb + o) * NT + tid] = v;
    }
}

// dx[n][c] = sum_o W[o][c] (*)^T dy[n][o], times the ReLU mask (x_in > 0)
// of the layer input when `mask` is given.
template <int S, int CIB>
__global__ __launch_bounds__(S * S) void k_conv_bwd_data(const float* __restrict__ dy, int co,
                                                         const float* __restrict__ W, int ci,
                                                         const float* __restrict__ mask,
                                                         float* __restrict__ dx) {
    constexpr int P = S + 2, NT = S * S;
    extern __shared__ float sm[];
    float* ds = sm;
    float* ws = ds + co * P * P;
    const int n = blockIdx.x, cb = blockIdx.y * CIB, tid = threadIdx.x;
    const int nci = min(CIB, ci - cb);
    const float* dn = dy + (size_t)n * co * NT;
    for (int t = tid; t < co * P * P; t += NT) {
        const int o = t / (P * P), r = t % (P * P), jj = r / P - 1, ii = r % P - 1;
        ds[t] = (jj >= 0 && jj < S && ii >= 0 && ii < S) ? dn[(size_t)o * NT + jj * S + ii] : 0.f;
    }
    for (int t = tid; t < co * CIB * 9; t += NT) {
        const int o = t / (CIB * 9), r = t % (CIB * 9), c = r / 9;
        ws[t] = c < nci ? W[((size_t)o * ci + cb + c) * 9 + r % 9] : 0.f;
    }
    __syncthreads();
    const int j = tid / S, i = tid % S;
    float acc[CIB];
#pragma unroll
    for (int c = 0; c < CIB; ++c) acc[c] = 0.f;
    for (int o = 0; o < co; ++o) {
        // x[j][i] feeds y[j - a + 1][i - d + 1]: padded row j - a + 2
        const float* dc = ds + o * P * P + (j + 2) * P + (i + 2);
        float dv[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int d = 0; d < 3; ++d) dv[a * 3 + d] = dc[-a * P - d];
#pragma unroll
        for (int c = 0; c < CIB; ++c) {
            const float* w = ws + (o * CIB + c) * 9;
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[c] = fmaf(w[k], dv[k], acc[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < CIB; ++c) {
        if (c >= nci) break;
        const size_t o = ((size_t)n * ci + cb + c) * NT + tid;
        float v = acc[c];
        if (mask && !(mask[o] > 0.f)) v = 0.f;
        dx[o] = v;
    }
}

// Partial weight and bias gradients of one chunk of samples:
// part[chunk][o][q], q < ci*9: sum_n sum_p dy[n][o][p] x[n][c][p + offset],
// q = ci*9: sum_n sum_p dy[n][o][p].  One workgroup per (chunk, o).
template <int S>
__global__ __launch_bounds__(256) void k_conv_bwd_w(const float* __restrict__ x, int ci,
                                                    const float* __restrict__ dy, int co, int nb,
                                                    int chunk, float* __restrict__ part) {
    constexpr int P = S + 2, NT = S * S;
    extern __shared__ float sm[];
    float* ds = sm;            // NT
    float* xs = ds + NT;       // ci * P * P
    const int ck = blockIdx.x, o = blockIdx.y, tid = threadIdx.x;
    const int nq = ci * 9 + 1;
    float acc[2] = {0.f, 0.f};
    const int n0 = ck * chunk, n1 = min(nb, n0 + chunk);
    for (int n = n0; n < n1; ++n) {
        const float* xn = x + (size_t)n * ci * NT;
        for (int t = tid; t < NT; t += 256) ds[t] = dy[((size_t)n * co + o) * NT + t];
        for (int t = tid; t < ci * P * P; t += 256) {
            const int c = t / (P * P), r = t % (P * P), jj = r / P - 1, ii = r % P - 1;
            xs[t] = (jj >= 0 && jj < S && ii >= 0 && ii < S) ? xn[(size_t)c * NT + jj * S + ii] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int q = tid + 256 * u;
            if (q >= nq) continue;
            float s = 0.f;
            if (q == nq - 1) {
                for (int p = 0; p < NT; ++p) s += ds[p];
            } else {
                const int c = q / 9, k = q % 9, a = k / 3, d = k % 3;
                const float* xc = xs + c * P * P + a * P + d;
                for (int jj = 0; jj < S; ++jj)
                    for (int ii = 0; ii < S; ++ii) s = fmaf(ds[jj * S + ii], xc[jj * P + ii], s);
            }
            acc[u] += s;
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int q = tid + 256 * u;
        if (q < nq) part[((size_t)ck * co + o) * nq + q] = acc[u];
    }
}

// Sum of the chunk partials in chunk order into the layer's slice of the
// gradient vector (W then b).
__global__ void k_conv_reduce_w(const float* __restrict__ part, int nchunk, int co, int ci,
                                float* __restrict__ gW, float* __restrict__ gb) {
    const int nq = ci * 9 + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= co * nq) return;
    const int o = t / nq, q = t % nq;
    float s = 0.f;
    for (int k = 0; k < nchunk; ++k) s += part[((size_t)k * co + o) * nq + q];
    if (q < nq - 1) gW[(size_t)o * ci * 9 + q] = s;
    else gb[o] = s;
}

// Gradient of the mean field: sum over the batch of the output gradient.
__global__ void k_bmap_grad(const float* __restrict__ dy, int nb, int m, float* __restrict__ g) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    float s = 0.f;
    for (int n = 0; n < nb; ++n) s += dy[(size_t)n * m + t];
    g[t] = s;
}

// Mean squared error: dy = 2 (y - t) / total and per-block partial sums of
// (y - t)^2 in FP64.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             size_t total, float* __restrict__ dy,
                                             double* __restrict__ part) {
    __shared__ double s[256];
    double acc = 0.0;
    const float sc = 2.0f / (float)total;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < total; k += (size_t)gridDim.x * 256) {
        const float d = y[k] - t[k];
        dy[k] = sc * d;
        acc += (double)d * d;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_mse_final(const double* __restrict__ part, int nb, size_t total,
                            double* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += part[k];
    *loss = s / (double)total;
}

// Adam on the FP32 master parameters, then the working copy (convolution
// weights rounded to bfloat16).
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, const unsigned char* __restrict__ isw,
                       float* __restrict__ wr, size_t np, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float t = th[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    th[k] = t;
    wr[k] = isw[k] ? bf16_rne(t) : t;
}

__global__ void k_round_copy(const float* __restrict__ th, const unsigned char* __restrict__ isw,
                             float* __restrict__ wr, size_t np) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < np) wr[k] = isw[k] ? bf16_rne(th[k]) : th[k];
}

// ---------------------------------------------------------------- launchers
namespace {
constexpr int kCOB = 8, kCIB = 8;

template <int S>
hipError_t conv_fwd_s(hipStream_t st, int nb, const float* x, int ci, const float* W, const float* b,
                      int co, const float* bmap, int relu, float* y) {
    const size_t lds = sizeof(float) * ((size_t)ci * (S + 2) * (S + 2) + (size_t)kCOB * ci * 9);
    hipError_t e = hipFuncSetAttribute((const void*)k_conv_fwd<S, kCOB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_conv_fwd<S, kCOB>), dim3(nb, (co + kCOB - 1) / kCOB), dim3(S * S), lds, st,
                       x, ci, W, b, co, bmap, relu, y);
    return hipGetLastError();
}

template <int S>
hipError_t conv_bwd_s(hipStream_t st, int nb, const float* x, int ci, const float* W, int co,
                      const float* dy, float* dx, const float* mask, float* part, int chunk,
                      float* gW, float* gb) {
    const int nchunk = (nb + chunk - 1) / chunk;
    size_t lds = sizeof(float) * ((size_t)S * S + (size_t)ci * (S + 2) * (S + 2));
    hipError_t e = hipFuncSetAttribute((const void*)k_conv_bwd_w<S>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_conv_bwd_w<S>, dim3(nchunk, co), dim3(256), lds, st, x, ci, dy, co, nb, chunk,
                       part);
    const int nq = co * (ci * 9 + 1);
    hipLaunchKernelGGL(k_conv_reduce_w, dim3((nq + 255) / 256), dim3(256), 0, st, part, nchunk, co, ci,
                       gW, gb);
    if (dx) {
        lds = sizeof(float) * ((size_t)co * (S + 2) * (S + 2) + (size_t)co * kCIB * 9);
        e = hipFuncSetAttribute((const void*)k_conv_bwd_data<S, kCIB>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_conv_bwd_data<S, kCIB>), dim3(nb, (ci + kCIB - 1) / kCIB), dim3(S * S),
                           lds, st, dy, co, W, ci, mask, dx);
    }
    return hipGetLastError();
}
}  // namespace

hipError_t cnn_conv_fwd(hipStream_t st, int S, int nb, const float* x, int ci, const float* W,
                        const float* b, int co, const float* bmap, int relu, float* y) {
    switch (S) {
        case 8: return conv_fwd_s<8>(st, nb, x, ci, W, b, co, bmap, relu, y);
        case 16: return conv_fwd_s<16>(st, nb, x, ci, W, b, co, bmap, relu, y);
        case 32: return conv_fwd_s<32>(st, nb, x, ci, W, b, co, bmap, relu, y);
    }
    return hipErrorInvalidValue;
}

hipError_t cnn_conv_bwd(hipStream_t st, int S, int nb, const float* x, int ci, const float* W, int co,
                        const float* dy, float* dx, const float* mask, float* part, int chunk,
                        float* gW, float* gb) {
    switch (S) {
        case 8: return conv_bwd_s<8>(st, nb, x, ci, W, co, dy, dx, mask, part, chunk, gW, gb);
        case 16: return conv_bwd_s<16>(st, nb, x, ci, W, co, dy, dx, mask, part, chunk, gW, gb);
        case 32: return conv_bwd_s<32>(st, nb, x, ci, W, co, dy, dx, mask, part, chunk, gW, gb);
    }
    return hipErrorInvalidValue;
}

hipError_t cnn_bmap_grad(hipStream_t st, const float* dy, int nb, int m, float* g) {
    hipLaunchKernelGGL(k_bmap_grad, dim3((m + 255) / 256), dim3(256), 0, st, dy, nb, m, g);
    return hipGetLastError();
}

hipError_t cnn_mse(hipStream_t st, const float* y, const float* t, size_t total, float* dy,
                   double* part, int nblk, double* loss) {
    hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, st, y, t, total, dy, part);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, st, part, nblk, total, loss);
    return hipGetLastError();
}

hipError_t cnn_adam(hipStream_t st, float* th, const float* g, float* m, float* v,
                    const unsigned char* isw, float* wr, size_t np, float lr, float b1, float b2,
                    float eps, float c1, float c2) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, th, g, m, v, isw,
                       wr, np, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t cnn_round_copy(hipStream_t st, const float* th, const unsigned char* isw, float* wr,
                          size_t np) {
    hipLaunchKernelGGL(k_round_copy, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, th, isw, wr,
                       np);
    return hipGetLastError();
}

}  // namespace rmrcm
