// Local-basis surrogate network: inference and training kernels.
//
// The network maps the input features of an S x S subdomain patch (the
// centred log-permeability and the log Robin parameters on the boundary
// cells) to its R local basis fields (the basis problems of Section 2.1):
// L 3x3 convolution layers with zero padding, ReLU between them, and a
// learned mean field added to the output.  The convolution weights enter
// rounded to bfloat16 (round to nearest even) from FP32 master weights,
// which Adam updates; activations and accumulation are FP32.  The
// convolutions run on the matrix cores: forward and backward-data as
// implicit GEMMs on the bfloat16 units with every FP32 input split exactly
// in three bfloat16 pieces (so the products are the FP32 products), the
// weight gradient on the FP32 matrix cores (v_mfma_f32_16x16x4f32).
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

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// bfloat16 bits of f, round to nearest even.
__device__ inline unsigned bf16_bits(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

// Three bfloat16 pieces whose sum is f exactly: the first holds f to 8
// significant bits, the second the next 8 of the (exact) remainder, the
// third the last 8; every product of a piece with a bfloat16 weight is
// exact in FP32, so the matrix cores reproduce the FP32 products.
__device__ inline void split3(float f, unsigned& h0, unsigned& h1, unsigned& h2) {
    h0 = bf16_bits(f);
    float r = f - __uint_as_float(h0 << 16);
    h1 = bf16_bits(r);
    r -= __uint_as_float(h1 << 16);
    h2 = bf16_bits(r);
}

__device__ inline bf8v pack8(const unsigned (&h)[8]) {
    u4v w;
    w.x = h[0] | (h[1] << 16);
    w.y = h[2] | (h[3] << 16);
    w.z = h[4] | (h[5] << 16);
    w.w = h[6] | (h[7] << 16);
    return __builtin_bit_cast(bf8v, w);
}

// A 3x3 convolution with zero padding as an implicit GEMM on the bfloat16
// matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation): rows = output
// channels (MT tiles of 16), columns = pixels, reduction over (input
// channel, tap) in steps of 32.  Forward (BWD false):
//     y[n][o][p] = b[o] + sum_{c,tap} W[o][c][tap] x[n][c][p + tap] (+ mean field) (ReLU);
// backward data (BWD true), the transposed and flipped weights:
//     dx[n][c][p] = sum_{o,tap} W[o][c][8 - tap] dy[n][o][p + tap - (1,1)...]
// i.e. the same access of the zero-padded planes with tap' = 8 - tap, then
// the ReLU mask of the layer input.  A workgroup (four waves, 64 pixels
// each) takes 256 consecutive pixels: several whole samples (S = 8), one
// sample (16) or a band of rows of one (32); its input planes with a
// one-cell halo are staged in LDS.  Each input value is split in three
// bfloat16 pieces (exact), the weights are bfloat16 already: three products
// per step give the FP32 products exactly.
template <int S, int MT, bool BWD>
__global__ __launch_bounds__(256) void k_conv_mfma(const float* __restrict__ x, int cin,
                                                   const float* __restrict__ W, int wci,
                                                   const float* __restrict__ b, int cout,
                                                   const float* __restrict__ bmap, int relu,
                                                   const float* __restrict__ mask, int nb,
                                                   float* __restrict__ y) {
    constexpr int NT = S * S, P = S + 2;
    constexpr int SPW = NT >= 256 ? 1 : 256 / NT;      // samples per workgroup
    constexpr int RW = NT >= 256 ? 256 / S : S;         // rows per workgroup
    constexpr int PR = RW + 2;                          // staged padded rows
    extern __shared__ float xs[];                       // [SPW][cin][PR][P]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    int n0, r0;
    if (NT >= 256) {
        constexpr int per = NT / 256;
        n0 = blockIdx.x / per;
        r0 = (blockIdx.x % per) * RW;
    } else {
        n0 = blockIdx.x * SPW;
        r0 = 0;
    }
    for (int t = tid; t < SPW * cin * PR * P; t += 256) {
        const int pc = t % P, pr = (t / P) % PR, c = (t / (P * PR)) % cin, ls = t / (P * PR * cin);
        const int n = n0 + ls, jj = r0 + pr - 1, ii = pc - 1;
        xs[t] = (n < nb && jj >= 0 && jj < S && ii >= 0 && ii < S) ? x[((size_t)n * cin + c) * NT + jj * S + ii]
                                                                    : 0.f;
    }
    __syncthreads();
    const int K = cin * 9, KS = (K + 31) / 32;
    f4v acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < KS; ++ks) {
        // weights of rows 16 mt + l16 at reduction indices 32 ks + 8 lq + j
        bf8v a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            unsigned h[8];
            const int o = 16 * mt + l16;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * ks + 8 * lq + j, c = k / 9, tap = k % 9;
                float v = 0.f;
                if (o < cout && k < K)
                    v = BWD ? W[((size_t)c * wci + o) * 9 + (8 - tap)] : W[((size_t)o * wci + c) * 9 + tap];
                h[j] = bf16_bits(v);                    // exact: the weights are bfloat16
            }
            a[mt] = pack8(h);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int q = 64 * w + 16 * nt + l16;       // pixel column of this lane
            const int ls = q / NT, p = q % NT + r0 * S;
            const int row = p / S, col = p % S;
            unsigned h0[8], h1[8], h2[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 32 * ks + 8 * lq + j, c = k / 9, tap = k % 9;
                const float v = k < K ? xs[((ls * cin + c) * PR + (row - r0 + tap / 3)) * P + col + tap % 3] : 0.f;
                split3(v, h0[j], h1[j], h2[j]);
            }
            const bf8v b0 = pack8(h0), b1 = pack8(h1), b2 = pack8(h2);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b0, acc[mt][nt], 0, 0, 0);
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b1, acc[mt][nt], 0, 0, 0);
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b2, acc[mt][nt], 0, 0, 0);
            }
        }
    }
    // lane l holds column l % 16 (a pixel) and rows 4 (l / 16) + v (channels)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int q = 64 * w + 16 * nt + l16;
        const int n = n0 + q / NT, p = q % NT + r0 * S;
        if (n >= nb) continue;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 16 * mt + 4 * lq + v;
                if (o >= cout) continue;
                const size_t at = ((size_t)n * cout + o) * NT + p;
                float r = acc[mt][nt][v];
                if (BWD) {
                    if (mask && !(mask[at] > 0.f)) r = 0.f;
                } else {
                    r += b[o];
                    if (bmap) r += bmap[(size_t)o * NT + p];
                    if (relu) r = fmaxf(r, 0.f);
                }
                y[at] = r;
            }
    }
}

// Partial weight and bias gradients of one chunk of samples on the FP32
// matrix cores (v_mfma_f32_16x16x4f32): part[chunk][o][q] =
// sum over the chunk's samples and pixels p of dy[n][o][p] x[n][c][p + tap]
// for q = 9 c + tap, and of dy[n][o][p] for q = 9 cin (the bias column, a
// column of ones).  Rows = output channels (MT tiles), columns = q (tiles
// of 16 over the four waves), reduction over pixels in bands of RB rows
// staged in LDS (the input with a one-cell halo, the output gradient).
// One workgroup per chunk; samples and bands in a fixed order.
template <int S, int MT>
__global__ __launch_bounds__(256) void k_conv_bwd_w_mfma(const float* __restrict__ x, int ci,
                                                         const float* __restrict__ dy, int co, int nb,
                                                         int chunk, float* __restrict__ part) {
    constexpr int NT = S * S, P = S + 2;
    constexpr int RB = NT >= 256 ? 256 / S : S;         // rows per band (256 pixels or the sample)
    constexpr int PR = RB + 2;
    extern __shared__ float sm[];
    float* xs = sm;                                     // [ci][PR][P]
    float* ds = xs + ci * PR * P;                       // [co][RB][S]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int ck = blockIdx.x;
    const int nq = ci * 9 + 1, NQT = (nq + 15) / 16;
    constexpr int MAXT = 5;                             // column tiles per wave (ci <= 35)
    f4v acc[MT][MAXT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int u = 0; u < MAXT; ++u) acc[mt][u] = f4v{0.f, 0.f, 0.f, 0.f};
    const int n0 = ck * chunk, n1 = min(nb, n0 + chunk);
    for (int n = n0; n < n1; ++n) {
        for (int r0 = 0; r0 < S; r0 += RB) {
            __syncthreads();
            for (int t = tid; t < ci * PR * P; t += 256) {
                const int pc = t % P, pr = (t / P) % PR, c = t / (P * PR);
                const int jj = r0 + pr - 1, ii = pc - 1;
                xs[t] = (jj >= 0 && jj < S && ii >= 0 && ii < S) ? x[((size_t)n * ci + c) * NT + jj * S + ii] : 0.f;
            }
            for (int t = tid; t < co * RB * S; t += 256) {
                const int o = t / (RB * S), p = t % (RB * S);
                ds[t] = dy[((size_t)n * co + o) * NT + r0 * S + p];
            }
            __syncthreads();
            for (int k0 = 0; k0 < RB * S; k0 += 4) {
                const int pk = k0 + lq;                 // pixel of this lane's reduction index
                const int row = pk / S, col = pk % S;
                float av[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int o = 16 * mt + l16;
                    av[mt] = o < co ? ds[(o * RB + row) * S + col] : 0.f;
                }
#pragma unroll
                for (int u = 0; u < MAXT; ++u) {
                    const int tq = w + 4 * u;
                    if (tq >= NQT) break;               // uniform per wave
                    const int q = 16 * tq + l16;
                    float bv = 0.f;
                    if (q < nq - 1) {
                        const int c = q / 9, tap = q % 9;
                        bv = xs[(c * PR + row + tap / 3) * P + col + tap % 3];
                    } else if (q == nq - 1) {
                        bv = 1.f;
                    }
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        acc[mt][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mt], bv, acc[mt][u], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < MAXT; ++u) {
        const int tq = w + 4 * u;
        if (tq >= NQT) break;
        const int q = 16 * tq + l16;
        if (q >= nq) continue;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 16 * mt + 4 * lq + v;
                if (o < co) part[((size_t)ck * co + o) * nq + q] = acc[mt][u][v];
            }
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
template <int S>
constexpr int conv_workgroups(int nb) {
    return S * S >= 256 ? nb * (S * S / 256) : (nb + 256 / (S * S) - 1) / (256 / (S * S));
}
template <int S>
constexpr size_t conv_lds(int cin) {
    return sizeof(float) * (size_t)(S * S >= 256 ? 1 : 256 / (S * S)) * cin *
           ((S * S >= 256 ? 256 / S : S) + 2) * (S + 2);
}

template <int S, bool BWD>
hipError_t conv_mfma_s(hipStream_t st, int nb, const float* x, int cin, const float* W, int wci,
                       const float* b, int cout, const float* bmap, int relu, const float* mask, float* y) {
    const size_t lds = conv_lds<S>(cin);
    auto go = [&](auto kern) -> hipError_t {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(conv_workgroups<S>(nb)), dim3(256), lds, st, x, cin, W, wci, b, cout,
                           bmap, relu, mask, nb, y);
        return hipGetLastError();
    };
    return cout <= 16 ? go(k_conv_mfma<S, 1, BWD>) : go(k_conv_mfma<S, 2, BWD>);
}

template <int S>
hipError_t conv_fwd_s(hipStream_t st, int nb, const float* x, int ci, const float* W, const float* b,
                      int co, const float* bmap, int relu, float* y) {
    return conv_mfma_s<S, false>(st, nb, x, ci, W, ci, b, co, bmap, relu, nullptr, y);
}

template <int S>
hipError_t conv_bwd_s(hipStream_t st, int nb, const float* x, int ci, const float* W, int co,
                      const float* dy, float* dx, const float* mask, float* part, int chunk,
                      float* gW, float* gb) {
    const int nchunk = (nb + chunk - 1) / chunk;
    constexpr int RB = S * S >= 256 ? 256 / S : S;
    const size_t lds = sizeof(float) * ((size_t)ci * (RB + 2) * (S + 2) + (size_t)co * RB * S);
    auto go = [&](auto kern) -> hipError_t {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(nchunk), dim3(256), lds, st, x, ci, dy, co, nb, chunk, part);
        return hipGetLastError();
    };
    hipError_t e = co <= 16 ? go(k_conv_bwd_w_mfma<S, 1>) : go(k_conv_bwd_w_mfma<S, 2>);
    if (e != hipSuccess) return e;
    const int nq = co * (ci * 9 + 1);
    hipLaunchKernelGGL(k_conv_reduce_w, dim3((nq + 255) / 256), dim3(256), 0, st, part, nchunk, co, ci,
                       gW, gb);
    if (dx) {
        e = conv_mfma_s<S, true>(st, nb, dy, co, W, ci, nullptr, ci, nullptr, 0, mask, dx);
        if (e != hipSuccess) return e;
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
