// Internal declarations of the local-basis surrogate network (host object
// and kernel launchers).  Not part of the public ABI.
#pragma once

#include "rmrcm_internal.h"

struct rmrcm_cnn {
    int S = 0, C = 0, L = 0, R = 0, maxnb = 0, device = 0;
    hipStream_t stream = nullptr, own = nullptr;
    size_t np = 0;
    std::vector<size_t> offW, offb;        // per layer: weights, biases in the parameter vector
    size_t offB = 0;                       // mean field
    std::vector<int> co, ci;               // per layer
    float* th = nullptr;                   // FP32 master parameters
    float* wr = nullptr;                   // working copy (convolution weights in bfloat16)
    float* g = nullptr;                    // gradient
    float* m = nullptr;                    // Adam moments
    float* v = nullptr;
    unsigned char* isw = nullptr;          // 1 where the parameter is a convolution weight
    std::vector<float*> h;                 // h[1 .. L-1]: hidden activations [maxnb][C][S][S]
    float* y = nullptr;                    // output of loss_grad's forward [maxnb][R][S][S]
    float* g0 = nullptr;                   // activation gradients (ping-pong)
    float* g1 = nullptr;
    float* part = nullptr;                 // weight-gradient partials per chunk
    double* lpart = nullptr;               // loss partials
    double* loss = nullptr;
    int adam_t = 0;
    int chunk = 1;                         // samples per weight-gradient partial
    static constexpr int kLossBlocks = 256;
};

namespace rmrcm {
hipError_t cnn_conv_fwd(hipStream_t st, int S, int nb, const float* x, int ci, const float* W,
                        const float* b, int co, const float* bmap, int relu, float* y);
hipError_t cnn_conv_bwd(hipStream_t st, int S, int nb, const float* x, int ci, const float* W, int co,
                        const float* dy, float* dx, const float* mask, float* part, int chunk,
                        float* gW, float* gb);
hipError_t cnn_bmap_grad(hipStream_t st, const float* dy, int nb, int m, float* g);
hipError_t cnn_mse(hipStream_t st, const float* y, const float* t, size_t total, float* dy,
                   double* part, int nblk, double* loss);
hipError_t cnn_adam(hipStream_t st, float* th, const float* g, float* m, float* v,
                    const unsigned char* isw, float* wr, size_t np, float lr, float b1, float b2,
                    float eps, float c1, float c2);
hipError_t cnn_round_copy(hipStream_t st, const float* th, const unsigned char* isw, float* wr,
                          size_t np);
// Forward pass of nb <= maxnb samples on the network's stream.
hipError_t cnn_forward(rmrcm_cnn* net, int nb, const float* x, float* y);
}  // namespace rmrcm
