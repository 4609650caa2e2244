// Host side of the local-basis surrogate network: parameter layout, device
// buffers, forward / backward orchestration, Adam, save and load.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "rmrcm_cnn.h"

namespace {

#define CNN_TRY(expr)                                              \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) {                                    \
            (void)hipGetLastError();                               \
            return e_ == hipErrorOutOfMemory ? RMRCM_ENOMEM : RMRCM_EDEVICE; \
        }                                                          \
    } while (0)

template <typename T>
int cnn_alloc(T** p, size_t count) {
    *p = nullptr;
    CNN_TRY(hipMalloc((void**)p, (count ? count : 1) * sizeof(T)));
    CNN_TRY(hipMemset(*p, 0, (count ? count : 1) * sizeof(T)));
    return RMRCM_OK;
}

void cnn_free(rmrcm_cnn* n) {
    auto f = [](void* p) {
        if (p) (void)hipFree(p);
    };
    f(n->th);
    f(n->wr);
    f(n->g);
    f(n->m);
    f(n->v);
    f(n->isw);
    for (float* p : n->h) f(p);
    f(n->y);
    f(n->g0);
    f(n->g1);
    f(n->part);
    f(n->lpart);
    f(n->loss);
    if (n->own) (void)hipStreamDestroy(n->own);
}

int build(int S, int C, int L, int R, int maxnb, int device, rmrcm_cnn** out) {
    *out = nullptr;
    if ((S != 8 && S != 16 && S != 32) || C < 1 || C > 32 || L < 2 || L > 16 || R < 1 || R > 32 ||
        maxnb < 1)
        return RMRCM_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return RMRCM_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return RMRCM_EDEVICE;
    rmrcm_cnn* n = new (std::nothrow) rmrcm_cnn();
    if (!n) return RMRCM_ENOMEM;
    n->S = S, n->C = C, n->L = L, n->R = R, n->maxnb = maxnb, n->device = device;
    size_t k = 0;
    for (int l = 0; l < L; ++l) {
        const int co = l == L - 1 ? R : C, ci = l == 0 ? 2 : C;
        n->co.push_back(co);
        n->ci.push_back(ci);
        n->offW.push_back(k);
        k += (size_t)co * ci * 9;
        n->offb.push_back(k);
        k += co;
    }
    n->offB = k;
    k += (size_t)R * S * S;
    n->np = k;
    const size_t plane = (size_t)S * S, wide = (size_t)(C > R ? C : R);
    int r = RMRCM_OK;
    auto fail = [&](int rr) {
        cnn_free(n);
        delete n;
        return rr;
    };
    if (hipStreamCreateWithFlags(&n->own, hipStreamNonBlocking) != hipSuccess) return fail(RMRCM_EDEVICE);
    n->stream = n->own;
    n->h.assign(L, nullptr);
    if ((r = cnn_alloc(&n->th, k)) || (r = cnn_alloc(&n->wr, k)) || (r = cnn_alloc(&n->g, k)) ||
        (r = cnn_alloc(&n->m, k)) || (r = cnn_alloc(&n->v, k)) || (r = cnn_alloc(&n->isw, k)) ||
        (r = cnn_alloc(&n->y, (size_t)maxnb * R * plane)) ||
        (r = cnn_alloc(&n->g0, (size_t)maxnb * wide * plane)) ||
        (r = cnn_alloc(&n->g1, (size_t)maxnb * wide * plane)) ||
        (r = cnn_alloc(&n->part, (size_t)((maxnb + n->chunk - 1) / n->chunk) * wide * (C * 9 + 1))) ||
        (r = cnn_alloc(&n->lpart, rmrcm_cnn::kLossBlocks)) || (r = cnn_alloc(&n->loss, 1)))
        return fail(r);
    for (int l = 1; l < L; ++l)
        if ((r = cnn_alloc(&n->h[l], (size_t)maxnb * C * plane))) return fail(r);
    std::vector<unsigned char> isw(k, 0);
    for (int l = 0; l < L; ++l)
        for (size_t q = 0; q < (size_t)n->co[l] * n->ci[l] * 9; ++q) isw[n->offW[l] + q] = 1;
    if (hipMemcpy(n->isw, isw.data(), k, hipMemcpyHostToDevice) != hipSuccess) return fail(RMRCM_EDEVICE);
    *out = n;
    return RMRCM_OK;
}

// Loss, output gradient and every parameter gradient of one batch.
int loss_grad(rmrcm_cnn* n, int nb, const float* x, const float* t) {
    CNN_TRY(rmrcm::cnn_forward(n, nb, x, n->y));
    const int S = n->S, L = n->L, R = n->R;
    const size_t total = (size_t)nb * R * S * S;
    CNN_TRY(rmrcm::cnn_mse(n->stream, n->y, t, total, n->g0, n->lpart, rmrcm_cnn::kLossBlocks, n->loss));
    CNN_TRY(rmrcm::cnn_bmap_grad(n->stream, n->g0, nb, R * S * S, n->g + n->offB));
    float* cur = n->g0;
    for (int l = L - 1; l >= 0; --l) {
        const float* in = l == 0 ? x : n->h[l];
        float* nxt = cur == n->g0 ? n->g1 : n->g0;
        CNN_TRY(rmrcm::cnn_conv_bwd(n->stream, S, nb, in, n->ci[l], n->wr + n->offW[l], n->co[l], cur,
                                    l > 0 ? nxt : nullptr, l > 0 ? n->h[l] : nullptr, n->part, n->chunk,
                                    n->g + n->offW[l], n->g + n->offb[l]));
        cur = nxt;
    }
    return RMRCM_OK;
}

}  // namespace

namespace rmrcm {

hipError_t cnn_forward(rmrcm_cnn* n, int nb, const float* x, float* y) {
    const float* in = x;
    for (int l = 0; l < n->L; ++l) {
        const bool last = l == n->L - 1;
        float* out = last ? y : n->h[l + 1];
        hipError_t e = cnn_conv_fwd(n->stream, n->S, nb, in, n->ci[l], n->wr + n->offW[l],
                                    n->wr + n->offb[l], n->co[l], last ? n->wr + n->offB : nullptr,
                                    last ? 0 : 1, out);
        if (e != hipSuccess) return e;
        in = out;
    }
    return hipSuccess;
}

}  // namespace rmrcm

extern "C" {

int rmrcm_cnn_create(int32_t S, int32_t C, int32_t L, int32_t R, int32_t max_batch, int32_t device,
                     rmrcm_cnn** out) {
    if (!out) return RMRCM_EINVAL;
    return build(S, C, L, R, max_batch, device, out);
}

int rmrcm_cnn_num_params(const rmrcm_cnn* n, int64_t* np) {
    if (!n || !np) return RMRCM_EINVAL;
    *np = (int64_t)n->np;
    return RMRCM_OK;
}

int rmrcm_cnn_set_stream(rmrcm_cnn* n, void* stream) {
    if (!n) return RMRCM_EINVAL;
    n->stream = stream ? (hipStream_t)stream : n->own;
    return RMRCM_OK;
}

int rmrcm_cnn_set_params(rmrcm_cnn* n, const float* theta) {
    if (!n || !theta) return RMRCM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return RMRCM_EDEVICE;
    for (size_t k = 0; k < n->np; ++k)
        if (!std::isfinite(theta[k])) return RMRCM_EINVAL;
    CNN_TRY(hipMemcpyAsync(n->th, theta, n->np * sizeof(float), hipMemcpyHostToDevice, n->stream));
    CNN_TRY(hipMemsetAsync(n->m, 0, n->np * sizeof(float), n->stream));
    CNN_TRY(hipMemsetAsync(n->v, 0, n->np * sizeof(float), n->stream));
    CNN_TRY(rmrcm::cnn_round_copy(n->stream, n->th, n->isw, n->wr, n->np));
    CNN_TRY(hipStreamSynchronize(n->stream));
    n->adam_t = 0;
    return RMRCM_OK;
}

int rmrcm_cnn_get_params(rmrcm_cnn* n, float* theta) {
    if (!n || !theta) return RMRCM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return RMRCM_EDEVICE;
    CNN_TRY(hipMemcpyAsync(theta, n->th, n->np * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    CNN_TRY(hipStreamSynchronize(n->stream));
    return RMRCM_OK;
}

int rmrcm_cnn_forward(rmrcm_cnn* n, int32_t nb, const float* x, float* y) {
    if (!n || !x || !y || nb < 1 || nb > n->maxnb) return RMRCM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return RMRCM_EDEVICE;
    CNN_TRY(rmrcm::cnn_forward(n, nb, x, y));
    return RMRCM_OK;
}

int rmrcm_cnn_loss_grad(rmrcm_cnn* n, int32_t nb, const float* x, const float* t, double* loss,
                        float* grad) {
    if (!n || !x || !t || nb < 1 || nb > n->maxnb) return RMRCM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return RMRCM_EDEVICE;
    const int r = loss_grad(n, nb, x, t);
    if (r != RMRCM_OK) return r;
    if (grad) CNN_TRY(hipMemcpyAsync(grad, n->g, n->np * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    if (loss) CNN_TRY(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    if (grad || loss) CNN_TRY(hipStreamSynchronize(n->stream));
    return RMRCM_OK;
}

int rmrcm_cnn_train_step(rmrcm_cnn* n, int32_t nb, const float* x, const float* t, float lr,
                         double* loss) {
    if (!n || !x || !t || nb < 1 || nb > n->maxnb || !(lr > 0)) return RMRCM_EINVAL;
    if (hipSetDevice(n->device) != hipSuccess) return RMRCM_EDEVICE;
    const int r = loss_grad(n, nb, x, t);
    if (r != RMRCM_OK) return r;
    n->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)n->adam_t), c2 = 1.f - std::pow(b2, (float)n->adam_t);
    CNN_TRY(rmrcm::cnn_adam(n->stream, n->th, n->g, n->m, n->v, n->isw, n->wr, n->np, lr, b1, b2, 1e-8f,
                            c1, c2));
    if (loss) {
        CNN_TRY(hipMemcpyAsync(loss, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
        CNN_TRY(hipStreamSynchronize(n->stream));
    }
    return RMRCM_OK;
}

int rmrcm_cnn_save(rmrcm_cnn* n, const char* path) {
    if (!n || !path) return RMRCM_EINVAL;
    std::vector<float> th(n->np);
    const int r = rmrcm_cnn_get_params(n, th.data());
    if (r != RMRCM_OK) return r;
    FILE* f = std::fopen(path, "wb");
    if (!f) return RMRCM_EINVAL;
    const char magic[8] = {'R', 'M', 'R', 'C', 'M', 'C', 'N', 'N'};
    const int32_t hdr[4] = {n->S, n->C, n->L, n->R};
    const int64_t np = (int64_t)n->np;
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 4, f) == 4 &&
              std::fwrite(&np, sizeof(np), 1, f) == 1 &&
              std::fwrite(th.data(), sizeof(float), n->np, f) == n->np;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? RMRCM_OK : RMRCM_EINVAL;
}

int rmrcm_cnn_load(const char* path, int32_t max_batch, int32_t device, rmrcm_cnn** out) {
    if (!path || !out) return RMRCM_EINVAL;
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return RMRCM_EINVAL;
    char magic[8];
    int32_t hdr[4];
    int64_t np = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "RMRCMCNN", 8) == 0 &&
              std::fread(hdr, sizeof(int32_t), 4, f) == 4 && std::fread(&np, sizeof(np), 1, f) == 1;
    std::vector<float> th;
    if (ok && np > 0 && np < (int64_t)1 << 28) {
        th.resize((size_t)np);
        ok = std::fread(th.data(), sizeof(float), (size_t)np, f) == (size_t)np;
    } else {
        ok = false;
    }
    std::fclose(f);
    if (!ok) return RMRCM_EINVAL;
    rmrcm_cnn* n = nullptr;
    int r = build(hdr[0], hdr[1], hdr[2], hdr[3], max_batch, device, &n);
    if (r != RMRCM_OK) return r;
    if ((int64_t)n->np != np || (r = rmrcm_cnn_set_params(n, th.data())) != RMRCM_OK) {
        cnn_free(n);
        delete n;
        return r != RMRCM_OK ? r : RMRCM_EINVAL;
    }
    *out = n;
    return RMRCM_OK;
}

void rmrcm_cnn_destroy(rmrcm_cnn* n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    cnn_free(n);
    delete n;
}

}  // extern "C"
