// Host runtime behind the C ABI of include/rmrcm.h: validation, the level
// tables of the nested binary hierarchy (Section 3.1), the device memory
// plan and the order of kernel launches for setup and solve.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rmrcm_cnn.h"
#include "rmrcm_internal.h"

using rmrcm::Geo;
using rmrcm::Level;

namespace {

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int v) {
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// With RMRCM_DEBUG set in the environment, a failing HIP call is reported
// on stderr (file, line, HIP's message) before its status is returned.
bool debug_enabled() {
    static const bool on = std::getenv("RMRCM_DEBUG") != nullptr;
    return on;
}
void report_hip(hipError_t e, const char* what, int line) {
    if (debug_enabled()) std::fprintf(stderr, "rmrcm: %s failed at api.cpp:%d: %s\n", what, line, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                 \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) {                       \
            report_hip(e_, #expr, __LINE__);          \
            if (e_ == hipErrorOutOfMemory) return RMRCM_ENOMEM; \
            return RMRCM_EDEVICE;                     \
        }                                             \
    } while (0)

// Device array of count elements, zero-filled in stream order.  With an
// arena (the allocation-free entry point) the array is carved from it at a
// 256-byte boundary and NOT filled here: the caller zero-fills the used part
// of the arena once every array is carved; RMRCM_ETOOBIG when it does not fit.
// In a memory plan (c->counting) only the bytes are added up.  With a memory
// cap, an array that would take the context past it is RMRCM_ENOMEM.
template <typename T>
int dalloc(rmrcm_ctx* c, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    if (c->counting) {
        c->device_bytes += bytes;
        return RMRCM_OK;
    }
    if (!c->arena && c->prm.mem_cap && c->device_bytes + bytes > c->prm.mem_cap) return RMRCM_ENOMEM;
    if (c->arena) {
        const size_t off = (c->arena_used + 255) & ~(size_t)255;
        const size_t end = (off + bytes + 255) & ~(size_t)255;
        if (end > c->arena_cap || end < off) return RMRCM_ETOOBIG;
        *p = reinterpret_cast<T*>(c->arena + off);
        c->arena_used = end;
        c->device_bytes += bytes;
        return RMRCM_OK;
    }
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return e == hipErrorOutOfMemory ? RMRCM_ENOMEM : RMRCM_EDEVICE;
    }
    c->device_bytes += bytes;
    if (hipMemsetAsync(*p, 0, bytes, c->stream) != hipSuccess) return RMRCM_EDEVICE;
    return RMRCM_OK;
}

#define TRY(expr)                \
    do {                         \
        int r_ = (expr);         \
        if (r_ != RMRCM_OK) return r_; \
    } while (0)

int validate(const rmrcm_params* p) {
    if (!p) return RMRCM_EINVAL;
    if (p->nx <= 0 || p->ny <= 0 || p->sub_nx <= 0 || p->sub_ny <= 0 || p->seg <= 0)
        return RMRCM_EINVAL;
    if (!(p->lx > 0) || !(p->ly > 0) || !std::isfinite(p->lx) || !std::isfinite(p->ly))
        return RMRCM_EINVAL;
    if (!(p->alpha > 0) || !std::isfinite(p->alpha)) return RMRCM_EINVAL;
    if (p->nx % p->sub_nx || p->ny % p->sub_ny) return RMRCM_EINVAL;
    if (p->seg_u < 0 || p->seg_p < 0) return RMRCM_EINVAL;
    const int su = p->seg_u ? p->seg_u : p->seg, sp = p->seg_p ? p->seg_p : p->seg;
    const int piece = std::min(su, sp);
    if (p->sub_nx % su || p->sub_ny % su || p->sub_nx % sp || p->sub_ny % sp) return RMRCM_EINVAL;
    if (std::max(su, sp) % piece) return RMRCM_EINVAL;
    if (!is_pow2(p->nx / p->sub_nx) || !is_pow2(p->ny / p->sub_ny)) return RMRCM_EINVAL;
    if (p->precision < RMRCM_FP64 || p->precision > RMRCM_MIXED_LEARNED) return RMRCM_EINVAL;
    if (p->nz < 0) return RMRCM_EINVAL;
    if (p->nz > 0) {
        // the 3D problem: columns of sub_nx x sub_ny x nz cells, FP64, MuMM spaces
        if (!(p->lz > 0) || !std::isfinite(p->lz)) return RMRCM_EINVAL;
        if (p->precision != RMRCM_FP64) return RMRCM_ENOTSUP;
        if ((p->seg_u && p->seg_u != p->seg) || (p->seg_p && p->seg_p != p->seg)) return RMRCM_ENOTSUP;
        if ((size_t)p->sub_nx * p->nz > 64 || p->sub_ny > 64) return RMRCM_ENOTSUP;
        // one column's factor block, right-hand sides and products in LDS
        const size_t nb = (size_t)p->sub_nx * p->nz, ncol = 2 * (size_t)(p->sub_nx + p->sub_ny) / p->seg + 1;
        const size_t ts = (nb + 15) / 16, zl = nb * (ncol > 12 ? ncol : 12);
        const size_t zlen = zl > 66 * ts * ts ? zl : 66 * ts * ts;
        if (sizeof(double) * (nb * (nb + 1) + nb * ncol + zlen + 2 * nb + 2) > 160 * 1024)
            return RMRCM_ENOTSUP;
        return RMRCM_OK;
    }
    if (p->sub_nx != 4 && p->sub_nx != 8 && p->sub_nx != 16 && p->sub_nx != 32) return RMRCM_ENOTSUP;
    if (p->sub_ny > 64) return RMRCM_ENOTSUP;
    if (p->precision != RMRCM_FP64 && (!(p->ir_tol > 0) || p->ir_max_iter < 1)) return RMRCM_EINVAL;
    if (p->precision == RMRCM_MIXED_LEARNED) {
        if (!p->cnn_weights || !(p->gate_tol >= 0)) return RMRCM_EINVAL;
        if (p->sub_nx != p->sub_ny || p->sub_nx < 8) return RMRCM_ENOTSUP;
    }
    // the basis block of one subdomain row must fit the local kernel's LDS
    const int R = 2 * (p->sub_nx + p->sub_ny) / piece;
    const size_t lds = sizeof(double) * (size_t)(3 * p->sub_nx * p->sub_nx + 2 * p->sub_nx * R + 4 * p->sub_nx);
    if (lds > 160 * 1024) return RMRCM_ENOTSUP;
    return RMRCM_OK;
}

Geo geo_of(const rmrcm_params& p) {
    Geo g{};
    g.nx = p.nx;
    g.ny = p.ny;
    g.bx = p.sub_nx;
    g.by = p.sub_ny;
    const int su = p.seg_u ? p.seg_u : p.seg, sp = p.seg_p ? p.seg_p : p.seg;
    g.sg = std::min(su, sp);
    g.mu = su / g.sg;
    g.mp = sp / g.sg;
    g.mx = p.nx / p.sub_nx;
    g.my = p.ny / p.sub_ny;
    g.nsx = g.bx / g.sg;
    g.nsy = g.by / g.sg;
    g.lines_v = g.ny / g.sg;
    g.lines_h = g.nx / g.sg;
    g.nv = (g.mx - 1) * g.lines_v;
    g.nseg = g.nv + (g.my - 1) * g.lines_h;
    g.hx = p.lx / p.nx;
    g.hy = p.ly / p.ny;
    g.alpha = p.alpha;
    g.three_d = p.nz > 0 ? 1 : 0;
    g.nz = p.nz > 0 ? p.nz : 1;
    g.hz = p.nz > 0 ? p.lz / p.nz : 1.0;
    return g;
}

void build_geo(rmrcm_ctx* c) { c->geo = geo_of(c->prm); }

// Host tables of every level: node grid, slots, slot codes, merge maps.
void build_levels(rmrcm_ctx* c) {
    const Geo& g = c->geo;
    c->D = ilog2(g.mx) + ilog2(g.my);
    c->levels.assign(c->D + 1, Level());
    int nxn = 1, nyn = 1, sx = g.mx, sy = g.my;
    for (int d = 0; d <= c->D; ++d) {
        Level& L = c->levels[d];
        L.depth = d;
        L.nodes_x = nxn;
        L.nodes_y = nyn;
        L.nnodes = nxn * nyn;
        L.sx = sx;
        L.sy = sy;
        const int hw = sy * g.nsy, hs = sx * g.nsx;
        L.nslot = 2 * (hw + hs);
        L.ld = L.nslot + 1;
        L.h_slotseg.assign((size_t)L.nnodes * L.nslot, -1);
        for (int iy = 0; iy < nyn; ++iy)
            for (int ix = 0; ix < nxn; ++ix) {
                int* s = &L.h_slotseg[(size_t)(iy * nxn + ix) * L.nslot];
                const int I0 = ix * sx, J0 = iy * sy;
                for (int t = 0; t < hw; ++t) {
                    if (I0 > 0) s[t] = rmrcm::slot_code((I0 - 1) * g.lines_v + J0 * g.nsy + t, 0);
                    if (I0 + sx < g.mx)
                        s[hw + t] = rmrcm::slot_code((I0 + sx - 1) * g.lines_v + J0 * g.nsy + t, 1);
                }
                for (int t = 0; t < hs; ++t) {
                    if (J0 > 0)
                        s[2 * hw + t] = rmrcm::slot_code(g.nv + (J0 - 1) * g.lines_h + I0 * g.nsx + t, 0);
                    if (J0 + sy < g.my)
                        s[2 * hw + hs + t] =
                            rmrcm::slot_code(g.nv + (J0 + sy - 1) * g.lines_h + I0 * g.nsx + t, 1);
                }
            }
        if (d == c->D) break;
        // merge of this level from its children: split the side with more
        // subdomains, x on ties
        L.cut = sx >= sy ? 0 : 1;
        L.h_pmap.assign(L.nslot, 0);
        if (L.cut == 0) {
            const int chw = hw, chs = hs / 2;
            L.g = chw;
            for (int t = 0; t < hw; ++t) {
                L.h_pmap[t] = (0 << 24) | t;
                L.h_pmap[hw + t] = (1 << 24) | (chw + t);
            }
            for (int t = 0; t < hs; ++t) {
                L.h_pmap[2 * hw + t] = t < chs ? ((0 << 24) | (2 * chw + t)) : ((1 << 24) | (2 * chw + t - chs));
                L.h_pmap[2 * hw + hs + t] =
                    t < chs ? ((0 << 24) | (2 * chw + chs + t)) : ((1 << 24) | (2 * chw + t));
            }
            L.h_gmap.resize(2 * L.g);
            for (int t = 0; t < L.g; ++t) {
                L.h_gmap[t] = chw + t;   // child 1, E side
                L.h_gmap[L.g + t] = t;   // child 2, W side
            }
            nxn *= 2;
            sx /= 2;
        } else {
            const int chw = hw / 2, chs = hs;
            L.g = chs;
            for (int t = 0; t < hw; ++t) {
                L.h_pmap[t] = t < chw ? ((0 << 24) | t) : ((1 << 24) | (t - chw));
                L.h_pmap[hw + t] = t < chw ? ((0 << 24) | (chw + t)) : ((1 << 24) | t);
            }
            for (int t = 0; t < hs; ++t) {
                L.h_pmap[2 * hw + t] = (0 << 24) | (2 * chw + t);
                L.h_pmap[2 * hw + hs + t] = (1 << 24) | (2 * chw + chs + t);
            }
            L.h_gmap.resize(2 * L.g);
            for (int t = 0; t < L.g; ++t) {
                L.h_gmap[t] = 2 * chw + chs + t;   // child 1, N side
                L.h_gmap[L.g + t] = 2 * chw + t;   // child 2, S side
            }
            nyn *= 2;
            sy /= 2;
        }
        L.xi = 2 * L.g;
    }
}

// Device arrays of every level and of the fused downward pass (no copies:
// upload_levels sends the tables once every array exists).
int alloc_levels(rmrcm_ctx* c) {
    for (int d = 0; d <= c->D; ++d) {
        Level& L = c->levels[d];
        TRY(dalloc(c, &L.slotseg, L.h_slotseg.size()));
        if (d >= 1) TRY(dalloc(c, &L.T, (size_t)L.nnodes * L.nslot * L.ld));
        if (d < c->D) {
            TRY(dalloc(c, &L.pmap, L.h_pmap.size()));
            TRY(dalloc(c, &L.gmap, L.h_gmap.size()));
            // gamma segment t of merge n: the code of gamma slot t in child 1
            const Level& C = c->levels[d + 1];
            L.h_gseg.assign((size_t)L.nnodes * L.g, 0);
            for (int n = 0; n < L.nnodes; ++n) {
                const int ix = n % L.nodes_x, iy = n / L.nodes_x;
                const int c1 = L.cut == 0 ? iy * (2 * L.nodes_x) + 2 * ix : (2 * iy) * L.nodes_x + ix;
                for (int t = 0; t < L.g; ++t)
                    L.h_gseg[(size_t)n * L.g + t] = C.h_slotseg[(size_t)c1 * C.nslot + L.h_gmap[t]] >> 1;
            }
            TRY(dalloc(c, &L.gseg, L.h_gseg.size()));
            TRY(dalloc(c, &L.M, (size_t)L.nnodes * L.xi * L.xi));
            TRY(dalloc(c, &L.X, (size_t)L.nnodes * L.xi * L.ld));
            const size_t wk = rmrcm::merge_work_doubles(c, L);
            if (wk) TRY(dalloc(c, &L.work, wk));
            // 64-slot tiles of every node that hold an active slot or the
            // particular column (the merge products skip the others)
            const int nt = (L.nslot + 1 + 63) / 64;
            L.h_tflag.assign((size_t)L.nnodes * nt, 0);
            for (int n = 0; n < L.nnodes; ++n) {
                for (int s = 0; s < L.nslot; ++s)
                    if (L.h_slotseg[(size_t)n * L.nslot + s] >= 0) L.h_tflag[(size_t)n * nt + s / 64] = 1;
                L.h_tflag[(size_t)n * nt + L.nslot / 64] = 1;
            }
            TRY(dalloc(c, &L.tflag, L.h_tflag.size()));
        }
    }
    // the root level keeps a trace buffer only when it is also the leaf level
    if (c->D == 0) TRY(dalloc(c, &c->levels[0].T, (size_t)c->levels[0].nslot * c->levels[0].ld));
    TRY(rmrcm::build_down_sub(c));
    if (!c->h_down_tab.empty()) TRY(dalloc(c, &c->down_tab, c->h_down_tab.size()));
    return RMRCM_OK;
}

// Every device array of a context built by rmrcm_setup (the surrogate
// network of the learned mode allocates its own).
int alloc_arrays(rmrcm_ctx* c) {
    const Geo& g = c->geo;
    const size_t ncell = geo_ncell(g);
    const size_t nbf = geo_nbf(g);
    const size_t nsub = (size_t)g.mx * g.my;
    const size_t n = (size_t)g.bx * g.by * g.nz;
    const size_t nb = (size_t)g.bx * g.nz;     // cells of one row of a column (the factor's block)
    const int R = c->levels[c->D].nslot;
    TRY(dalloc(c, &c->K, ncell));
    TRY(dalloc(c, &c->bct, nbf));
    TRY(dalloc(c, &c->beta, g.nseg));
    TRY(dalloc(c, &c->seglen, g.nseg));
    TRY(dalloc(c, &c->Pstore, nsub * g.by * nb * nb));
    TRY(dalloc(c, &c->Psi, nsub * R * n));
    TRY(dalloc(c, &c->pbar, nsub * n));
    TRY(dalloc(c, &c->glo, g.nseg));
    TRY(dalloc(c, &c->ghi, g.nseg));
    TRY(dalloc(c, &c->q, ncell));
    TRY(dalloc(c, &c->bcv, nbf));
    TRY(dalloc(c, &c->pout, ncell));
    TRY(dalloc(c, &c->fout, (size_t)geo_nflux(g) * ncell));
    TRY(dalloc(c, &c->Uout, g.nseg));
    TRY(dalloc(c, &c->Pout, g.nseg));
    TRY(dalloc(c, &c->flags, rmrcm::kNumFlags));
    TRY(dalloc(c, &c->gauge, 256));
    TRY(dalloc(c, &c->dscal, 1));
    TRY(dalloc(c, &c->iref_res, 2 * (size_t)g.nseg + 4));
    TRY(dalloc(c, &c->iref_save, 2 * (size_t)g.nseg));
    TRY(dalloc(c, &c->iref_flag, 2));
    if (c->prm.precision != RMRCM_FP64) {
        TRY(dalloc(c, &c->P32, nsub * g.by * g.bx * g.bx));
        TRY(dalloc(c, &c->Wsc, nsub * R * n));
        TRY(dalloc(c, &c->resid, nsub));
        TRY(dalloc(c, &c->pfb, nsub));
        TRY(dalloc(c, &c->fb, nsub));
        TRY(dalloc(c, &c->irst, 4));
        TRY(dalloc(c, &c->irhist, 2 * rmrcm::kIrHist));
    }
    if (c->prm.precision == RMRCM_MIXED_LEARNED) {
        TRY(dalloc(c, &c->lx, nsub * 2 * n));
        TRY(dalloc(c, &c->ly, nsub * R * n));
        TRY(dalloc(c, &c->lint, nsub));
        TRY(dalloc(c, &c->gres, nsub));
    }
    return alloc_levels(c);
}

// The host tables of every level into their device arrays, in stream order.
int upload_levels(rmrcm_ctx* c) {
    auto up = [&](int* dst, const std::vector<int>& src) -> int {
        if (!src.empty())
            HIP_TRY(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
        return RMRCM_OK;
    };
    for (int d = 0; d <= c->D; ++d) {
        const Level& L = c->levels[d];
        TRY(up(L.slotseg, L.h_slotseg));
        if (d < c->D) {
            if (!L.h_tflag.empty())
                HIP_TRY(hipMemcpyAsync(L.tflag, L.h_tflag.data(), L.h_tflag.size(), hipMemcpyHostToDevice,
                                       c->stream));
            TRY(up(L.gseg, L.h_gseg));
            TRY(up(L.pmap, L.h_pmap));
            TRY(up(L.gmap, L.h_gmap));
        }
    }
    TRY(up(c->down_tab, c->h_down_tab));
    return RMRCM_OK;
}

void free_all(rmrcm_ctx* c) {
    // arrays carved from an arena belong to its owner
    const bool own = c->arena == nullptr;
    auto f = [own](void* p) {
        if (p && own) (void)hipFree(p);
    };
    f(c->down_tab);
    f(c->ds_P);
    f(c->ds_q);
    f(c->ds_pb);
    f(c->ds_pin);
    f(c->ds_stage);
    c->down_tab = nullptr;
    for (Level& L : c->levels) {
        f(L.T);
        f(L.slotseg);
        f(L.pmap);
        f(L.gmap);
        f(L.gseg);
        f(L.M);
        f(L.X);
        f(L.work);
        f(L.tflag);
    }
    f(c->K);
    f(c->bct);
    f(c->beta);
    f(c->seglen);
    f(c->Pstore);
    f(c->Psi);
    f(c->pbar);
    f(c->glo);
    f(c->ghi);
    f(c->q);
    f(c->bcv);
    f(c->pout);
    f(c->fout);
    f(c->Uout);
    f(c->Pout);
    f(c->flags);
    f(c->gauge);
    f(c->dscal);
    f(c->iref_res);
    f(c->iref_save);
    f(c->iref_flag);
    f(c->P32);
    f(c->Wsc);
    f(c->resid);
    f(c->pfb);
    f(c->fb);
    f(c->irst);
    f(c->irhist);
    f(c->lx);
    f(c->ly);
    f(c->lint);
    f(c->gres);
    if (c->net) rmrcm_cnn_destroy(c->net);
    c->net = nullptr;
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : c->lev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : {c->ev_ls, c->ev_done, c->ev_aux})
        if (e) (void)hipEventDestroy(e);
    if (c->gstep) (void)hipGraphExecDestroy(c->gstep);
    c->gstep = nullptr;
    if (c->aux) {
        (void)hipStreamSynchronize(c->aux);
        (void)hipStreamDestroy(c->aux);
    }
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
}

int check_flags(rmrcm_ctx* c) {
    int h[rmrcm::kNumFlags] = {};
    HIP_TRY(hipMemcpyAsync(h, c->flags, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (h[rmrcm::FLAG_BAD_PERM] || h[rmrcm::FLAG_BAD_DATA]) return RMRCM_EINVAL;
    if (h[rmrcm::FLAG_LOCAL_SINGULAR] || h[rmrcm::FLAG_MERGE_SINGULAR]) return RMRCM_ESINGULAR;
    if (h[rmrcm::FLAG_NOTCONV]) return RMRCM_ENOTCONV;
    return RMRCM_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return -1.f;
    }
    return ms;
}

bool mixed(const rmrcm_ctx* c) { return c->prm.precision != RMRCM_FP64; }
int mark(rmrcm_ctx* c, int i);

// Refinement passes, enqueued without host synchronisation (so that the
// mixed path can be captured in a graph): ir_max_iter passes of correction
// and residual, each pass returning at once on the device after the largest
// relative residual measured before a correction was within ir_tol.
int refine_loop(rmrcm_ctx* c, int part) {
    HIP_TRY(rmrcm::launch_fill_i32(c, c->irst + 2 * part, 2, 0));
    for (int it = 0; it < c->prm.ir_max_iter; ++it) {
        HIP_TRY(rmrcm::launch_local_refine(c, part, 1));
        HIP_TRY(rmrcm::launch_max_resid(c, part));
    }
    return RMRCM_OK;
}

// Local phase of the mixed-precision mode: FP32 factorisation and basis,
// FP64-residual refinement, FP64 redo of the subdomains that do not reach
// the tolerance, traces.
bool learned(const rmrcm_ctx* c) { return c->prm.precision == RMRCM_MIXED_LEARNED; }

// Learned mode: features of every subdomain, the surrogate's basis, and
// the residual gate (fb = 2 for accepted subdomains, whose basis is then
// the surrogate's; fb = 0 for the others).
int surrogate_basis(rmrcm_ctx* c) {
    const int nsub = c->geo.mx * c->geo.my;
    const size_t n = (size_t)c->geo.bx * c->geo.by;
    const int R = c->levels[c->D].nslot;
    HIP_TRY(rmrcm::launch_features(c, c->lx, c->lint));
    c->net->stream = c->stream;
    for (int k = 0; k < nsub; k += c->net->maxnb) {
        const int nb = nsub - k < c->net->maxnb ? nsub - k : c->net->maxnb;
        HIP_TRY(rmrcm::cnn_forward(c->net, nb, c->lx + (size_t)k * 2 * n, c->ly + (size_t)k * R * n));
    }
    HIP_TRY(rmrcm::launch_gate(c, c->ly, c->lint, c->prm.gate_tol));
    return RMRCM_OK;
}

int mixed_local_setup(rmrcm_ctx* c) {
    const int nsub = c->geo.mx * c->geo.my;
    HIP_TRY(rmrcm::launch_fill_i32(c, c->fb, nsub, 0));
    if (learned(c)) {
        TRY(surrogate_basis(c));
        HIP_TRY(rmrcm::launch_local_setup(c, true, c->fb, 0, 0, 1));   // rejected: factor + basis
        HIP_TRY(rmrcm::launch_local_setup(c, true, c->fb, 2, 0, 0));   // accepted: factor only
    } else {
        HIP_TRY(rmrcm::launch_local_setup(c, true, nullptr, 0, 0));
    }
    TRY(refine_loop(c, 0));
    // subdomains still above ir_tol (only if the refinement did not
    // converge: both kernels return at once otherwise) are redone in FP64
    HIP_TRY(rmrcm::launch_local_refine(c, 0, 0));   // measure only
    HIP_TRY(rmrcm::launch_mark_fallback(c, c->prm.ir_tol));
    HIP_TRY(rmrcm::launch_local_setup(c, false, c->fb, 1, 1));
    HIP_TRY(rmrcm::launch_local_traces(c, 0, c->fb, 0));
    if (learned(c)) HIP_TRY(rmrcm::launch_local_traces(c, 0, c->fb, 2));
    TRY(mark(c, 15));
    HIP_TRY(rmrcm::launch_trace_correct(c, 1, 0));
    return RMRCM_OK;
}

// Event i of the phase timers, unless the work is being captured in a graph
// (the timers then keep the values of the last run outside a graph).
int mark(rmrcm_ctx* c, int i) {
    if (!c->capturing) HIP_TRY(hipEventRecord(c->ev[i], c->stream));
    return RMRCM_OK;
}

// FP64 contexts outside graph capture run the particular chain (local
// particular solves, merges of the particular column below the top) on the
// auxiliary stream, each level after its own setup merge.
bool overlap(const rmrcm_ctx* c) { return c->aux && !c->capturing && !mixed(c) && !c->geo.three_d; }

// Every permeability-dependent step, enqueued on c->stream (no host
// synchronisation in FP64 mode, so that it can be captured in a graph).
// kcopy non-null: the permeability check also copies the permeability there
// (a step reading the caller's array keeps the library's copy current).
int enqueue_setup(rmrcm_ctx* c, double* kcopy = nullptr) {
    TRY(mark(c, 0));
    HIP_TRY(rmrcm::launch_fill_i32(c, c->flags, rmrcm::kNumFlags, 0));
    HIP_TRY(rmrcm::launch_check_beta(c, kcopy));
    TRY(mark(c, 1));
    if (mixed(c)) {
        TRY(mixed_local_setup(c));
    } else {
        HIP_TRY(rmrcm::launch_local_setup(c, false, nullptr, 0, 1));
        TRY(mark(c, 15));
        HIP_TRY(rmrcm::launch_trace_correct(c, 1, 0));
    }
    TRY(mark(c, 2));
    const bool ov = overlap(c);
    if (ov) HIP_TRY(hipEventRecord(c->ev_ls, c->stream));
    for (int d = c->D - 1; d >= 0; --d) {
        HIP_TRY(rmrcm::launch_merge_setup(c, d));
        if (ov && (d == 1 || d == 2)) HIP_TRY(hipEventRecord(c->lev[d], c->stream));
    }
    c->lev_recorded = ov;
    TRY(mark(c, 3));
    return RMRCM_OK;
}

int run_setup(rmrcm_ctx* c, bool wait) {
    TRY(enqueue_setup(c));
    c->setup_recorded = true;
    if (!wait) {
        c->check_pending = true;
        return RMRCM_OK;
    }
    c->check_pending = false;
    return check_flags(c);
}

// One step of iterative refinement of the interface data, enqueued after
// the reconstruction (graph-capturable, no host synchronisation): the
// residuals of eq. 13.2 and 14.2 of every segment from the reconstructed
// fluxes and the Robin data; when the largest of them exceeds
// kIfaceTol times the pressure scale, the device flag runs the particular
// chain once more with the residual shares as the leaf particular traces,
// and the correction it yields is added to the Robin data before the
// reconstruction and the gauge run again.  With the flag clear every
// kernel of that chain returns at once.
constexpr double kIfaceTol = 1e-13;
// one step: at alpha = 1e6 it takes the residual from ~1e-11 to ~1e-15;
// where it gains little (alpha = 1e-6: the residual is the cancellation in
// the fluxes of the nearly-Dirichlet Robin faces) a second one gains
// nothing more.  The flag and maxima arrays hold kIfaceSteps + 1 entries
// (the last for the residual after the steps).
constexpr int kIfaceSteps = 1;

int interface_refine(rmrcm_ctx* c) {
    if (c->D == 0 || c->geo.nseg == 0) return RMRCM_OK;
    double* mx = c->iref_res + 2 * (size_t)c->geo.nseg;
    for (int k = 0; k < kIfaceSteps; ++k) {
        // step k > 0 runs only after step k - 1 ran (its residual kernel
        // is skipped otherwise, and the cleared maxima then clear its flag)
        HIP_TRY(rmrcm::launch_fill_i32(c, c->iref_flag + k, 1, 0));
        HIP_TRY(rmrcm::launch_fill_i32(c, reinterpret_cast<int*>(mx + 2 * k), 4, 0));
        HIP_TRY(rmrcm::launch_iface_resid(c, kIfaceTol, mx + 2 * k, c->iref_flag + k,
                                          k ? c->iref_flag + k - 1 : nullptr));
        c->run_ptr = c->iref_flag + k;
        hipError_t e = rmrcm::launch_iface_inject(c);
        for (int d = c->D - 1; d >= 0 && e == hipSuccess; --d) e = rmrcm::launch_merge_particular(c, d);
        if (e == hipSuccess) e = rmrcm::launch_down_all(c);
        if (e == hipSuccess) e = rmrcm::launch_iface_apply(c);
        if (e == hipSuccess) e = rmrcm::launch_reconstruct(c);
        if (e == hipSuccess && !c->any_dirichlet) e = rmrcm::launch_gauge(c);
        c->run_ptr = nullptr;
        HIP_TRY(e);
    }
    // the residual after the last step, for the statistics (measured only
    // when that step ran; its flag slot is not acted on)
    const int k = kIfaceSteps;
    HIP_TRY(rmrcm::launch_fill_i32(c, c->iref_flag + k, 1, 0));
    HIP_TRY(rmrcm::launch_fill_i32(c, reinterpret_cast<int*>(mx + 2 * k), 4, 0));
    HIP_TRY(rmrcm::launch_iface_resid(c, kIfaceTol, mx + 2 * k, c->iref_flag + k, c->iref_flag + k - 1));
    return RMRCM_OK;
}

// Inputs of a solve into the context's staging buffers.
int solve_inputs(rmrcm_ctx* c, const double* source, const double* bc_value) {
    const size_t ncell = geo_ncell(c->geo);
    const size_t nbf = geo_nbf(c->geo);
    TRY(mark(c, 4));
    if (source) {
        HIP_TRY(hipMemcpyAsync(c->q, source, ncell * sizeof(double), hipMemcpyDefault, c->stream));
    } else {
        HIP_TRY(rmrcm::launch_fill_f64(c, c->q, ncell, 0.0));
    }
    HIP_TRY(hipMemcpyAsync(c->bcv, bc_value, nbf * sizeof(double), hipMemcpyDefault, c->stream));
    TRY(mark(c, 5));
    return RMRCM_OK;
}

// Solve with the particular chain on the auxiliary stream (FP64, see
// overlap): the inputs (after the previous solve has finished with them),
// the local particular solves (after the local setup) and the particular
// column of every merge level below the top (after the setup merges of
// level 2, and of level 1 for that level); the main stream joins for the
// top level, the downward pass and the reconstruction.
int solve_overlapped(rmrcm_ctx* c, const double* source, const double* bc_value) {
    hipStream_t main = c->stream;
    c->stream = c->aux;
    int r = RMRCM_OK;
    hipError_t e = c->done_recorded ? hipStreamWaitEvent(c->aux, c->ev_done, 0) : hipSuccess;
    if (e == hipSuccess) r = solve_inputs(c, source, bc_value);
    if (e == hipSuccess && r == RMRCM_OK && !c->any_dirichlet) e = rmrcm::launch_compat_check(c);
    if (e == hipSuccess && r == RMRCM_OK) e = hipStreamWaitEvent(c->aux, c->ev_ls, 0);
    if (e == hipSuccess && r == RMRCM_OK) e = hipEventRecord(c->ev[13], c->aux);
    if (e == hipSuccess && r == RMRCM_OK) e = rmrcm::launch_local_particular(c, false, nullptr, 0, 1);
    if (e == hipSuccess && r == RMRCM_OK) e = rmrcm::launch_trace_correct(c, 0, 1);
    if (e == hipSuccess && r == RMRCM_OK) e = hipEventRecord(c->ev[14], c->aux);
    // the particular merges of levels 2 and deeper start once the setup
    // merges have reached level 2, that of level 1 after its own: two
    // cross-stream dependencies only (each costs the setup chain, the longer
    // one, a few microseconds)
    for (int d = c->D - 1; d >= 1 && e == hipSuccess && r == RMRCM_OK; --d) {
        if (d == c->D - 1 && d >= 2) e = hipStreamWaitEvent(c->aux, c->lev[2], 0);
        if (d == 1 && e == hipSuccess) e = hipStreamWaitEvent(c->aux, c->lev[1], 0);
        if (e == hipSuccess) e = rmrcm::launch_merge_particular(c, d);
    }
    if (e == hipSuccess && r == RMRCM_OK) e = hipEventRecord(c->ev_aux, c->aux);
    c->stream = main;
    TRY(r);
    HIP_TRY(e);
    HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_aux, 0));
    TRY(mark(c, 6));
    HIP_TRY(rmrcm::launch_merge_particular(c, 0));
    TRY(mark(c, 7));
    HIP_TRY(rmrcm::launch_down_all(c));
    TRY(mark(c, 8));
    HIP_TRY(rmrcm::launch_reconstruct(c));
    if (!c->any_dirichlet) HIP_TRY(rmrcm::launch_gauge(c));
    TRY(mark(c, 9));
    TRY(interface_refine(c));
    TRY(mark(c, 16));
    HIP_TRY(hipEventRecord(c->ev_done, c->stream));
    c->done_recorded = true;
    c->solve_overlapped = true;
    return RMRCM_OK;
}

// Particular solutions, their merges, the top solve, the downward pass and
// the reconstruction, enqueued on c->stream (graph-capturable in FP64 mode).
int enqueue_solve(rmrcm_ctx* c) {
    if (!c->any_dirichlet) HIP_TRY(rmrcm::launch_compat_check(c));
    if (mixed(c)) {
        HIP_TRY(rmrcm::launch_local_particular(c, true, c->fb, 0, 0));
        if (learned(c)) HIP_TRY(rmrcm::launch_local_particular(c, true, c->fb, 2, 0));
        HIP_TRY(rmrcm::launch_local_particular(c, false, c->fb, 1, 1));   // FP64-redone subdomains
        HIP_TRY(rmrcm::launch_fill_i32(c, c->flags + rmrcm::FLAG_PFALLBACK, 1, 0));
        HIP_TRY(rmrcm::launch_fill_i32(c, c->pfb, (size_t)c->geo.mx * c->geo.my, 0));
        TRY(refine_loop(c, 1));
        // particular solutions still above ir_tol (only if the refinement
        // did not converge: these kernels return at once otherwise) are
        // solved again in FP64, with an FP64 factor of their subdomain
        HIP_TRY(rmrcm::launch_local_refine(c, 1, 0));   // measure only
        HIP_TRY(rmrcm::launch_mark_part_fallback(c));
        HIP_TRY(rmrcm::launch_local_setup(c, false, c->pfb, 1, 0, 0));
        HIP_TRY(rmrcm::launch_local_particular(c, false, c->pfb, 1, 1));
        HIP_TRY(rmrcm::launch_local_traces(c, 1, c->fb, 0));
        if (learned(c)) HIP_TRY(rmrcm::launch_local_traces(c, 1, c->fb, 2));
        HIP_TRY(rmrcm::launch_trace_correct(c, 0, 1));
    }
    if (!mixed(c)) {
        HIP_TRY(rmrcm::launch_local_particular(c, false, nullptr, 0, 1));
        HIP_TRY(rmrcm::launch_trace_correct(c, 0, 1));
    }
    TRY(mark(c, 6));
    for (int d = c->D - 1; d >= 0; --d) HIP_TRY(rmrcm::launch_merge_particular(c, d));
    TRY(mark(c, 7));
    HIP_TRY(rmrcm::launch_down_all(c));
    TRY(mark(c, 8));
    HIP_TRY(rmrcm::launch_reconstruct(c));
    if (!c->any_dirichlet) HIP_TRY(rmrcm::launch_gauge(c));
    TRY(mark(c, 9));
    TRY(interface_refine(c));
    TRY(mark(c, 16));
    return RMRCM_OK;
}

// Refactor and solve as one chain on c->stream (the body of a step graph):
// the particular problem is carried as one more column beside the basis,
// through the local sweeps (subdomains 16 or 32 cells wide; otherwise its
// own local solve follows the setup) and every merge below the top, so that
// the particular chain of a separate solve is not needed.  c->K, c->q and
// c->bcv point at the step's inputs; the permeability check also copies the
// permeability to kcopy (the library's own copy, for later calls).
int enqueue_step_fused(rmrcm_ctx* c, double* kcopy) {
    // phase timers outside a graph: setup (beta, local, merges with the
    // particular column), then the top's particular column, the downward
    // pass and the reconstruction (no inputs to upload, no separate local
    // particular solves)
    TRY(mark(c, 0));
    HIP_TRY(rmrcm::launch_fill_i32(c, c->flags, rmrcm::kNumFlags, 0));
    HIP_TRY(rmrcm::launch_check_beta(c, kcopy));
    if (!c->any_dirichlet) HIP_TRY(rmrcm::launch_compat_check(c));
    TRY(mark(c, 1));
    if (rmrcm::local_setup_solves_particular(c, false)) {
        HIP_TRY(rmrcm::launch_local_setup(c, false, nullptr, 0, 1, 1, 1));
    } else {
        HIP_TRY(rmrcm::launch_local_setup(c, false, nullptr, 0, 1));
        HIP_TRY(rmrcm::launch_local_particular(c, false, nullptr, 0, 1));
    }
    TRY(mark(c, 15));
    HIP_TRY(rmrcm::launch_trace_correct(c, 1, 1));
    TRY(mark(c, 2));
    for (int d = c->D - 1; d >= 0; --d) HIP_TRY(rmrcm::launch_merge_setup(c, d, true));
    TRY(mark(c, 3));
    for (int i = 4; i <= 6; ++i) TRY(mark(c, i));
    if (c->D > 0) HIP_TRY(rmrcm::launch_merge_particular(c, 0));   // the top's particular column
    TRY(mark(c, 7));
    HIP_TRY(rmrcm::launch_down_all(c));
    TRY(mark(c, 8));
    HIP_TRY(rmrcm::launch_reconstruct(c));
    if (!c->any_dirichlet) HIP_TRY(rmrcm::launch_gauge(c));
    TRY(mark(c, 9));
    TRY(interface_refine(c));
    TRY(mark(c, 16));
    TRY(mark(c, 10));
    return RMRCM_OK;
}

int solve_outputs(rmrcm_ctx* c, double* pressure, double* flux) {
    const size_t ncell = geo_ncell(c->geo);
    HIP_TRY(hipMemcpyAsync(pressure, c->pout, ncell * sizeof(double), hipMemcpyDefault, c->stream));
    HIP_TRY(hipMemcpyAsync(flux, c->fout, geo_nflux(c->geo) * ncell * sizeof(double), hipMemcpyDefault,
                           c->stream));
    TRY(mark(c, 10));
    return RMRCM_OK;
}

}  // namespace

extern "C" {

void rmrcm_default_params(rmrcm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->lx = 1.0;
    p->ly = 1.0;
    p->alpha = 1.0;
    p->precision = RMRCM_FP64;
    p->ir_tol = 1e-11;
    p->ir_max_iter = 6;
    p->gate_tol = 1e-6;
    p->cnn_weights = nullptr;
    p->device = 0;
    p->lz = 1.0;
}

const char* rmrcm_strerror(int s) {
    switch (s) {
        case RMRCM_OK: return "ok";
        case RMRCM_EINVAL: return "invalid argument";
        case RMRCM_ENOMEM: return "out of memory";
        case RMRCM_EDEVICE: return "HIP device error";
        case RMRCM_ESINGULAR: return "singular local or interface system";
        case RMRCM_ENOTCONV: return "iterative refinement did not converge";
        case RMRCM_ESTATE: return "call out of order";
        case RMRCM_ENOTSUP: return "configuration not supported";
        case RMRCM_ETOOBIG: return "problem exceeds the fixed scratch of the allocation-free step";
    }
    return "unknown status";
}

int rmrcm_plan_bytes(const rmrcm_params* prm, uint64_t* bytes) {
    if (!bytes) return RMRCM_EINVAL;
    *bytes = 0;
    const int v = validate(prm);
    if (v != RMRCM_OK) return v;
    rmrcm_ctx* c = new (std::nothrow) rmrcm_ctx();
    if (!c) return RMRCM_ENOMEM;
    c->prm = *prm;
    c->counting = true;
    build_geo(c);
    build_levels(c);
    const int r = alloc_arrays(c);
    if (r == RMRCM_OK) *bytes = c->device_bytes;
    delete c;
    return r;
}

int rmrcm_setup(const rmrcm_params* prm, const double* perm, const int8_t* bc_type,
                rmrcm_ctx** out) {
    if (!out) return RMRCM_EINVAL;
    *out = nullptr;
    int v = validate(prm);
    if (v != RMRCM_OK) return v;
    if (!perm || !bc_type) return RMRCM_EINVAL;
    if (prm->mem_cap) {
        // the memory plan against the cap before any device work
        uint64_t need = 0;
        if ((v = rmrcm_plan_bytes(prm, &need)) != RMRCM_OK) return v;
        if (need > prm->mem_cap) return RMRCM_ENOMEM;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return RMRCM_EDEVICE;
    }
    if (prm->device < 0 || prm->device >= ndev) return RMRCM_EINVAL;
    if (hipSetDevice(prm->device) != hipSuccess) return RMRCM_EDEVICE;

    const rmrcm::Geo pg = geo_of(*prm);
    const size_t ncell = geo_ncell(pg);
    const size_t nbf = geo_nbf(pg);
    const bool kdev = is_device_ptr(perm), tdev = is_device_ptr(bc_type);
    // Validate the host-side copies before any device work.
    std::vector<int8_t> ht(nbf);
    if (tdev) {
        if (hipMemcpy(ht.data(), bc_type, nbf, hipMemcpyDeviceToHost) != hipSuccess) return RMRCM_EDEVICE;
    } else {
        std::memcpy(ht.data(), bc_type, nbf);
    }
    bool any_dir = false;
    for (int8_t t : ht) {
        if (t != RMRCM_BC_NEUMANN && t != RMRCM_BC_DIRICHLET) return RMRCM_EINVAL;
        any_dir |= t == RMRCM_BC_DIRICHLET;
    }
    std::vector<double> hk;
    if (kdev) {
        hk.resize(ncell);
        if (hipMemcpy(hk.data(), perm, ncell * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            return RMRCM_EDEVICE;
    }
    const double* kp = kdev ? hk.data() : perm;
    for (size_t i = 0; i < ncell; ++i)
        if (!(kp[i] > 0) || !std::isfinite(kp[i])) return RMRCM_EINVAL;

    rmrcm_ctx* c = new (std::nothrow) rmrcm_ctx();
    if (!c) return RMRCM_ENOMEM;
    c->prm = *prm;
    c->device = prm->device;
    c->any_dirichlet = any_dir;
    build_geo(c);
    build_levels(c);
    if (!any_dir && c->D == 0) {
        delete c;
        return RMRCM_ENOTSUP;   // one subdomain with no Dirichlet face: singular local system
    }
    auto fail = [&](int r) {
        free_all(c);
        delete c;
        return r;
    };
    if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(RMRCM_EDEVICE);
    c->stream = c->own_stream;
    for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(RMRCM_EDEVICE);
    // ev_done marks the end of a step (any context) or of an overlapped
    // solve; the auxiliary stream and its events serve the overlapped
    // particular chain of FP64 contexts with merges
    if (hipEventCreateWithFlags(&c->ev_ls, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_aux, hipEventDisableTiming) != hipSuccess)
        return fail(RMRCM_EDEVICE);
    if (prm->precision == RMRCM_FP64 && c->D > 0 && c->D <= 32) {
        if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess)
            return fail(RMRCM_EDEVICE);
        for (int d = 0; d < c->D; ++d)
            if (hipEventCreateWithFlags(&c->lev[d], hipEventDisableTiming) != hipSuccess)
                return fail(RMRCM_EDEVICE);
    }
    int r = RMRCM_OK;
    if ((r = alloc_arrays(c)) != RMRCM_OK) return fail(r);
    if (prm->precision == RMRCM_MIXED_LEARNED) {
        if ((r = rmrcm_cnn_load(prm->cnn_weights, 256, prm->device, &c->net)) != RMRCM_OK) return fail(r);
        if (c->net->S != c->geo.bx || c->net->R != c->levels[c->D].nslot) return fail(RMRCM_EINVAL);
    }
    if ((r = upload_levels(c)) != RMRCM_OK) return fail(r);
    if (hipMemcpyAsync(c->K, perm, ncell * sizeof(double), hipMemcpyDefault, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->bct, ht.data(), nbf, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return fail(RMRCM_EDEVICE);
    c->n_local_solves = 2 * (int64_t)c->geo.nseg + (int64_t)c->geo.mx * c->geo.my;
    if ((r = run_setup(c, true)) != RMRCM_OK) return fail(r);
    *out = c;
    return RMRCM_OK;
}

int rmrcm_refactor(rmrcm_ctx* c, const double* perm) {
    if (!c || !perm) return RMRCM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    const size_t ncell = geo_ncell(c->geo);
    c->solved = false;
    HIP_TRY(hipMemcpyAsync(c->K, perm, ncell * sizeof(double), hipMemcpyDefault, c->stream));
    return run_setup(c, false);
}

int rmrcm_solve(rmrcm_ctx* c, const double* source, const double* bc_value, double* pressure,
                double* flux) {
    if (!c || !bc_value || !pressure || !flux) return RMRCM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    const Geo& g = c->geo;
    const size_t ncell = geo_ncell(g);
    const size_t nbf = geo_nbf(g);
    if (!c->any_dirichlet) {
        // all faces Neumann: the data must be compatible (net source equals
        // the prescribed net outflow)
        std::vector<double> hq, hb(nbf);
        if (source) {
            hq.resize(ncell);
            if (hipMemcpy(hq.data(), source, ncell * sizeof(double), hipMemcpyDefault) != hipSuccess)
                return RMRCM_EDEVICE;
        }
        if (hipMemcpy(hb.data(), bc_value, nbf * sizeof(double), hipMemcpyDefault) != hipSuccess)
            return RMRCM_EDEVICE;
        double s = 0.0, sa = 0.0;
        for (double v : hq) s += v, sa += std::fabs(v);
        for (double v : hb) s -= v, sa += std::fabs(v);
        if (!(std::fabs(s) <= 1e-12 * sa + 1e-300)) return RMRCM_EINVAL;
    }
    c->solve_overlapped = false;
    if (overlap(c) && c->lev_recorded) {
        TRY(solve_overlapped(c, source, bc_value));
    } else {
        TRY(solve_inputs(c, source, bc_value));
        TRY(enqueue_solve(c));
    }
    TRY(solve_outputs(c, pressure, flux));
    c->solve_recorded = true;
    const bool host_out = !is_device_ptr(pressure) || !is_device_ptr(flux);
    c->solved = true;
    if (mixed(c)) c->check_pending = true;   // the refinement's convergence is known on the device
    if (host_out || c->stream == c->own_stream) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        if (c->check_pending) {
            c->check_pending = false;
            return check_flags(c);
        }
    }
    return RMRCM_OK;
}

int rmrcm_sync(rmrcm_ctx* c) {
    if (!c) return RMRCM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (!c->check_pending) return RMRCM_OK;
    c->check_pending = false;
    return check_flags(c);
}

int rmrcm_get_interface(rmrcm_ctx* c, double* U, double* P) {
    if (!c || !U || !P) return RMRCM_EINVAL;
    if (!c->solved) return RMRCM_ESTATE;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    if (c->geo.nseg == 0) return RMRCM_OK;
    HIP_TRY(rmrcm::launch_interface_values(c));
    const size_t b = (size_t)c->geo.nseg * sizeof(double);
    HIP_TRY(hipMemcpyAsync(U, c->Uout, b, hipMemcpyDefault, c->stream));
    HIP_TRY(hipMemcpyAsync(P, c->Pout, b, hipMemcpyDefault, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return RMRCM_OK;
}

int rmrcm_counts(const rmrcm_ctx* c, int64_t* nseg, int64_t* nlocal) {
    if (!c) return RMRCM_EINVAL;
    if (nseg) *nseg = c->geo.nseg;
    if (nlocal) *nlocal = c->n_local_solves;
    return RMRCM_OK;
}

int rmrcm_set_stream(rmrcm_ctx* c, void* s) {
    if (!c) return RMRCM_EINVAL;
    c->stream = s ? (hipStream_t)s : c->own_stream;
    return RMRCM_OK;
}

int rmrcm_get_stats(const rmrcm_ctx* cc, char* json, size_t cap) {
    if (!cc) return RMRCM_EINVAL;
    rmrcm_ctx* c = const_cast<rmrcm_ctx*>(cc);
    // phase times of the last setup and solve, read from their events
    if (c->setup_recorded && hipEventSynchronize(c->ev[3]) == hipSuccess) {
        c->t_setup_ms[0] = elapsed(c->ev[0], c->ev[1]);
        // the local phase and, within it, the trace correction (event 15)
        c->t_setup_ms[1] = elapsed(c->ev[1], c->ev[15]);
        c->t_setup_ms[4] = elapsed(c->ev[15], c->ev[2]);
        c->t_setup_ms[2] = elapsed(c->ev[2], c->ev[3]);
        c->t_setup_ms[3] = elapsed(c->ev[0], c->ev[3]);
    }
    if (c->solve_recorded && hipEventSynchronize(c->ev[10]) == hipSuccess) {
        c->t_solve_ms[0] = elapsed(c->ev[4], c->ev[5]);
        // overlapped solves: the local particular solves run on the
        // auxiliary stream, between events 13 and 14
        c->t_solve_ms[1] = c->solve_overlapped ? elapsed(c->ev[13], c->ev[14]) : elapsed(c->ev[5], c->ev[6]);
        c->t_solve_ms[2] = elapsed(c->ev[6], c->ev[7]);
        c->t_solve_ms[3] = elapsed(c->ev[7], c->ev[8]);
        c->t_solve_ms[4] = elapsed(c->ev[8], c->ev[9]);
        c->t_solve_ms[7] = elapsed(c->ev[9], c->ev[16]);
        c->t_solve_ms[5] = elapsed(c->ev[16], c->ev[10]);
        c->t_solve_ms[6] = elapsed(c->ev[4], c->ev[10]);
    }
    if (mixed(c) && hipStreamSynchronize(c->stream) == hipSuccess) {
        // refinement passes, last residuals, fallbacks and accepted
        // surrogate bases of the last setup and solve, kept on the device
        int h[rmrcm::kNumFlags] = {};
        int st[4] = {};
        double hist[2 * rmrcm::kIrHist] = {};
        if (hipMemcpy(h, c->flags, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(st, c->irst, sizeof(st), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(hist, c->irhist, sizeof(hist), hipMemcpyDeviceToHost) == hipSuccess) {
            c->n_accepted = h[rmrcm::FLAG_ACCEPTED];
            c->n_fallback = h[rmrcm::FLAG_FALLBACK];
            c->n_pfallback = h[rmrcm::FLAG_PFALLBACK];
            c->ir_iters_setup = st[1];
            c->ir_iters_solve = st[3];
            const int k0 = std::min(st[1], rmrcm::kIrHist), k1 = std::min(st[3], rmrcm::kIrHist);
            c->ir_resid_setup = k0 > 0 ? hist[k0 - 1] : 0.0;
            c->ir_resid_solve = k1 > 0 ? hist[rmrcm::kIrHist + k1 - 1] : 0.0;
        } else {
            (void)hipGetLastError();
        }
    }
    // the interface residual before the last refinement check, its
    // pressure scale and whether the refinement ran
    if (c->iref_flag && c->geo.nseg > 0 && c->D > 0 && hipStreamSynchronize(c->stream) == hipSuccess) {
        double m[4] = {};
        int fl[2] = {};
        if (hipMemcpy(m, c->iref_res + 2 * (size_t)c->geo.nseg, sizeof(m), hipMemcpyDeviceToHost) == hipSuccess &&
            hipMemcpy(fl, c->iref_flag, sizeof(fl), hipMemcpyDeviceToHost) == hipSuccess) {
            c->iface_resid = m[1] > 0.0 ? m[0] / m[1] : m[0];
            c->iface_resid_after = fl[0] ? (m[3] > 0.0 ? m[2] / m[3] : m[2]) : 0.0;
            c->iface_refined = fl[0];
        } else {
            (void)hipGetLastError();
        }
    }
    char buf[2048];
    const int n = std::snprintf(
        buf, sizeof(buf),
        "{\"setup_ms\": {\"beta\": %.6f, \"local\": %.6f, \"trace_correct\": %.6f, \"merge\": %.6f, "
        "\"total\": %.6f}, "
        "\"solve_ms\": {\"upload\": %.6f, \"local\": %.6f, \"merge\": %.6f, \"down\": %.6f, "
        "\"reconstruct\": %.6f, \"download\": %.6f, \"total\": %.6f}, "
        "\"levels\": %d, \"nseg\": %d, \"subdomains\": %d, \"local_solves\": %lld, "
        "\"device_bytes\": %zu, \"precision\": %d, \"ir_iters_setup\": %d, "
        "\"ir_iters_solve\": %d, \"ir_resid_setup\": %.3e, \"ir_resid_solve\": %.3e, "
        "\"fp64_fallback_subdomains\": %d, \"surrogate_accepted_subdomains\": %d, "
        "\"gate_tol\": %.3e, \"particular_overlapped\": %s, \"interface_residual\": %.3e, "
        "\"interface_residual_refined\": %.3e, \"interface_refined\": %d, \"refine_ms\": %.6f, "
        "\"fp64_particular_fallback_subdomains\": %d}",
        c->t_setup_ms[0], c->t_setup_ms[1], c->t_setup_ms[4], c->t_setup_ms[2], c->t_setup_ms[3], c->t_solve_ms[0],
        c->t_solve_ms[1], c->t_solve_ms[2], c->t_solve_ms[3], c->t_solve_ms[4], c->t_solve_ms[5],
        c->t_solve_ms[6], c->D, c->geo.nseg, c->geo.mx * c->geo.my, (long long)c->n_local_solves,
        c->device_bytes, c->prm.precision, c->ir_iters_setup, c->ir_iters_solve, c->ir_resid_setup,
        c->ir_resid_solve, c->n_fallback, c->n_accepted, c->prm.gate_tol,
        c->solve_overlapped ? "true" : "false", c->iface_resid, c->iface_resid_after, c->iface_refined,
        c->t_solve_ms[7], c->n_pfallback);
    if (json && cap > 0) {
        std::strncpy(json, buf, cap - 1);
        json[cap - 1] = '\0';
    }
    return n + 1;
}

void rmrcm_destroy(rmrcm_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

// Training pairs for the local-basis surrogate: the network's input
// features of every subdomain (device, FP32 [nsub][2][S][S]), the exact
// local basis from the last setup (host or device, FP64 [nsub][R][S*S]) and
// the interior mask (host, [nsub]).
int rmrcm_export_local(rmrcm_ctx* c, float* features, double* basis, int32_t* interior) {
    if (!c || !features) return RMRCM_EINVAL;
    if (c->geo.bx != c->geo.by) return RMRCM_ENOTSUP;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    const size_t nsub = (size_t)c->geo.mx * c->geo.my;
    const size_t n = (size_t)c->geo.bx * c->geo.by;
    const int R = c->levels[c->D].nslot;
    int* dint = nullptr;
    HIP_TRY(hipMallocAsync((void**)&dint, nsub * sizeof(int), c->stream));
    hipError_t e = rmrcm::launch_features(c, features, dint);
    if (e == hipSuccess && basis)
        e = hipMemcpyAsync(basis, c->Psi, nsub * R * n * sizeof(double), hipMemcpyDefault, c->stream);
    std::vector<int> hi(nsub);
    if (e == hipSuccess) e = hipMemcpyAsync(hi.data(), dint, nsub * sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFreeAsync(dint, c->stream);
    (void)hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return RMRCM_EDEVICE;
    if (interior)
        for (size_t k = 0; k < nsub; ++k) interior[k] = hi[k];
    return RMRCM_OK;
}

int rmrcm_get_gate(rmrcm_ctx* c, double* residual, int32_t* accepted) {
    if (!c || c->prm.precision != RMRCM_MIXED_LEARNED) return RMRCM_EINVAL;
    if (!c->setup_recorded && !c->gstep) return RMRCM_ESTATE;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    const size_t nsub = (size_t)c->geo.mx * c->geo.my;
    std::vector<double> r(nsub);
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(r.data(), c->gres, nsub * sizeof(double), hipMemcpyDeviceToHost));
    for (size_t k = 0; k < nsub; ++k) {
        if (residual) residual[k] = r[k];
        if (accepted) accepted[k] = r[k] <= c->prm.gate_tol ? 1 : 0;
    }
    return RMRCM_OK;
}

// ---------------------------------------------------------------- autotuner
namespace {
std::mutex g_tune_mu;
std::map<std::array<int, 4>, int> g_tune_cache;   // (g, nslot, nnodes, ld) -> column tile
}  // namespace

int rmrcm_autotune(rmrcm_ctx* c) {
    if (!c) return RMRCM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int d = 1; d < c->D; ++d) {
        if (!rmrcm::merge_apply_tunable(c, d)) continue;
        const Level& L = c->levels[d];
        const std::array<int, 4> key{L.g, L.nslot, L.nnodes, L.ld};
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                c->ct_tune[d] = it->second;
                continue;
            }
        }
        int best = 0;
        float bt = 1e30f;
        for (int ct : {16, 32}) {
            HIP_TRY(rmrcm::launch_merge_apply(c, d, ct));      // warm-up
            HIP_TRY(hipEventRecord(c->ev[11], c->stream));
            for (int r = 0; r < 3; ++r) HIP_TRY(rmrcm::launch_merge_apply(c, d, ct));
            HIP_TRY(hipEventRecord(c->ev[12], c->stream));
            HIP_TRY(hipEventSynchronize(c->ev[12]));
            const float ms = elapsed(c->ev[11], c->ev[12]);
            if (ms >= 0.f && ms < bt) {
                bt = ms;
                best = ct;
            }
        }
        c->ct_tune[d] = best;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    return RMRCM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batches
struct rmrcm_batch {
    int device = 0;
    std::vector<rmrcm_ctx*> m;             // members
    std::vector<int> order;                // largest member first
    std::vector<hipGraphExec_t> gsetup;    // per member (null: enqueued eagerly)
    std::vector<hipGraphExec_t> gsolve;
    std::vector<hipStream_t> streams;      // pool
    int nstreams = 1;
    hipStream_t master = nullptr;
    hipEvent_t e[4] = {};                  // refactor start/end, solve start/end
    std::vector<hipEvent_t> done;          // per pool stream
    bool ref_recorded = false, sol_recorded = false;
    int64_t cells = 0, local_solves = 0;
    size_t device_bytes = 0;
    int graphs = 0;
    // Host arrays travel through pinned buffers of each member: inputs are
    // copied there on the host and sent by DMA in stream order (a buffer is
    // rewritten only once its previous DMA has completed); host outputs
    // land there and are copied to the caller's arrays at the next sync.
    struct Stage {
        double* K = nullptr;
        double* q = nullptr;
        double* bcv = nullptr;
        double* p = nullptr;
        double* f = nullptr;
        hipEvent_t in = nullptr;       // after the last DMA out of K / q / bcv
        bool in_pending = false;
        double* user_p = nullptr;      // host outputs to deliver at sync
        double* user_f = nullptr;
    };
    std::vector<Stage> stage;
};

namespace {

constexpr int kMaxStreams = 16;

void batch_free(rmrcm_batch* b) {
    (void)hipSetDevice(b->device);
    if (b->master) (void)hipStreamSynchronize(b->master);
    for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
    for (auto g : b->gsetup)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto g : b->gsolve)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto& st : b->stage) {
        for (double* p : {st.K, st.q, st.bcv, st.p, st.f})
            if (p) (void)hipHostFree(p);
        if (st.in) (void)hipEventDestroy(st.in);
    }
    for (rmrcm_ctx* c : b->m) {
        if (c) c->stream = c->own_stream;
        rmrcm_destroy(c);
    }
    for (hipEvent_t e : b->done)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : b->e)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    if (b->master) (void)hipStreamDestroy(b->master);
    delete b;
}

// Capture one member's enqueued work into an executable graph.
template <typename F>
int capture(rmrcm_ctx* c, hipStream_t cap, F enqueue, hipGraphExec_t* out) {
    *out = nullptr;
    hipStream_t saved = c->stream;
    c->stream = cap;
    c->capturing = true;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
        c->stream = saved;
        c->capturing = false;
        return RMRCM_EDEVICE;
    }
    const int r = enqueue(c);
    const hipError_t e = hipStreamEndCapture(cap, &graph);
    if (e != hipSuccess) report_hip(e, "hipStreamEndCapture", __LINE__);
    c->stream = saved;
    c->capturing = false;
    if (r != RMRCM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (e != hipSuccess) return RMRCM_EDEVICE;
    const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) report_hip(ei, "hipGraphInstantiate", __LINE__);
    (void)hipGraphDestroy(graph);
    return ei == hipSuccess ? RMRCM_OK : RMRCM_EDEVICE;
}

// Fork: every pool stream in use waits for the master; join: the master
// waits for every pool stream.
int fork_streams(rmrcm_batch* b, hipEvent_t start) {
    HIP_TRY(hipEventRecord(start, b->master));
    for (int k = 0; k < b->nstreams; ++k) HIP_TRY(hipStreamWaitEvent(b->streams[k], start, 0));
    return RMRCM_OK;
}

int join_streams(rmrcm_batch* b, hipEvent_t end) {
    for (int k = 0; k < b->nstreams; ++k) {
        HIP_TRY(hipEventRecord(b->done[k], b->streams[k]));
        HIP_TRY(hipStreamWaitEvent(b->master, b->done[k], 0));
    }
    HIP_TRY(hipEventRecord(end, b->master));
    return RMRCM_OK;
}

// Host-to-device copy of a member's input through its pinned buffer (a
// device source is copied directly).
int stage_in(rmrcm_batch::Stage& st, hipStream_t s, double* dst, const double* src, double* pin,
             size_t count) {
    if (is_device_ptr(src)) {
        HIP_TRY(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToDevice, s));
        return RMRCM_OK;
    }
    if (st.in_pending) {
        HIP_TRY(hipEventSynchronize(st.in));
        st.in_pending = false;
    }
    std::memcpy(pin, src, count * sizeof(double));
    HIP_TRY(hipMemcpyAsync(dst, pin, count * sizeof(double), hipMemcpyHostToDevice, s));
    return RMRCM_OK;
}

int stage_in_done(rmrcm_batch::Stage& st, hipStream_t s) {
    HIP_TRY(hipEventRecord(st.in, s));
    st.in_pending = true;
    return RMRCM_OK;
}

// Host outputs of the last solve, once the device has produced them.
int deliver_outputs(rmrcm_batch* b) {
    bool any = false;
    for (auto& st : b->stage) any |= st.user_p || st.user_f;
    if (!any) return RMRCM_OK;
    HIP_TRY(hipStreamSynchronize(b->master));
    for (size_t i = 0; i < b->m.size(); ++i) {
        auto& st = b->stage[i];
        const size_t ncell = (size_t)b->m[i]->geo.nx * b->m[i]->geo.ny;
        if (st.user_p) std::memcpy(st.user_p, st.p, ncell * sizeof(double));
        if (st.user_f) std::memcpy(st.user_f, st.f, 4 * ncell * sizeof(double));
        st.user_p = st.user_f = nullptr;
    }
    return RMRCM_OK;
}

int batch_refactor(rmrcm_batch* b, const double* const* perms) {
    TRY(fork_streams(b, b->e[0]));
    for (size_t r = 0; r < b->order.size(); ++r) {
        const int i = b->order[r];
        rmrcm_ctx* c = b->m[i];
        c->stream = b->streams[r % b->nstreams];
        c->solved = false;
        if (perms && perms[i]) {
            const size_t ncell = (size_t)c->geo.nx * c->geo.ny;
            auto& st = b->stage[i];
            TRY(stage_in(st, c->stream, c->K, perms[i], st.K, ncell));
            TRY(stage_in_done(st, c->stream));
        }
        if (b->gsetup[i]) {
            HIP_TRY(hipGraphLaunch(b->gsetup[i], c->stream));
        } else {
            TRY(enqueue_setup(c));
        }
        c->setup_recorded = !b->gsetup[i];
        c->check_pending = true;
    }
    TRY(join_streams(b, b->e[1]));
    b->ref_recorded = true;
    return RMRCM_OK;
}

int batch_solve(rmrcm_batch* b, const double* const* sources, const double* const* bcv,
                double* const* pressures, double* const* fluxes) {
    TRY(deliver_outputs(b));        // host outputs of a previous solve first
    TRY(fork_streams(b, b->e[2]));
    for (size_t r = 0; r < b->order.size(); ++r) {
        const int i = b->order[r];
        rmrcm_ctx* c = b->m[i];
        auto& st = b->stage[i];
        c->stream = b->streams[r % b->nstreams];
        const size_t ncell = (size_t)c->geo.nx * c->geo.ny;
        const size_t nbf = 2 * (size_t)c->geo.nx + 2 * (size_t)c->geo.ny;
        if (bcv) {
            if (sources && sources[i]) TRY(stage_in(st, c->stream, c->q, sources[i], st.q, ncell));
            else HIP_TRY(rmrcm::launch_fill_f64(c, c->q, ncell, 0.0));
            TRY(stage_in(st, c->stream, c->bcv, bcv[i], st.bcv, nbf));
            TRY(stage_in_done(st, c->stream));
        }
        if (b->gsolve[i]) {
            HIP_TRY(hipGraphLaunch(b->gsolve[i], c->stream));
        } else {
            TRY(enqueue_solve(c));
        }
        if (pressures && fluxes) {
            const bool dp = is_device_ptr(pressures[i]), df = is_device_ptr(fluxes[i]);
            HIP_TRY(hipMemcpyAsync(dp ? pressures[i] : st.p, c->pout, ncell * sizeof(double),
                                   dp ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipMemcpyAsync(df ? fluxes[i] : st.f, c->fout, 4 * ncell * sizeof(double),
                                   df ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
            st.user_p = dp ? nullptr : pressures[i];
            st.user_f = df ? nullptr : fluxes[i];
        }
        c->solve_recorded = !b->gsolve[i];
        c->solved = true;
    }
    TRY(join_streams(b, b->e[3]));
    b->sol_recorded = true;
    return RMRCM_OK;
}

// Pick the number of pool streams by timing one refactor + solve pass of
// the whole batch for each candidate.
int tune_streams(rmrcm_batch* b) {
    const int cands[] = {1, 2, 4, 8, 16};
    int best = b->nstreams;
    float bt = 1e30f;
    for (int ns : cands) {
        if (ns > (int)b->m.size() || ns > kMaxStreams) break;
        b->nstreams = ns;
        for (int rep = 0; rep < 2; ++rep) {     // the first pass warms up
            TRY(batch_refactor(b, nullptr));
            TRY(batch_solve(b, nullptr, nullptr, nullptr, nullptr));
        }
        HIP_TRY(hipEventSynchronize(b->e[3]));
        const float ms = elapsed(b->e[0], b->e[3]);
        if (ms >= 0.f && ms < bt) {
            bt = ms;
            best = ns;
        }
    }
    b->nstreams = best;
    return RMRCM_OK;
}

}  // namespace

extern "C" {

int rmrcm_batch_create(int32_t count, const rmrcm_params* prms, const double* const* perms,
                       const int8_t* const* bc_types, int32_t autotune, rmrcm_batch** out) {
    if (!out) return RMRCM_EINVAL;
    *out = nullptr;
    if (count <= 0 || !prms || !perms || !bc_types) return RMRCM_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (prms[i].device != prms[0].device || !perms[i] || !bc_types[i]) return RMRCM_EINVAL;
        if (prms[i].nz > 0) return RMRCM_ENOTSUP;   // ensembles of 2D problems
    }
    rmrcm_batch* b = new (std::nothrow) rmrcm_batch();
    if (!b) return RMRCM_ENOMEM;
    b->device = prms[0].device;
    b->m.assign(count, nullptr);
    for (int i = 0; i < count; ++i) {
        const int r = rmrcm_setup(&prms[i], perms[i], bc_types[i], &b->m[i]);
        if (r != RMRCM_OK) {
            batch_free(b);
            return r;
        }
        const rmrcm_ctx* c = b->m[i];
        b->cells += (int64_t)c->geo.nx * c->geo.ny;
        b->local_solves += c->n_local_solves;
        b->device_bytes += c->device_bytes;
    }
    if (hipSetDevice(b->device) != hipSuccess) {
        batch_free(b);
        return RMRCM_EDEVICE;
    }
    b->stage.assign(count, rmrcm_batch::Stage());
    for (int i = 0; i < count; ++i) {
        auto& st = b->stage[i];
        const size_t ncell = (size_t)b->m[i]->geo.nx * b->m[i]->geo.ny;
        const size_t nbf = 2 * (size_t)b->m[i]->geo.nx + 2 * (size_t)b->m[i]->geo.ny;
        if (hipHostMalloc((void**)&st.K, ncell * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&st.q, ncell * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&st.bcv, nbf * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&st.p, ncell * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&st.f, 4 * ncell * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&st.in, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            batch_free(b);
            return RMRCM_ENOMEM;
        }
    }
    // largest local work first (cells x subdomain width ~ band-Cholesky flops)
    b->order.resize(count);
    for (int i = 0; i < count; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        const rmrcm_ctx* a = b->m[x];
        const rmrcm_ctx* c = b->m[y];
        return (int64_t)a->geo.nx * a->geo.ny * a->geo.bx > (int64_t)c->geo.nx * c->geo.ny * c->geo.bx;
    });
    auto fail = [&](int r) {
        batch_free(b);
        return r;
    };
    if (hipStreamCreateWithFlags(&b->master, hipStreamNonBlocking) != hipSuccess) return fail(RMRCM_EDEVICE);
    b->streams.assign(kMaxStreams, nullptr);
    b->done.assign(kMaxStreams, nullptr);
    for (int k = 0; k < kMaxStreams; ++k)
        if (hipStreamCreateWithFlags(&b->streams[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&b->done[k]) != hipSuccess)
            return fail(RMRCM_EDEVICE);
    for (auto& e : b->e)
        if (hipEventCreate(&e) != hipSuccess) return fail(RMRCM_EDEVICE);
    if (autotune)
        for (rmrcm_ctx* c : b->m) {
            const int r = rmrcm_autotune(c);
            if (r != RMRCM_OK) return fail(r);
        }
    // graphs of every member (the mixed path's refinement loop runs on the
    // device, without host synchronisation)
    b->gsetup.assign(count, nullptr);
    b->gsolve.assign(count, nullptr);
    for (int i = 0; i < count; ++i) {
        rmrcm_ctx* c = b->m[i];
        int r = capture(c, b->streams[0], [](rmrcm_ctx* cc) { return enqueue_setup(cc); }, &b->gsetup[i]);
        if (r == RMRCM_OK) r = capture(c, b->streams[0], enqueue_solve, &b->gsolve[i]);
        if (r != RMRCM_OK) return fail(r);
        ++b->graphs;
    }
    b->nstreams = count < 4 ? count : 4;
    if (autotune) {
        const int r = tune_streams(b);
        if (r != RMRCM_OK) return fail(r);
    }
    if (hipStreamSynchronize(b->master) != hipSuccess) return fail(RMRCM_EDEVICE);
    for (rmrcm_ctx* c : b->m) c->check_pending = false;
    *out = b;
    return RMRCM_OK;
}

int rmrcm_batch_refactor(rmrcm_batch* b, const double* const* perms) {
    if (!b || !perms) return RMRCM_EINVAL;
    for (size_t i = 0; i < b->m.size(); ++i)
        if (!perms[i]) return RMRCM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return RMRCM_EDEVICE;
    return batch_refactor(b, perms);
}

int rmrcm_batch_solve(rmrcm_batch* b, const double* const* sources, const double* const* bc_values,
                      double* const* pressures, double* const* fluxes) {
    if (!b || !bc_values || !pressures || !fluxes) return RMRCM_EINVAL;
    for (size_t i = 0; i < b->m.size(); ++i)
        if (!bc_values[i] || !pressures[i] || !fluxes[i]) return RMRCM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return RMRCM_EDEVICE;
    return batch_solve(b, sources, bc_values, pressures, fluxes);
}

int rmrcm_batch_sync(rmrcm_batch* b, int32_t* status) {
    if (!b) return RMRCM_EINVAL;
    if (hipSetDevice(b->device) != hipSuccess) return RMRCM_EDEVICE;
    HIP_TRY(hipStreamSynchronize(b->master));
    TRY(deliver_outputs(b));
    int first = RMRCM_OK;
    for (size_t i = 0; i < b->m.size(); ++i) {
        rmrcm_ctx* c = b->m[i];
        c->check_pending = false;
        const int r = check_flags(c);
        if (status) status[i] = r;
        if (first == RMRCM_OK) first = r;
    }
    return first;
}

int rmrcm_batch_get_stats(rmrcm_batch* b, char* json, size_t cap) {
    if (!b) return RMRCM_EINVAL;
    (void)hipSetDevice(b->device);
    float tr = -1.f, ts = -1.f;
    if (b->ref_recorded && hipEventSynchronize(b->e[1]) == hipSuccess) tr = elapsed(b->e[0], b->e[1]);
    if (b->sol_recorded && hipEventSynchronize(b->e[3]) == hipSuccess) ts = elapsed(b->e[2], b->e[3]);
    std::string ct = "[";
    for (size_t i = 0; i < b->m.size(); ++i) {
        const rmrcm_ctx* c = b->m[i];
        ct += i ? ", [" : "[";
        for (int d = 1; d < c->D; ++d) ct += (d > 1 ? ", " : "") + std::to_string(c->ct_tune[d]);
        ct += "]";
    }
    ct += "]";
    std::string buf = "{\"members\": " + std::to_string(b->m.size()) +
                      ", \"streams\": " + std::to_string(b->nstreams) +
                      ", \"graph_members\": " + std::to_string(b->graphs) +
                      ", \"cells\": " + std::to_string(b->cells) +
                      ", \"local_solves\": " + std::to_string(b->local_solves) +
                      ", \"device_bytes\": " + std::to_string(b->device_bytes) +
                      ", \"refactor_ms\": " + std::to_string(tr) +
                      ", \"solve_ms\": " + std::to_string(ts) +
                      ", \"merge_column_tiles\": " + ct + "}";
    if (json && cap > 0) {
        std::strncpy(json, buf.c_str(), cap - 1);
        json[cap - 1] = '\0';
    }
    return (int)buf.size() + 1;
}

void rmrcm_batch_destroy(rmrcm_batch* b) {
    if (b) batch_free(b);
}

// Refactor and solve as one unit (rmrcm.h).  FP64 contexts with all arrays
// in device memory replay a captured graph of the whole step: the setup on
// the context's stream, the particular chain on the auxiliary stream forked
// at the start, the outputs written in place.  The graph is captured again
// when a pointer differs from those of the last capture.
int rmrcm_set_step_graph(rmrcm_ctx* c, int enabled) {
    if (!c) return RMRCM_EINVAL;
    c->step_graph = enabled != 0;
    return RMRCM_OK;
}

int rmrcm_downscale(rmrcm_ctx* c, const double* source, const double* bc_value, const double* pressure,
                    const double* flux, double* pressure_out, double* flux_out) {
    if (!c || !bc_value || !pressure || !flux || !pressure_out || !flux_out) return RMRCM_EINVAL;
    if (c->geo.three_d || c->geo.mu > 1 || c->geo.mp > 1) return RMRCM_ENOTSUP;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    const Geo& g = c->geo;
    const size_t ncell = (size_t)g.nx * g.ny;
    const size_t nbf = 2 * (size_t)g.nx + 2 * (size_t)g.ny;
    const int nsub = g.mx * g.my;
    if (!c->ds_P) {
        // first call: the Neumann factor store and buffers, and the gauge
        // flag of every subdomain without a Dirichlet face
        std::vector<int8_t> ht(nbf);
        HIP_TRY(hipStreamSynchronize(c->stream));
        HIP_TRY(hipMemcpy(ht.data(), c->bct, nbf, hipMemcpyDeviceToHost));
        std::vector<int> pin(nsub, 1);
        for (int J = 0; J < g.my; ++J)
            for (int I = 0; I < g.mx; ++I) {
                bool dir = false;
                for (int j = 0; j < g.by; ++j) {
                    if (I == 0) dir |= ht[J * g.by + j] == RMRCM_BC_DIRICHLET;
                    if (I == g.mx - 1) dir |= ht[g.ny + J * g.by + j] == RMRCM_BC_DIRICHLET;
                }
                for (int i = 0; i < g.bx; ++i) {
                    if (J == 0) dir |= ht[2 * g.ny + I * g.bx + i] == RMRCM_BC_DIRICHLET;
                    if (J == g.my - 1) dir |= ht[2 * g.ny + g.nx + I * g.bx + i] == RMRCM_BC_DIRICHLET;
                }
                pin[J * g.mx + I] = dir ? 0 : 1;
            }
        int r = RMRCM_OK;
        if ((r = dalloc(c, &c->ds_P, (size_t)nsub * g.by * g.bx * g.bx)) ||
            (r = dalloc(c, &c->ds_q, ncell)) || (r = dalloc(c, &c->ds_pb, ncell)) ||
            (r = dalloc(c, &c->ds_pin, nsub)) || (r = dalloc(c, &c->ds_stage, 10 * ncell)))
            return r;
        HIP_TRY(hipMemcpyAsync(c->ds_pin, pin.data(), nsub * sizeof(int), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    // inputs in device memory (host arrays staged)
    const bool pdev = is_device_ptr(pressure), fdev = is_device_ptr(flux);
    const bool podev = is_device_ptr(pressure_out), fodev = is_device_ptr(flux_out);
    double* pin_d = pdev ? const_cast<double*>(pressure) : c->ds_stage;
    double* fin_d = fdev ? const_cast<double*>(flux) : c->ds_stage + ncell;
    double* pout_d = podev ? pressure_out : c->ds_stage + 5 * ncell;
    double* fout_d = fodev ? flux_out : c->ds_stage + 6 * ncell;
    if (!pdev) HIP_TRY(hipMemcpyAsync(pin_d, pressure, ncell * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (!fdev) HIP_TRY(hipMemcpyAsync(fin_d, flux, 4 * ncell * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->bcv, bc_value, nbf * sizeof(double), hipMemcpyDefault, c->stream));
    if (source) HIP_TRY(hipMemcpyAsync(c->q, source, ncell * sizeof(double), hipMemcpyDefault, c->stream));
    HIP_TRY(rmrcm::launch_fill_i32(c, c->flags + rmrcm::FLAG_LOCAL_SINGULAR, 1, 0));
    HIP_TRY(rmrcm::launch_ds_source(c, fin_d, source ? c->q : nullptr, c->ds_q));
    HIP_TRY(rmrcm::launch_ds_compat(c, c->ds_pin, c->ds_q));
    // the Neumann factorisation and solve: the local kernels with the
    // geometry in Neumann mode and the downscaling buffers in place of the
    // factor store, the source and the particular solution
    const Geo g0 = c->geo;
    double* const P0 = c->Pstore;
    double* const q0 = c->q;
    double* const pb0 = c->pbar;
    c->geo.neumann = 1;
    c->geo.pin = c->ds_pin;
    c->Pstore = c->ds_P;
    c->q = c->ds_q;
    c->pbar = c->ds_pb;
    hipError_t e = rmrcm::launch_local_setup(c, false, nullptr, 0, 0, 0, 0);
    if (e == hipSuccess) e = rmrcm::launch_local_particular(c, false, nullptr, 0, 0);
    c->geo = g0;
    c->Pstore = P0;
    c->q = q0;
    c->pbar = pb0;
    HIP_TRY(e);
    HIP_TRY(rmrcm::launch_ds_finish(c, c->ds_pb, pin_d, fin_d, c->ds_pin, pout_d, fout_d));
    if (!podev)
        HIP_TRY(hipMemcpyAsync(pressure_out, pout_d, ncell * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (!fodev)
        HIP_TRY(hipMemcpyAsync(flux_out, fout_d, 4 * ncell * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return check_flags(c);
}

int rmrcm_set_refinement(rmrcm_ctx* c, double ir_tol, int32_t ir_max_iter) {
    if (!c || !(ir_tol > 0) || ir_max_iter < 1) return RMRCM_EINVAL;
    if (!mixed(c)) return RMRCM_ENOTSUP;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    c->prm.ir_tol = ir_tol;
    c->prm.ir_max_iter = ir_max_iter;
    if (c->gstep) {
        // the captured step holds the old pass count and tolerance
        HIP_TRY(hipStreamSynchronize(c->stream));
        (void)hipGraphExecDestroy(c->gstep);
        c->gstep = nullptr;
    }
    return RMRCM_OK;
}

int rmrcm_step(rmrcm_ctx* c, const double* perm, const double* source, const double* bc_value,
               double* pressure, double* flux) {
    if (!c || !perm || !bc_value || !pressure || !flux) return RMRCM_EINVAL;
    if (hipSetDevice(c->device) != hipSuccess) return RMRCM_EDEVICE;
    const bool dev = is_device_ptr(perm) && (!source || is_device_ptr(source)) &&
                     is_device_ptr(bc_value) && is_device_ptr(pressure) && is_device_ptr(flux);
    if (!dev) {
        TRY(rmrcm_refactor(c, perm));
        return rmrcm_solve(c, source, bc_value, pressure, flux);
    }
    // FP64: the fused chain (the particular column carried through the local
    // solves and the merges); mixed modes: the setup followed by the solve,
    // their refinement loops on the device
    auto body = [&](rmrcm_ctx* cc, double* kcopy) -> int {
        if (!mixed(cc)) return enqueue_step_fused(cc, kcopy);
        TRY(enqueue_setup(cc, kcopy));
        TRY(mark(cc, 4));          // no inputs to upload
        TRY(mark(cc, 5));
        TRY(enqueue_solve(cc));
        return mark(cc, 10);       // no outputs to download
    };
    // the step's inputs and outputs in place of the context's own buffers
    double* po = c->pout;
    double* fo = c->fout;
    double* ko = c->K;
    double* qo = c->q;
    double* bo = c->bcv;
    auto point = [&](rmrcm_ctx* cc) -> int {
        // the kernels read the caller's permeability, source and boundary
        // data; the library's copy of the permeability (for later calls) is
        // written by the permeability check
        const size_t ncell = geo_ncell(cc->geo);
        cc->pout = pressure;
        cc->fout = flux;
        cc->K = const_cast<double*>(perm);
        cc->bcv = const_cast<double*>(bc_value);
        if (source) cc->q = const_cast<double*>(source);
        else HIP_TRY(rmrcm::launch_fill_f64(cc, cc->q, ncell, 0.0));
        return RMRCM_OK;
    };
    auto restore = [&]() {
        c->pout = po;
        c->fout = fo;
        c->K = ko;
        c->q = qo;
        c->bcv = bo;
    };
    if (!c->step_graph) {
        int r = point(c);
        if (r == RMRCM_OK) r = body(c, ko);
        restore();
        TRY(r);
        c->setup_recorded = true;
        c->solve_recorded = true;
        c->solve_overlapped = false;
    } else {
        const void* key[5] = {perm, source, bc_value, pressure, flux};
        bool same = c->gstep != nullptr;
        for (int i = 0; i < 5 && same; ++i) same = key[i] == c->gstep_key[i];
        if (!same) {
            if (c->gstep) {
                HIP_TRY(hipStreamSynchronize(c->stream));
                (void)hipGraphExecDestroy(c->gstep);
                c->gstep = nullptr;
            }
            const int r = capture(
                c, c->stream,
                [&](rmrcm_ctx* cc) -> int {
                    TRY(point(cc));
                    return body(cc, ko);
                },
                &c->gstep);
            restore();
            if (r != RMRCM_OK) return r;
            for (int i = 0; i < 5; ++i) c->gstep_key[i] = key[i];
        }
        HIP_TRY(hipGraphLaunch(c->gstep, c->stream));
    }
    HIP_TRY(hipEventRecord(c->ev_done, c->stream));
    c->done_recorded = true;
    c->lev_recorded = false;                // a later solve runs its particular chain in order
    c->solved = true;
    c->check_pending = true;
    if (c->stream == c->own_stream) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        c->check_pending = false;
        return check_flags(c);
    }
    return RMRCM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free step
namespace {

constexpr size_t kScratchBytes = (size_t)RMRCM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Every device array of rmrcm_step_noalloc: one such array per GPU the
// library runs on, created with the code object and held until the process
// ends.  In host code `scratch` names a host-side stand-in, not device
// memory: the device address comes from hipGetSymbolAddress, once per
// device (scratch_address), and only that address is handed to kernels and
// copies.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_noalloc_mu[kMaxDevices];   // one allocation-free step per device at a time

// Device address of this device's scratch (the device must be current).
int scratch_address(int dev, char** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            report_hip(e, "hipGetSymbolAddress(scratch)", __LINE__);
            (void)hipGetLastError();
            return RMRCM_EDEVICE;
        }
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return RMRCM_OK;
}

// The work of rmrcm_step_noalloc once the context is built: carve the
// arrays, zero them, upload the tables, enqueue the fused step chain.
int noalloc_enqueue(rmrcm_ctx* c, const std::vector<int8_t>& ht, const double* perm,
                    const double* source, const double* bc_value, double* pressure, double* flux) {
    const Geo& g = c->geo;
    const size_t ncell = (size_t)g.nx * g.ny;
    const size_t nbf = ht.size();
    const size_t nsub = (size_t)g.mx * g.my;
    const size_t n = (size_t)g.bx * g.by;
    const int R = c->levels[c->D].nslot;
    TRY(dalloc(c, &c->bct, nbf));
    TRY(dalloc(c, &c->beta, g.nseg));
    TRY(dalloc(c, &c->seglen, g.nseg));
    TRY(dalloc(c, &c->Pstore, nsub * g.by * g.bx * g.bx));
    TRY(dalloc(c, &c->Psi, nsub * R * n));
    TRY(dalloc(c, &c->pbar, nsub * n));
    TRY(dalloc(c, &c->glo, g.nseg));
    TRY(dalloc(c, &c->ghi, g.nseg));
    TRY(dalloc(c, &c->flags, rmrcm::kNumFlags));
    TRY(dalloc(c, &c->gauge, 256));
    TRY(dalloc(c, &c->dscal, 1));
    TRY(dalloc(c, &c->iref_res, 2 * (size_t)g.nseg + 4));
    TRY(dalloc(c, &c->iref_save, 2 * (size_t)g.nseg));
    TRY(dalloc(c, &c->iref_flag, 2));
    if (!source) TRY(dalloc(c, &c->q, ncell));   // a zero source
    TRY(alloc_levels(c));
    // every array starts at zero, as hipMalloc'ed arrays do after dalloc
    HIP_TRY(rmrcm::launch_fill_i32(c, reinterpret_cast<int*>(c->arena), c->arena_used / sizeof(int), 0));
    HIP_TRY(hipMemcpyAsync(c->bct, ht.data(), nbf, hipMemcpyHostToDevice, c->stream));
    TRY(upload_levels(c));
    c->K = const_cast<double*>(perm);
    if (source) c->q = const_cast<double*>(source);
    c->bcv = const_cast<double*>(bc_value);
    c->pout = pressure;
    c->fout = flux;
    return enqueue_step_fused(c, nullptr);
}

}  // namespace

extern "C" int rmrcm_step_noalloc(const rmrcm_params* prm, const double* perm, const int8_t* bc_type,
                                  const double* source, const double* bc_value, double* pressure,
                                  double* flux, void* hip_stream) {
    const int v = validate(prm);
    if (v != RMRCM_OK) return v;
    if (prm->precision != RMRCM_FP64) return RMRCM_ENOTSUP;
    if ((prm->seg_u && prm->seg_u != prm->seg) || (prm->seg_p && prm->seg_p != prm->seg)) return RMRCM_ENOTSUP;
    if (prm->nz > 0) return RMRCM_ENOTSUP;
    if (!perm || !bc_type || !bc_value || !pressure || !flux) return RMRCM_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return RMRCM_EDEVICE;
    }
    if (prm->device < 0 || prm->device >= ndev || prm->device >= kMaxDevices) return RMRCM_EINVAL;
    if (hipSetDevice(prm->device) != hipSuccess) return RMRCM_EDEVICE;
    if (!is_device_ptr(perm) || (source && !is_device_ptr(source)) || !is_device_ptr(bc_value) ||
        !is_device_ptr(pressure) || !is_device_ptr(flux))
        return RMRCM_EINVAL;
    const size_t nbf = 2 * (size_t)prm->nx + 2 * (size_t)prm->ny;
    std::vector<int8_t> ht(nbf);
    if (is_device_ptr(bc_type)) {
        if (hipMemcpy(ht.data(), bc_type, nbf, hipMemcpyDeviceToHost) != hipSuccess) return RMRCM_EDEVICE;
    } else {
        std::memcpy(ht.data(), bc_type, nbf);
    }
    bool any_dir = false;
    for (int8_t t : ht) {
        if (t != RMRCM_BC_NEUMANN && t != RMRCM_BC_DIRICHLET) return RMRCM_EINVAL;
        any_dir |= t == RMRCM_BC_DIRICHLET;
    }
    rmrcm_ctx* c = new (std::nothrow) rmrcm_ctx();
    if (!c) return RMRCM_ENOMEM;
    c->prm = *prm;
    c->device = prm->device;
    c->any_dirichlet = any_dir;
    build_geo(c);
    build_levels(c);
    int r = RMRCM_OK;
    if (!any_dir && c->D == 0) r = RMRCM_ENOTSUP;   // one subdomain, no Dirichlet face
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->capturing = true;   // no events, no host waits inside the chain
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu[prm->device]);
        char* base = nullptr;
        if (r == RMRCM_OK) r = scratch_address(prm->device, &base);
        if (r == RMRCM_OK) {
            c->arena = base;
            c->arena_cap = kScratchBytes;
            r = noalloc_enqueue(c, ht, perm, source, bc_value, pressure, flux);
            // the scratch is free for the next call once this stream is idle
            const hipError_t e = hipStreamSynchronize(c->stream);
            if (r == RMRCM_OK && e != hipSuccess) r = RMRCM_EDEVICE;
            if (r == RMRCM_OK) r = check_flags(c);
        }
    }
    free_all(c);
    delete c;
    return r;
}
