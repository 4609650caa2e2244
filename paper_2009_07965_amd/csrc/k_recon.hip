// Final reconstruction (eq. final, Section 2.2) and flux assembly.
//
// Each finest subdomain gathers the Robin datum of each of its boundary
// slots (the one-sided datum g = P - beta (n_i.n) U of its own side), then
//     p = pbar + sum_a Psi_a g_a
// over its cells, and the four outward integrated fluxes of every cell:
// interior faces by the two-point law, Robin faces by
// |f| (p_c - g) / (rho_c + beta), outer faces by the boundary data.

#include "rmrcm_internal.h"

namespace rmrcm {

__device__ inline double kc(const double* __restrict__ K, const Geo& g, int gi, int gj) {
    return K[(size_t)gj * g.nx + gi];
}

// One thread per cell (up to 1024 per workgroup); the basis sum is unrolled
// so that the loads of a cell's coefficients are in flight together.
template <int BX>
__global__ __launch_bounds__(1024) void k_reconstruct(Geo g, const double* __restrict__ K,
                                                     const int8_t* __restrict__ bct,
                                                     const double* __restrict__ bcv,
                                                     const double* __restrict__ beta,
                                                     const int* __restrict__ slotseg, int R,
                                                     const double* __restrict__ Psi,
                                                     const double* __restrict__ pbar,
                                                     const double* __restrict__ glo,
                                                     const double* __restrict__ ghi,
                                                     double* __restrict__ p_out,
                                                     double* __restrict__ f_out,
                                                     const int* __restrict__ run) {
    if (run && !*run) return;
    extern __shared__ double sm[];
    double* gs = sm;            // R
    double* ps = gs + R;        // BX * BY
    double* ks = ps + BX * g.by;   // BX * BY: the subdomain's permeabilities
    const int sub = blockIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int BY = g.by, n = BX * BY;
    const int* ss = slotseg + (size_t)sub * R;
    for (int a = threadIdx.x; a < R; a += blockDim.x) {
        const int code = ss[a];
        gs[a] = code < 0 ? 0.0 : ((code & 1) ? glo[code >> 1] : ghi[code >> 1]);
    }
    __syncthreads();
    const double* Ps = Psi + (size_t)sub * R * n;
    const double* pb = pbar + (size_t)sub * n;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        double s = pb[c];
#pragma unroll 16
        for (int a = 0; a < R; ++a) s += Ps[(size_t)a * n + c] * gs[a];
        ps[c] = s;
        const int i = c % BX, j = c / BX;
        ks[c] = kc(K, g, I * BX + i, J * BY + j);
        p_out[(size_t)(J * BY + j) * g.nx + I * BX + i] = s;
    }
    __syncthreads();
    const size_t plane = (size_t)g.nx * g.ny;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const int i = c % BX, j = c / BX;
        const int gi = I * BX + i, gj = J * BY + j;
        const double k0 = ks[c];
        const double p = ps[c];
        double F[4];
        for (int side = 0; side < 4; ++side) {
            const bool inside = side == 0 ? i > 0 : side == 1 ? i < BX - 1 : side == 2 ? j > 0 : j < BY - 1;
            const double area = side < 2 ? g.hy : g.hx;
            const double h = side < 2 ? g.hx : g.hy;
            const double rc = h / (2.0 * k0);
            if (inside) {
                const int ni = i + (side == 0 ? -1 : side == 1 ? 1 : 0);
                const int nj = j + (side == 2 ? -1 : side == 3 ? 1 : 0);
                const double rn = h / (2.0 * ks[nj * BX + ni]);
                F[side] = area / (rc + rn) * (p - ps[nj * BX + ni]);
                continue;
            }
            const int t = (side < 2 ? j : i) / g.sg;
            const int a = side == 0 ? t : side == 1 ? g.nsy + t : side == 2 ? 2 * g.nsy + t
                                                                               : 2 * g.nsy + g.nsx + t;
            const int code = ss[a];
            if (code >= 0) {
                F[side] = area / (rc + beta[code >> 1]) * (p - gs[a]);
            } else {
                const int f = side == 0 ? gj : side == 1 ? g.ny + gj : side == 2 ? 2 * g.ny + gi
                                                                                   : 2 * g.ny + g.nx + gi;
                F[side] = bct[f] == RMRCM_BC_DIRICHLET ? area / rc * (p - bcv[f]) : bcv[f];
            }
        }
        const size_t o = (size_t)gj * g.nx + gi;
        f_out[o] = F[0];
        f_out[plane + o] = F[1];
        f_out[2 * plane + o] = F[2];
        f_out[3 * plane + o] = F[3];
    }
}

// Interface values per segment from the two one-sided Robin data:
// P = (g_lo + g_hi) / 2, U = (g_hi - g_lo) / (2 beta).
__global__ void k_interface_values(int nseg, const double* __restrict__ glo,
                                   const double* __restrict__ ghi, const double* __restrict__ beta,
                                   double* __restrict__ U, double* __restrict__ P) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nseg) return;
    P[e] = 0.5 * (glo[e] + ghi[e]);
    U[e] = (ghi[e] - glo[e]) / (2.0 * beta[e]);
}

// Zero-mean gauge of all-Neumann problems: per-block partial sums of the
// pressure, then every block re-adds the partials in the same order (the
// result does not depend on scheduling) and subtracts the mean.
constexpr int kGB = 256;      // blocks of the gauge reduction

__global__ __launch_bounds__(256) void k_pressure_partial(const double* __restrict__ p, size_t n,
                                                          double* __restrict__ part,
                                                          const int* __restrict__ run) {
    if (run && !*run) return;
    __shared__ double s[256];
    double acc = 0.0;
    const size_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const size_t b0 = blockIdx.x * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
    for (size_t t = b0 + threadIdx.x; t < b1; t += blockDim.x) acc += p[t];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_pressure_shift(double* __restrict__ p, size_t n,
                                                        const double* __restrict__ part, int nb,
                                                        double* __restrict__ glo,
                                                        double* __restrict__ ghi, int nseg,
                                                        const int* __restrict__ run) {
    if (run && !*run) return;
    __shared__ double mean;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[b];
        mean = s / (double)n;
    }
    __syncthreads();
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t t = t0; t < n; t += stride) p[t] -= mean;
    // the same constant shifts every Robin datum (fluxes are unchanged)
    for (size_t t = t0; t < (size_t)nseg; t += stride) {
        glo[t] -= mean;
        ghi[t] -= mean;
    }
}

// Plain fills (used instead of memset nodes, so that enqueued work can be
// captured in a graph).
template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ p, size_t n, T v) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) p[t] = v;
}

// Compatibility of all-Neumann data (net source = net prescribed outflow),
// checked on the device: one workgroup, fixed summation order.
__global__ __launch_bounds__(1024) void k_compat(const double* __restrict__ q, size_t ncell,
                                                 const double* __restrict__ bcv, size_t nbf,
                                                 int* __restrict__ flags) {
    __shared__ double s1[1024], s2[1024];
    double a = 0.0, b = 0.0;
    for (size_t t = threadIdx.x; t < ncell; t += 1024) {
        a += q[t];
        b += fabs(q[t]);
    }
    for (size_t t = threadIdx.x; t < nbf; t += 1024) {
        a -= bcv[t];
        b += fabs(bcv[t]);
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) flags[FLAG_BAD_DATA] = (fabs(s1[0]) <= 1e-12 * s2[0] + 1e-300) ? 0 : 1;
}

// ---------------------------------------------------------------- interface refinement
// The recursive elimination applies explicit inverses of the gamma blocks;
// when a block is ill conditioned (large Robin parameters: the paper's
// accuracy runs take alpha = 1e6) the interface data it gives satisfy the
// interface conditions eq. 13.2 and 14.2 only to a few digits.  One step of
// iterative refinement of the whole interface system restores them: the
// residuals of the two conditions at every segment are computed from the
// cells' one-sided fluxes and the Robin data, split into one flux offset
// per side of the segment, and taken through the same recursion as the
// particular column of a solve (leaf particular traces = the offsets,
// particular solutions zero); its Robin data are the correction.  The
// residual of segment e between the low side (flux F_lo out of it, datum
// g_lo) and the high side:
//     r13 = F_lo + F_hi,   r14 = F_lo - F_hi - |e| (g_hi - g_lo) / beta_e
// (eq. 14.2 divided by beta_e, with U = (g_hi - g_lo) / (2 beta_e)); the
// equations of a merge read F_lo + W (g_lo - g_hi) = 0 and
// F_hi + W (g_hi - g_lo) = 0 with W = |e| / (2 beta_e), whose residuals
// are (r13 + r14) / 2 on the low side and (r13 - r14) / 2 on the high side.
// Each residual is measured in pressure units, divided by the sum of its
// segment's Robin face conductances |f| / (rho_f + beta_e) (the one-sided
// fluxes are those conductances times pressure differences); the step runs
// (flag set by k_iface_decide) when the largest of them exceeds tol times
// the pressure scale, the largest |p| of a cell next to the skeleton or
// |g| of a Robin datum.  Both maxima are non-negative doubles, whose bit
// patterns order as unsigned integers: one atomic maximum per wavefront.
__device__ inline void wave_max_u64(unsigned long long* dst, double v) {
    unsigned long long b = __double_as_longlong(v);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(b, o);
        b = t > b ? t : b;
    }
    if ((threadIdx.x & 63) == 0 && b) atomicMax(dst, b);
}

// One segment's one-sided flux sums, Robin conductance sum and largest
// |p| of its cells.
__device__ inline void iface_terms(const Geo& g, const double* __restrict__ K, const double* __restrict__ p,
                                   const double* __restrict__ f, double be, int e, double* flo, double* fhi,
                                   double* sc, double* mag) {
    const size_t plane = geo_ncell(g), layer = (size_t)g.nx * g.ny;
    for (int t = 0; t < g.sg * g.nz; ++t) {
        size_t olo, ohi;
        double area, rlo, rhi;
        int slo, shi;
        const int tz = t / g.sg, ta = t % g.sg;   // layer, face along the line
        if (e < g.nv) {
            const int I = e / g.lines_v + 1, j = (e % g.lines_v) * g.sg + ta;
            olo = tz * layer + (size_t)j * g.nx + I * g.bx - 1;
            ohi = olo + 1;
            area = g.hy * g.hz;
            rlo = g.hx / (2.0 * K[olo]);
            rhi = g.hx / (2.0 * K[ohi]);
            slo = 1;
            shi = 0;
        } else {
            const int r = e - g.nv, J = r / g.lines_h + 1, i = (r % g.lines_h) * g.sg + ta;
            olo = tz * layer + (size_t)(J * g.by - 1) * g.nx + i;
            ohi = olo + g.nx;
            area = g.hx * g.hz;
            rlo = g.hy / (2.0 * K[olo]);
            rhi = g.hy / (2.0 * K[ohi]);
            slo = 3;
            shi = 2;
        }
        *flo += f[slo * plane + olo];
        *fhi += f[shi * plane + ohi];
        *sc += area / (rlo + be) + area / (rhi + be);
        *mag = fmax(*mag, fmax(fabs(p[olo]), fabs(p[ohi])));
    }
}

// Per segment (piece, with general interface spaces): its two residuals
// for the refinement's leaf traces.  The test uses the residuals of the
// equations the method imposes: eq. 13.2 summed over each P-segment and
// eq. 14.2 over each U-segment (one piece each with the MuMM spaces), by
// the first piece of each.
__global__ __launch_bounds__(256) void k_iface_resid(Geo g, const double* __restrict__ K,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ f,
                                                     const double* __restrict__ glo,
                                                     const double* __restrict__ ghi,
                                                     const double* __restrict__ beta,
                                                     const double* __restrict__ seglen,
                                                     double* __restrict__ res,
                                                     unsigned long long* __restrict__ mx,
                                                     const int* __restrict__ run) {
    if (run && !*run) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double ratio = 0.0, mag = 0.0;
    if (e < g.nseg) {
        const int k = e < g.nv ? e % g.lines_v : (e - g.nv) % g.lines_h;
        double flo = 0.0, fhi = 0.0, sc = 0.0;
        iface_terms(g, K, p, f, beta[e], e, &flo, &fhi, &sc, &mag);
        const double gl = glo[e], gh = ghi[e];
        mag = fmax(mag, fmax(fabs(gl), fabs(gh)));
        res[e] = flo + fhi;
        res[g.nseg + e] = flo - fhi - seglen[e] * (gh - gl) / beta[e];
        if (g.mp == 1) ratio = fabs(res[e]) / sc;
        if (g.mu == 1) ratio = fmax(ratio, fabs(res[g.nseg + e]) / sc);
        if (g.mp > 1 && k % g.mp == 0) {        // eq. 13.2 on the P-segment starting here
            double a = 0.0, b = 0.0, s = 0.0, m = 0.0;
            for (int q = 0; q < g.mp; ++q) iface_terms(g, K, p, f, beta[e + q], e + q, &a, &b, &s, &m);
            ratio = fmax(ratio, fabs(a + b) / s);
        }
        if (g.mu > 1 && k % g.mu == 0) {        // eq. 14.2 on the U-segment starting here
            double a = 0.0, b = 0.0, s = 0.0, m = 0.0, u = 0.0;
            for (int q = 0; q < g.mu; ++q) {
                iface_terms(g, K, p, f, beta[e + q], e + q, &a, &b, &s, &m);
                u += seglen[e + q] * (ghi[e + q] - glo[e + q]) / beta[e + q];
            }
            ratio = fmax(ratio, fabs(a - b - u) / s);
        }
    }
    wave_max_u64(mx, ratio);
    wave_max_u64(mx + 1, mag);
}

__global__ void k_iface_decide(const double* __restrict__ mx, double tol, int* __restrict__ flag) {
    if (threadIdx.x == 0) *flag = !(mx[0] <= tol * mx[1]);   // NaN residuals refine too
}

// Leaf particular traces of the refinement: the residual share of each
// active slot's side of its segment; the Robin data saved (the recursion's
// downward pass overwrites them with the correction).
__global__ __launch_bounds__(256) void k_iface_inject(int nsub, int R, const int* __restrict__ slotseg,
                                                      const double* __restrict__ res, int nseg,
                                                      double* __restrict__ T, int ld,
                                                      const double* __restrict__ glo,
                                                      const double* __restrict__ ghi,
                                                      double* __restrict__ gsave,
                                                      const int* __restrict__ flag) {
    if (!*flag) return;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (size_t)nseg) {
        gsave[t] = glo[t];
        gsave[nseg + t] = ghi[t];
    }
    if (t >= (size_t)nsub * R) return;
    const int code = slotseg[t];
    double v = 0.0;
    if (code >= 0) {
        const int e = code >> 1;
        v = (code & 1) ? 0.5 * (res[e] + res[nseg + e]) : 0.5 * (res[e] - res[nseg + e]);
    }
    T[t * ld + ld - 1] = v;
}

// Corrected Robin data: saved data + correction.
__global__ __launch_bounds__(256) void k_iface_apply(int nseg, double* __restrict__ glo,
                                                     double* __restrict__ ghi,
                                                     const double* __restrict__ gsave,
                                                     const int* __restrict__ flag) {
    if (!*flag) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nseg) return;
    glo[t] += gsave[t];
    ghi[t] += gsave[nseg + t];
}

hipError_t launch_iface_resid(rmrcm_ctx* c, double tol, double* mx, int* flag, const int* run) {
    const Geo& g = c->geo;
    if (g.nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iface_resid, dim3((g.nseg + 255) / 256), dim3(256), 0, c->stream, g, c->K, c->pout,
                       c->fout, c->glo, c->ghi, c->beta, c->seglen, c->iref_res,
                       reinterpret_cast<unsigned long long*>(mx), run);
    hipLaunchKernelGGL(k_iface_decide, dim3(1), dim3(64), 0, c->stream, (const double*)mx, tol, flag);
    return hipGetLastError();
}

hipError_t launch_iface_inject(rmrcm_ctx* c) {
    const Level& L = c->levels[c->D];
    const size_t nsub = (size_t)c->geo.mx * c->geo.my;
    const size_t n = nsub * L.nslot > (size_t)c->geo.nseg ? nsub * L.nslot : (size_t)c->geo.nseg;
    hipLaunchKernelGGL(k_iface_inject, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, (int)nsub,
                       L.nslot, L.slotseg, c->iref_res, c->geo.nseg, L.T, L.ld, c->glo, c->ghi, c->iref_save,
                       c->run_ptr);
    return hipGetLastError();
}

hipError_t launch_iface_apply(rmrcm_ctx* c) {
    if (c->geo.nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iface_apply, dim3((c->geo.nseg + 255) / 256), dim3(256), 0, c->stream, c->geo.nseg,
                       c->glo, c->ghi, c->iref_save, c->run_ptr);
    return hipGetLastError();
}

static unsigned fill_blocks(size_t n) {
    const size_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : b > 4096 ? 4096 : b);
}

hipError_t launch_fill_i32(rmrcm_ctx* c, int* p, size_t n, int v) {
    hipLaunchKernelGGL(k_fill<int>, dim3(fill_blocks(n)), dim3(256), 0, c->stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(rmrcm_ctx* c, double* p, size_t n, double v) {
    hipLaunchKernelGGL(k_fill<double>, dim3(fill_blocks(n)), dim3(256), 0, c->stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_compat_check(rmrcm_ctx* c) {
    const size_t ncell = geo_ncell(c->geo);
    const size_t nbf = geo_nbf(c->geo);
    hipLaunchKernelGGL(k_compat, dim3(1), dim3(1024), 0, c->stream, c->q, ncell, c->bcv, nbf, c->flags);
    return hipGetLastError();
}

hipError_t launch_gauge(rmrcm_ctx* c) {
    const size_t n = geo_ncell(c->geo);
    hipLaunchKernelGGL(k_pressure_partial, dim3(kGB), dim3(256), 0, c->stream, c->pout, n, c->gauge,
                       c->run_ptr);
    hipLaunchKernelGGL(k_pressure_shift, dim3(1024), dim3(256), 0, c->stream, c->pout, n, c->gauge, kGB,
                       c->glo, c->ghi, c->geo.nseg, c->run_ptr);
    return hipGetLastError();
}

template <int BX>
static hipError_t recon_bx(rmrcm_ctx* c) {
    const Level& L = c->levels[c->D];
    const int nsub = c->geo.mx * c->geo.my;
    const size_t lds = sizeof(double) * (size_t)(L.nslot + 2 * BX * c->geo.by);
    hipError_t e = hipFuncSetAttribute((const void*)k_reconstruct<BX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int nt = BX * c->geo.by < 1024 ? ((BX * c->geo.by + 63) / 64) * 64 : 1024;
    hipLaunchKernelGGL(k_reconstruct<BX>, dim3(nsub), dim3(nt), lds, c->stream, c->geo, c->K,
                       c->bct, c->bcv, c->beta, L.slotseg, L.nslot, c->Psi, c->pbar, c->glo,
                       c->ghi, c->pout, c->fout, c->run_ptr);
    return hipGetLastError();
}

hipError_t launch_reconstruct(rmrcm_ctx* c) {
    if (c->geo.three_d) return launch_reconstruct3d(c);
    switch (c->geo.bx) {
        case 4: return recon_bx<4>(c);
        case 8: return recon_bx<8>(c);
        case 16: return recon_bx<16>(c);
        case 32: return recon_bx<32>(c);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_interface_values(rmrcm_ctx* c) {
    if (c->geo.nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_interface_values, dim3((c->geo.nseg + 255) / 256), dim3(256), 0, c->stream,
                       c->geo.nseg, c->glo, c->ghi, c->beta, c->Uout, c->Pout);
    return hipGetLastError();
}

}  // namespace rmrcm
