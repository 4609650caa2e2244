// Downscaling across the skeleton.
//
// The coarse interface conditions (eq. 13.2, 14.2) hold on segments, so the
// two one-sided fluxes of the MRCM solution through a fine skeleton face
// differ; Section 4 leaves fine-scale conservation to downscaling methods
// from the literature.  This is a local Neumann post-processing:
//   1. every skeleton face between cell a and its neighbour b across the
//      skeleton gets Fbar_ab = (F_a - F_b) / 2 (F_a: a's outward flux,
//      F_b: b's through the same face), so Fbar_ba = -Fbar_ab;
//   2. every subdomain's fine two-point problem is solved again with the
//      source, the outer boundary data and Fbar prescribed on its skeleton
//      faces (the library's FP64 local factorisation in its Neumann mode:
//      no conductance on Robin faces, a gauge face on subdomains without a
//      Dirichlet face, see bface);
//   3. a gauged subdomain's right-hand side loses its mean (the round-off
//      defect of the input's compatibility, k_ds_compat) and its pressure
//      is shifted to the input's subdomain mean;
//   4. fluxes: interior faces by the two-point law from the new pressure,
//      skeleton faces Fbar, outer faces from the boundary data.
// Step 2's right-hand side enters the particular solve as a cell source:
// the source minus the cell's averaged skeleton outflow (k_ds_source).

#include "rmrcm_internal.h"

namespace rmrcm {

__global__ __launch_bounds__(256) void k_ds_source(Geo g, const double* __restrict__ F,
                                                   const double* __restrict__ q, double* __restrict__ qo) {
    const size_t plane = (size_t)g.nx * g.ny;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < plane; t += stride) {
        const int gi = (int)(t % g.nx), gj = (int)(t / g.nx);
        const int i = gi % g.bx, j = gj % g.by;
        double s = 0.0;   // the cell's averaged skeleton outflow, W E S N
        if (i == 0 && gi > 0) s += 0.5 * (F[t] - F[plane + t - 1]);
        if (i == g.bx - 1 && gi < g.nx - 1) s += 0.5 * (F[plane + t] - F[t + 1]);
        if (j == 0 && gj > 0) s += 0.5 * (F[2 * plane + t] - F[3 * plane + t - g.nx]);
        if (j == g.by - 1 && gj < g.ny - 1) s += 0.5 * (F[3 * plane + t] - F[2 * plane + t + g.nx]);
        qo[t] = (q ? q[t] : 0.0) - s;
    }
}

// A gauged subdomain (no Dirichlet face) has a singular Neumann problem whose
// data are compatible only up to the input's own defect (its segment fluxes
// balance to round-off): the mean of the right-hand side over its cells
// (source minus skeleton outflow, minus the prescribed outer outflow) is
// removed from every cell, which is the solution of the bordered system
// with one multiplier; the gauge face then carries no flux beyond rounding.
__global__ __launch_bounds__(256) void k_ds_compat(Geo g, const double* __restrict__ bcv,
                                                   const int* __restrict__ pin, double* __restrict__ qo) {
    __shared__ double red[256];
    const int sub = blockIdx.x, tid = threadIdx.x;
    if (!pin[sub]) return;                        // uniform per workgroup
    const int I = sub % g.mx, J = sub / g.mx;
    const int n = g.bx * g.by;
    double s = 0.0;
    for (int c = tid; c < n; c += 256) {
        const int i = c % g.bx, j = c / g.bx;
        const int gi = I * g.bx + i, gj = J * g.by + j;
        double v = qo[(size_t)gj * g.nx + gi];
        if (gi == 0) v -= bcv[gj];
        if (gi == g.nx - 1) v -= bcv[g.ny + gj];
        if (gj == 0) v -= bcv[2 * g.ny + gi];
        if (gj == g.ny - 1) v -= bcv[2 * g.ny + g.nx + gi];
        s += v;
    }
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double mean = red[0] / (double)n;
    for (int c = tid; c < n; c += 256) {
        const int i = c % g.bx, j = c / g.bx;
        qo[(size_t)(J * g.by + j) * g.nx + I * g.bx + i] -= mean;
    }
}

// Steps 3 and 4 for one subdomain per workgroup (256 threads): pb is the
// Neumann solution in the per-subdomain layout of the particular solves.
template <int BX>
__global__ __launch_bounds__(256) void k_ds_finish(Geo g, const double* __restrict__ K,
                                                   const int8_t* __restrict__ bct,
                                                   const double* __restrict__ bcv,
                                                   const double* __restrict__ pb,
                                                   const double* __restrict__ p_in,
                                                   const double* __restrict__ F_in,
                                                   const int* __restrict__ pin,
                                                   double* __restrict__ p_out,
                                                   double* __restrict__ f_out) {
    extern __shared__ double sm[];
    const int sub = blockIdx.x, tid = threadIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int BY = g.by, n = BX * BY;
    double* ps = sm;            // n: pressures
    double* ks = ps + n;        // n: permeabilities
    double* ra = ks + n;        // 256: partial sums
    double* rb = ra + 256;      // 256
    const double* pbs = pb + (size_t)sub * n;
    double a = 0.0, b = 0.0;
    for (int c = tid; c < n; c += 256) {
        const size_t o = (size_t)(J * BY + c / BX) * g.nx + I * BX + c % BX;
        ps[c] = pbs[c];
        ks[c] = K[o];
        a += ps[c];
        b += p_in[o];
    }
    double shift = 0.0;
    if (pin[sub]) {                               // uniform per workgroup
        ra[tid] = a;
        rb[tid] = b;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) {
                ra[tid] += ra[tid + w];
                rb[tid] += rb[tid + w];
            }
            __syncthreads();
        }
        shift = (rb[0] - ra[0]) / (double)n;
    }
    __syncthreads();
    const size_t plane = (size_t)g.nx * g.ny;
    for (int c = tid; c < n; c += 256) {
        ps[c] += shift;
        p_out[(size_t)(J * BY + c / BX) * g.nx + I * BX + c % BX] = ps[c];
    }
    __syncthreads();
    for (int c = tid; c < n; c += 256) {
        const int i = c % BX, j = c / BX;
        const int gi = I * BX + i, gj = J * BY + j;
        const size_t o = (size_t)gj * g.nx + gi;
        const double p = ps[c];
        double F[4];
#pragma unroll
        for (int side = 0; side < 4; ++side) {
            const bool inside = side == 0 ? i > 0 : side == 1 ? i < BX - 1 : side == 2 ? j > 0 : j < BY - 1;
            const bool outer = side == 0 ? gi == 0 : side == 1 ? gi == g.nx - 1 : side == 2 ? gj == 0
                                                                                              : gj == g.ny - 1;
            const double area = side < 2 ? g.hy : g.hx;
            const double h = side < 2 ? g.hx : g.hy;
            const double rc = h / (2.0 * ks[c]);
            if (inside) {
                const int nc = c + (side == 0 ? -1 : side == 1 ? 1 : side == 2 ? -BX : BX);
                F[side] = area / (rc + h / (2.0 * ks[nc])) * (p - ps[nc]);
            } else if (!outer) {
                const long long d = side == 0 ? -1 : side == 1 ? 1 : side == 2 ? -(long long)g.nx : g.nx;
                const int opp = side ^ 1;           // the neighbour's face: W<->E, S<->N
                F[side] = 0.5 * (F_in[side * plane + o] - F_in[opp * plane + o + d]);
            } else {
                const int f = side == 0 ? gj : side == 1 ? g.ny + gj : side == 2 ? 2 * g.ny + gi
                                                                                   : 2 * g.ny + g.nx + gi;
                F[side] = bct[f] == RMRCM_BC_DIRICHLET ? area / rc * (p - bcv[f]) : bcv[f];
            }
        }
        f_out[o] = F[0];
        f_out[plane + o] = F[1];
        f_out[2 * plane + o] = F[2];
        f_out[3 * plane + o] = F[3];
    }
}

hipError_t launch_ds_source(rmrcm_ctx* c, const double* F, const double* q, double* qo) {
    const size_t plane = (size_t)c->geo.nx * c->geo.ny;
    const size_t nb = (plane + 255) / 256;
    hipLaunchKernelGGL(k_ds_source, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, c->stream, c->geo,
                       F, q, qo);
    return hipGetLastError();
}

hipError_t launch_ds_compat(rmrcm_ctx* c, const int* pin, double* qo) {
    hipLaunchKernelGGL(k_ds_compat, dim3(c->geo.mx * c->geo.my), dim3(256), 0, c->stream, c->geo, c->bcv, pin,
                       qo);
    return hipGetLastError();
}

template <int BX>
static hipError_t ds_finish_bx(rmrcm_ctx* c, const double* pb, const double* p_in, const double* F_in,
                               const int* pin, double* p_out, double* f_out) {
    const int nsub = c->geo.mx * c->geo.my;
    const size_t lds = sizeof(double) * (2 * (size_t)BX * c->geo.by + 512);
    hipError_t e = hipFuncSetAttribute((const void*)k_ds_finish<BX>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ds_finish<BX>, dim3(nsub), dim3(256), lds, c->stream, c->geo, c->K, c->bct, c->bcv,
                       pb, p_in, F_in, pin, p_out, f_out);
    return hipGetLastError();
}

hipError_t launch_ds_finish(rmrcm_ctx* c, const double* pb, const double* p_in, const double* F_in,
                            const int* pin, double* p_out, double* f_out) {
    switch (c->geo.bx) {
        case 4: return ds_finish_bx<4>(c, pb, p_in, F_in, pin, p_out, f_out);
        case 8: return ds_finish_bx<8>(c, pb, p_in, F_in, pin, p_out, f_out);
        case 16: return ds_finish_bx<16>(c, pb, p_in, F_in, pin, p_out, f_out);
        case 32: return ds_finish_bx<32>(c, pb, p_in, F_in, pin, p_out, f_out);
    }
    return hipErrorInvalidValue;
}

}  // namespace rmrcm
