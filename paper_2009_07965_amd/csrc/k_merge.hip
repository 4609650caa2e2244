// Interface merges of the nested hierarchy (Algorithm 1, Section 3.2).
//
// Two children c1 (left / bottom) and c2 (right / top) share the interface
// gamma of g segments.  Each child is summarised by its trace matrix T_c:
// the outward integrated flux through each of its boundary segments per
// unit Robin datum on each segment, plus a particular column.  The
// interface unknowns are taken as the two one-sided Robin data of every
// gamma segment, y1 = P - beta U (seen from c1) and y2 = P + beta U (from
// c2); with U, P the paper's flux and pressure unknowns this is an
// invertible change of variables.  The flux-continuity condition eq. 13.2
// and the flux-definition condition eq. 14.2 on gamma become
//     (T1gg + W) y1 - W y2 = -r1
//     -W y1 + (T2gg + W) y2 = -r2,        W = diag(|e| / (2 beta_e)),
// where r_c collects the child's flux on gamma caused by the parent's
// boundary data (or by its particular solution).  The right-hand side of
// parent column s is the trace column of s in the child that owns s, so
// X = -M^{-1} R gives every parent basis function and the particular
// solution as combinations of the children's (eq. new_bfs, eq. particular),
// and the parent trace follows:
//     T_p[o, s] = T_k[o, s] (if s belongs to child k) + T_k[o, gamma] y_k[:, s].
// M is factored once (LU with partial pivoting) and kept with X for the
// downward pass (the Remark of Section 3.2: coefficients are tracked back to
// the finest level instead of storing coarse basis functions).

#include "rmrcm_internal.h"

namespace rmrcm {

struct MergeArgs {
    int nodes_x, nnodes, cut;
    int g, xi, nslot, ld;       // parent
    int cnslot, cld;            // child
    const double* Tc;           // child traces [cnodes][cnslot][cld]
    const int* css;             // child slot codes
    const int* pmap;            // [nslot]
    const int* gmap;            // [2][g]
    double* M;                  // [nnodes][xi][xi]
    int* piv;                   // [nnodes][xi]
    double* X;                  // [nnodes][xi][ld]
    double* Tp;                 // [nnodes][nslot][ld] (null at the root)
    const double* beta;
    const double* seglen;
    int* flags;
};

__device__ inline void children(const MergeArgs& a, int node, int* c1, int* c2) {
    const int ix = node % a.nodes_x, iy = node / a.nodes_x;
    if (a.cut == 0) {
        *c1 = iy * (2 * a.nodes_x) + 2 * ix;
        *c2 = *c1 + 1;
    } else {
        *c1 = (2 * iy) * a.nodes_x + ix;
        *c2 = (2 * iy + 1) * a.nodes_x + ix;
    }
}

// Interface matrix of every merge of the level.
__global__ __launch_bounds__(256) void k_merge_assemble(MergeArgs a) {
    const int node = blockIdx.x;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    const int* g1 = a.gmap;
    const int* g2 = a.gmap + a.g;
    const int* ss1 = a.css + (size_t)c1 * a.cnslot;
    double* M = a.M + (size_t)node * a.xi * a.xi;
    const int g = a.g;
    for (int t = threadIdx.x; t < a.xi * a.xi; t += blockDim.x) {
        const int r = t / a.xi, c = t % a.xi;
        const int rr = r % g, cc = c % g;
        double v = 0.0;
        double wdiag = 0.0;
        if (rr == cc) {
            const int e = ss1[g1[rr]] >> 1;
            wdiag = a.seglen[e] / (2.0 * a.beta[e]);
        }
        if (r < g && c < g) v = T1[(size_t)g1[r] * a.cld + g1[c]] + wdiag;
        else if (r >= g && c >= g) v = T2[(size_t)g2[rr] * a.cld + g2[cc]] + wdiag;
        else v = -wdiag;
        M[t] = v;
    }
}

// In-place LU with partial pivoting, one workgroup per merge (row swaps
// applied to whole rows, LAPACK getrf convention for piv).
__global__ __launch_bounds__(256) void k_merge_lu(MergeArgs a) {
    const int node = blockIdx.x;
    const int n = a.xi;
    double* M = a.M + (size_t)node * n * n;
    int* piv = a.piv + (size_t)node * n;
    __shared__ double sval[256];
    __shared__ int sidx[256];
    __shared__ int sing;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) sing = 0;
    for (int k = 0; k < n; ++k) {
        // pivot search in column k
        double best = -1.0;
        int bi = k;
        for (int i = k + tid; i < n; i += nt) {
            const double v = fabs(M[(size_t)i * n + k]);
            if (v > best) { best = v; bi = i; }
        }
        sval[tid] = best;
        sidx[tid] = bi;
        __syncthreads();
        for (int s = nt / 2; s > 0; s >>= 1) {
            if (tid < s) {
                if (sval[tid + s] > sval[tid] ||
                    (sval[tid + s] == sval[tid] && sidx[tid + s] < sidx[tid])) {
                    sval[tid] = sval[tid + s];
                    sidx[tid] = sidx[tid + s];
                }
            }
            __syncthreads();
        }
        const int p = sidx[0];
        const double pv = sval[0];
        __syncthreads();
        if (tid == 0) {
            piv[k] = p;
            if (!(pv > 0.0)) sing = 1;
        }
        if (p != k) {
            for (int c = tid; c < n; c += nt) {
                const double t0 = M[(size_t)k * n + c];
                M[(size_t)k * n + c] = M[(size_t)p * n + c];
                M[(size_t)p * n + c] = t0;
            }
        }
        __syncthreads();
        const double d = M[(size_t)k * n + k];
        const double inv = d != 0.0 ? 1.0 / d : 0.0;
        for (int i = k + 1 + tid; i < n; i += nt) M[(size_t)i * n + k] *= inv;
        __syncthreads();
        const int m = n - 1 - k;
        for (int t = tid; t < m * m; t += nt) {
            const int i = k + 1 + t / m, c = k + 1 + t % m;
            M[(size_t)i * n + c] -= M[(size_t)i * n + k] * M[(size_t)k * n + c];
        }
        __syncthreads();
    }
    if (tid == 0 && sing) atomicOr(&a.flags[FLAG_MERGE_SINGULAR], 1);
}

// Right-hand sides (negated) of parent columns [col0, col0 + ncol).  A
// column < nslot is the parent basis column of that slot; col == nslot is
// the particular column.
__global__ __launch_bounds__(256) void k_merge_rhs(MergeArgs a, int col0, int ncol) {
    const int node = blockIdx.x;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    const int* g1 = a.gmap;
    const int* g2 = a.gmap + a.g;
    double* X = a.X + (size_t)node * a.xi * a.ld;
    const int g = a.g;
    for (int t = threadIdx.x; t < a.xi * ncol; t += blockDim.x) {
        const int r = t / ncol, col = col0 + t % ncol;
        const int rr = r % g;
        double v;
        if (col == a.nslot) {
            v = r < g ? T1[(size_t)g1[rr] * a.cld + a.cld - 1] : T2[(size_t)g2[rr] * a.cld + a.cld - 1];
        } else {
            const int pm = a.pmap[col];
            const int k = pm >> 24, o = pm & 0xffffff;
            if (k == 0) v = r < g ? T1[(size_t)g1[rr] * a.cld + o] : 0.0;
            else v = r >= g ? T2[(size_t)g2[rr] * a.cld + o] : 0.0;
        }
        X[(size_t)r * a.ld + col] = -v;
    }
}

// X[:, cols] <- M^{-1} X[:, cols] with the LU factors; one workgroup per
// (merge, chunk of CW columns), the chunk held in LDS.
template <int CW>
__global__ __launch_bounds__(256) void k_merge_solve(MergeArgs a, int col0, int ncol) {
    extern __shared__ double xs[];     // xi x CW
    const int node = blockIdx.x;
    const int cbase = col0 + blockIdx.y * CW;
    const int nc = min(CW, col0 + ncol - cbase);
    if (nc <= 0) return;
    const int n = a.xi;
    const double* M = a.M + (size_t)node * n * n;
    const int* piv = a.piv + (size_t)node * n;
    double* X = a.X + (size_t)node * n * a.ld;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int t = tid; t < n * CW; t += nt) {
        const int r = t / CW, c = t % CW;
        xs[t] = c < nc ? X[(size_t)r * a.ld + cbase + c] : 0.0;
    }
    __syncthreads();
    // row interchanges
    if (tid < CW) {
        for (int k = 0; k < n; ++k) {
            const int p = piv[k];
            if (p != k) {
                const double t0 = xs[k * CW + tid];
                xs[k * CW + tid] = xs[p * CW + tid];
                xs[p * CW + tid] = t0;
            }
        }
    }
    __syncthreads();
    // forward: unit lower
    for (int k = 0; k < n - 1; ++k) {
        const int m = n - 1 - k;
        for (int t = tid; t < m * CW; t += nt) {
            const int i = k + 1 + t / CW, c = t % CW;
            xs[i * CW + c] -= M[(size_t)i * n + k] * xs[k * CW + c];
        }
        __syncthreads();
    }
    // backward: upper
    for (int k = n - 1; k >= 0; --k) {
        const double inv = 1.0 / M[(size_t)k * n + k];
        if (tid < CW) xs[k * CW + tid] *= inv;
        __syncthreads();
        for (int t = tid; t < k * CW; t += nt) {
            const int i = t / CW, c = t % CW;
            xs[i * CW + c] -= M[(size_t)i * n + k] * xs[k * CW + c];
        }
        __syncthreads();
    }
    for (int t = tid; t < n * CW; t += nt) {
        const int r = t / CW, c = t % CW;
        if (c < nc) X[(size_t)r * a.ld + cbase + c] = xs[t];
    }
}

// Parent traces for columns [col0, col0 + ncol): one thread per entry.
__global__ __launch_bounds__(256) void k_merge_trace(MergeArgs a, int col0, int ncol) {
    const int node = blockIdx.x;
    const size_t t = (size_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (t >= (size_t)a.nslot * ncol) return;
    const int o = (int)(t / ncol), col = col0 + (int)(t % ncol);
    int c1, c2;
    children(a, node, &c1, &c2);
    const int pm = a.pmap[o];
    const int k = pm >> 24, oc = pm & 0xffffff;
    const double* Tk = a.Tc + (size_t)(k == 0 ? c1 : c2) * a.cnslot * a.cld + (size_t)oc * a.cld;
    const int* gk = a.gmap + k * a.g;
    const double* X = a.X + (size_t)node * a.xi * a.ld + (size_t)(k * a.g) * a.ld + col;
    double v;
    if (col == a.nslot) {
        v = Tk[a.cld - 1];
    } else {
        const int pc = a.pmap[col];
        v = (pc >> 24) == k ? Tk[pc & 0xffffff] : 0.0;
    }
    for (int i = 0; i < a.g; ++i) v += Tk[gk[i]] * X[(size_t)i * a.ld];
    a.Tp[(size_t)node * a.nslot * a.ld + (size_t)o * a.ld + col] = v;
}

// Downward pass at one level: gamma data y = X [d; 1] from the node's
// boundary data d, written to the low / high Robin data of the gamma
// segments.
struct DownArgs {
    int nodes_x, g, xi, nslot, ld, cut, cnslot;
    const double* X;
    const int* ss;      // node slot codes
    const int* css;     // child slot codes
    const int* gmap;
    double* glo;
    double* ghi;
};

__global__ __launch_bounds__(256) void k_down(DownArgs a) {
    extern __shared__ double dvec[];   // nslot + 1
    const int node = blockIdx.x;
    const int* ss = a.ss + (size_t)node * a.nslot;
    for (int s = threadIdx.x; s < a.nslot; s += blockDim.x) {
        const int code = ss[s];
        dvec[s] = code < 0 ? 0.0 : ((code & 1) ? a.glo[code >> 1] : a.ghi[code >> 1]);
    }
    if (threadIdx.x == 0) dvec[a.nslot] = 1.0;
    __syncthreads();
    const int ix = node % a.nodes_x, iy = node / a.nodes_x;
    const int c1 = a.cut == 0 ? iy * (2 * a.nodes_x) + 2 * ix : (2 * iy) * a.nodes_x + ix;
    const int* ss1 = a.css + (size_t)c1 * a.cnslot;
    const double* X = a.X + (size_t)node * a.xi * a.ld;
    for (int r = threadIdx.x; r < a.xi; r += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < a.ld; ++c) s += X[(size_t)r * a.ld + c] * dvec[c];
        const int rr = r % a.g;
        const int e = ss1[a.gmap[rr]] >> 1;
        if (r < a.g) a.glo[e] = s;
        else a.ghi[e] = s;
    }
}

static MergeArgs make_args(rmrcm_ctx* c, int d) {
    Level& P = c->levels[d];
    Level& C = c->levels[d + 1];
    MergeArgs a;
    a.nodes_x = P.nodes_x;
    a.nnodes = P.nnodes;
    a.cut = P.cut;
    a.g = P.g;
    a.xi = P.xi;
    a.nslot = P.nslot;
    a.ld = P.ld;
    a.cnslot = C.nslot;
    a.cld = C.ld;
    a.Tc = C.T;
    a.css = C.slotseg;
    a.pmap = P.pmap;
    a.gmap = P.gmap;
    a.M = P.M;
    a.piv = P.piv;
    a.X = P.X;
    a.Tp = P.T;
    a.beta = c->beta;
    a.seglen = c->seglen;
    a.flags = c->flags;
    return a;
}

static constexpr int kCW = 16;

static hipError_t solve_cols(rmrcm_ctx* c, const MergeArgs& a, int col0, int ncol) {
    const int nchunk = (ncol + kCW - 1) / kCW;
    const size_t lds = sizeof(double) * (size_t)a.xi * kCW;
    hipError_t e = hipFuncSetAttribute((const void*)k_merge_solve<kCW>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_solve<kCW>, dim3(a.nnodes, nchunk), dim3(256), lds, c->stream, a,
                       col0, ncol);
    return hipGetLastError();
}

hipError_t launch_merge_setup(rmrcm_ctx* c, int d) {
    MergeArgs a = make_args(c, d);
    hipLaunchKernelGGL(k_merge_assemble, dim3(a.nnodes), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_merge_lu, dim3(a.nnodes), dim3(256), 0, c->stream, a);
    if (d == 0) return hipGetLastError();     // the root has no boundary columns
    hipLaunchKernelGGL(k_merge_rhs, dim3(a.nnodes), dim3(256), 0, c->stream, a, 0, a.nslot);
    hipError_t e = solve_cols(c, a, 0, a.nslot);
    if (e != hipSuccess) return e;
    const size_t tot = (size_t)a.nslot * a.nslot;
    hipLaunchKernelGGL(k_merge_trace, dim3(a.nnodes, (unsigned)((tot + 255) / 256)), dim3(256), 0,
                       c->stream, a, 0, a.nslot);
    return hipGetLastError();
}

hipError_t launch_merge_particular(rmrcm_ctx* c, int d) {
    MergeArgs a = make_args(c, d);
    hipLaunchKernelGGL(k_merge_rhs, dim3(a.nnodes), dim3(256), 0, c->stream, a, a.nslot, 1);
    hipError_t e = solve_cols(c, a, a.nslot, 1);
    if (e != hipSuccess) return e;
    if (d == 0) return hipSuccess;
    hipLaunchKernelGGL(k_merge_trace, dim3(a.nnodes, (unsigned)((a.nslot + 255) / 256)), dim3(256),
                       0, c->stream, a, a.nslot, 1);
    return hipGetLastError();
}

hipError_t launch_down(rmrcm_ctx* c, int d) {
    Level& P = c->levels[d];
    Level& C = c->levels[d + 1];
    DownArgs a;
    a.nodes_x = P.nodes_x;
    a.g = P.g;
    a.xi = P.xi;
    a.nslot = P.nslot;
    a.ld = P.ld;
    a.cut = P.cut;
    a.cnslot = C.nslot;
    a.X = P.X;
    a.ss = P.slotseg;
    a.css = C.slotseg;
    a.gmap = P.gmap;
    a.glo = c->glo;
    a.ghi = c->ghi;
    const size_t lds = sizeof(double) * (size_t)(P.nslot + 1);
    hipLaunchKernelGGL(k_down, dim3(P.nnodes), dim3(256), lds, c->stream, a);
    return hipGetLastError();
}

}  // namespace rmrcm
