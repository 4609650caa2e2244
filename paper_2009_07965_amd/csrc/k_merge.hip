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
    int pin;                    // 1 at the root of an all-Neumann problem
};

// Element-wise copy t -> st(t, ld(t)) for t < n over the workgroup, in
// batches of B elements per thread whose loads are all issued before any
// store (independent loads in flight instead of one latency per element).
template <int B, typename Load, typename Store>
__device__ inline void batched(int n, Load ld, Store st) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int t0 = 0; t0 < n; t0 += B * nt) {
        double v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int t = t0 + u * nt + tid;
            v[u] = t < n ? ld(t) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int t = t0 + u * nt + tid;
            if (t < n) st(t, v[u]);
        }
    }
}

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
    const int t0 = blockIdx.y * blockDim.x + threadIdx.x;
    if (t0 >= a.xi * a.xi) return;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    const int* g1 = a.gmap;
    const int* g2 = a.gmap + a.g;
    const int* ss1 = a.css + (size_t)c1 * a.cnslot;
    double* M = a.M + (size_t)node * a.xi * a.xi;
    const int g = a.g;
    {
        const int t = t0;
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
        if (a.pin && r == a.xi - 1) v = c == a.xi - 1 ? 1.0 : 0.0;
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
    const int t0 = blockIdx.y * blockDim.x + threadIdx.x;
    if (t0 >= a.xi * ncol) return;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    const int* g1 = a.gmap;
    const int* g2 = a.gmap + a.g;
    double* X = a.X + (size_t)node * a.xi * a.ld;
    const int g = a.g;
    {
        const int t = t0;
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
        if (a.pin && r == a.xi - 1) v = 0.0;
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

// ---------------------------------------------------------------------------
// Small merges (xi <= 64): one workgroup per merge does everything in LDS.
// Setup mode: assemble M, invert it by Gauss-Jordan elimination with
// partial pivoting (row interchanges, undone as column interchanges at the
// end), store M^{-1}; then for chunks of parent columns: right-hand sides,
// X = -M^{-1} R as a product, coefficients out, parent trace columns.
// Particular mode: reload M^{-1} and process the particular column only.
constexpr int kSX = 64;
constexpr int kSCW = 64;
constexpr int kTR = 64;   // parent trace rows per block

__global__ __launch_bounds__(256) void k_merge_small(MergeArgs a, int mode) {
    __shared__ double M[kSX * (kSX + 1)];
    __shared__ double Rc[kSX * kSCW];
    __shared__ double Tg[kTR * kSX];
    __shared__ double Dt[kTR * kSCW];
    __shared__ int qk[kTR];
    __shared__ double f[kSX];
    __shared__ int piv[kSX];
    __shared__ int sing;
    const int n = a.xi, g = a.g, L = n + 1;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int node = blockIdx.x;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    const int* g1 = a.gmap;
    const int* g2 = a.gmap + g;
    double* Mg = a.M + (size_t)node * n * n;
    double* Xg = a.X + (size_t)node * n * a.ld;
    double* Tp = a.Tp ? a.Tp + (size_t)node * a.nslot * a.ld : nullptr;
    if (tid == 0) sing = 0;

    if (mode == 0) {
        const int* ss1 = a.css + (size_t)c1 * a.cnslot;
        for (int t = tid; t < g; t += nt) {
            const int e = ss1[g1[t]] >> 1;
            f[t] = a.seglen[e] / (2.0 * a.beta[e]);     // W, staged in f
        }
        __syncthreads();
        batched<8>(n * n,
                   [&](int t) {
                       const int r = t / n, c = t % n;
                       if (r < g && c < g) return T1[(size_t)g1[r] * a.cld + g1[c]];
                       if (r >= g && c >= g) return T2[(size_t)g2[r - g] * a.cld + g2[c - g]];
                       return 0.0;
                   },
                   [&](int t, double v) {
                       const int r = t / n, c = t % n;
                       M[r * L + c] = v + ((r % g) == (c % g) ? (((r < g) == (c < g)) ? f[r % g] : -f[r % g]) : 0.0);
                   });
        __syncthreads();
        // All-Neumann problem: the top system is singular (adding a constant
        // to every Robin datum changes no flux); fix the last unknown to 0.
        if (a.pin)
            for (int c = tid; c < n; c += nt) M[(n - 1) * L + c] = c == n - 1 ? 1.0 : 0.0;
        __syncthreads();
        for (int k = 0; k < n; ++k) {
            if (wave == 0) {
                const int r = k + lane;
                double v = r < n ? fabs(M[r * L + k]) : -1.0;
                int idx = r;
                for (int off = 32; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(v, off);
                    const int oi = __shfl_xor(idx, off);
                    if (ov > v || (ov == v && oi < idx)) {
                        v = ov;
                        idx = oi;
                    }
                }
                if (lane == 0) {
                    piv[k] = idx;
                    if (!(v > 0.0)) sing = 1;
                }
            }
            __syncthreads();
            const int p = piv[k];
            const double pv = M[p * L + k];
            const double inv = pv != 0.0 ? 1.0 / pv : 0.0;
            __syncthreads();
            // swap rows k, p and scale the pivot row (its diagonal becomes 1/pv)
            for (int c = tid; c < n; c += nt) {
                const double rk = M[k * L + c], rp = M[p * L + c];
                M[p * L + c] = rk;
                M[k * L + c] = (c == k ? 1.0 : rp) * inv;
            }
            __syncthreads();
            for (int i = tid; i < n; i += nt) f[i] = i == k ? 0.0 : M[i * L + k];
            __syncthreads();
            // rank-one update, thread (ty, tx): rows ty + 4 u, column tx
            if (lane < n) {
                const double mk = M[k * L + lane];
                for (int i = wave; i < n; i += 4) {
                    if (i == k) continue;
                    const double base = lane == k ? 0.0 : M[i * L + lane];
                    M[i * L + lane] = base - f[i] * mk;
                }
            }
            __syncthreads();
        }
        // undo the row interchanges as column interchanges, in reverse order
        for (int k = n - 1; k >= 0; --k) {
            const int p = piv[k];
            if (p != k)
                for (int i = tid; i < n; i += nt) {
                    const double t0 = M[i * L + k];
                    M[i * L + k] = M[i * L + p];
                    M[i * L + p] = t0;
                }
            __syncthreads();
        }
        for (int t = tid; t < n * n; t += nt) Mg[t] = M[(t / n) * L + t % n];
        if (tid == 0 && sing) atomicOr(&a.flags[FLAG_MERGE_SINGULAR], 1);
        if (!Tp) return;   // the root: no boundary columns
    } else {
        batched<16>(n * n, [&](int t) { return Mg[t]; },
                    [&](int t, double v) { M[(t / n) * L + t % n] = v; });
        __syncthreads();
    }

    const int col_begin = mode == 0 ? 0 : a.nslot;
    const int col_end = mode == 0 ? a.nslot : a.nslot + 1;
    for (int c0 = col_begin; c0 < col_end; c0 += kSCW) {
        const int nc = min(kSCW, col_end - c0);
        // right-hand sides R (not negated)
        batched<8>(n * kSCW,
                   [&](int t) {
                       const int r = t / kSCW, cc = t % kSCW, col = c0 + cc;
                       const int rr = r % g;
                       if (cc >= nc) return 0.0;
                       if (a.pin && r == n - 1) return 0.0;
                       if (col == a.nslot)
                           return r < g ? T1[(size_t)g1[rr] * a.cld + a.cld - 1]
                                        : T2[(size_t)g2[rr] * a.cld + a.cld - 1];
                       const int pm = a.pmap[col];
                       const int k = pm >> 24, o = pm & 0xffffff;
                       if (k == 0) return r < g ? T1[(size_t)g1[rr] * a.cld + o] : 0.0;
                       return r >= g ? T2[(size_t)g2[rr] * a.cld + o] : 0.0;
                   },
                   [&](int t, double v) { Rc[t] = v; });
        __syncthreads();
        // X = -M^{-1} R, kept in registers until every thread has read Rc
        constexpr int kIt = kSX * kSCW / 256;
        double xv[kIt];
        // thread (wave, lane): rows wave + 4 u, column lane
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int r = wave + 4 * it;
            double s = 0.0;
            if (r < n && lane < nc)
                for (int k = 0; k < n; ++k) s += M[r * L + k] * Rc[k * kSCW + lane];
            xv[it] = -s;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kIt; ++it) {
            const int r = wave + 4 * it;
            if (r < n && lane < nc) {
                Rc[r * kSCW + lane] = xv[it];
                Xg[(size_t)r * a.ld + c0 + lane] = xv[it];
            }
        }
        __syncthreads();
        if (Tp) {
            // parent trace rows in blocks of kTR: gamma columns of the owning
            // child's trace row staged in LDS, then a product with X
            for (int o0 = 0; o0 < a.nslot; o0 += kTR) {
                const int nr = min(kTR, a.nslot - o0);
                batched<8>(nr * g,
                           [&](int t) {
                               const int q = t / g, i = t % g;
                               const int pm = a.pmap[o0 + q];
                               const int k = pm >> 24, oc = pm & 0xffffff;
                               const double* Tk = (k == 0 ? T1 : T2) + (size_t)oc * a.cld;
                               return Tk[(k == 0 ? g1 : g2)[i]];
                           },
                           [&](int t, double v) { Tg[(t / g) * kSX + t % g] = v; });
                __syncthreads();
                // direct terms: the owning child's own entry, staged in Dt
                batched<8>(nr * kSCW,
                           [&](int t) {
                               const int q = t >> 6, cc = t & (kSCW - 1), col = c0 + cc;
                               if (cc >= nc) return 0.0;
                               const int pm = a.pmap[o0 + q];
                               const int k = pm >> 24, oc = pm & 0xffffff;
                               const double* Tk = (k == 0 ? T1 : T2) + (size_t)oc * a.cld;
                               if (col == a.nslot) return Tk[a.cld - 1];
                               const int pc = a.pmap[col];
                               return (pc >> 24) == k ? Tk[pc & 0xffffff] : 0.0;
                           },
                           [&](int t, double v) { Dt[t] = v; });
                for (int q = wave; q < nr; q += 4) qk[q] = a.pmap[o0 + q] >> 24;
                __syncthreads();
                for (int q = wave; q < nr; q += 4) {
                    const int cc = lane, o = o0 + q, col = c0 + cc;
                    if (cc >= nc) continue;
                    const int k = qk[q];
                    double v = Dt[q * kSCW + cc];
                    const double* xk = Rc + (k * g) * kSCW + cc;
                    const double* tg = Tg + q * kSX;
                    for (int i = 0; i < g; ++i) v += tg[i] * xk[i * kSCW];
                    Tp[(size_t)o * a.ld + col] = v;
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Large merges (64 < xi <= 256): blocked right-looking LU with partial
// pivoting, one workgroup of 512 threads per merge, the matrix in global
// memory (L2-resident).  Per 32-column panel: the panel is factored in LDS,
// its row interchanges are applied to the other columns as one composed
// permutation, the block row of U comes from a triangular solve in
// registers and the trailing matrix is updated by a register-tiled product.
constexpr int kNB = 32;
constexpr int kBX = 256;   // largest xi of this path

constexpr int kLUT = 512;   // threads of the blocked LU

__global__ __launch_bounds__(kLUT) void k_merge_lu_blocked(MergeArgs a) {
    extern __shared__ double sm[];
    const int n = a.xi;
    constexpr int PL = kNB + 1;
    double* Pn = sm;                    // n x PL panel
    double* Us = Pn + (size_t)n * PL;   // kNB x (n - kNB) block row of U
    __shared__ double rv[16];
    __shared__ int ri[16];
    __shared__ int pl[kNB];
    __shared__ int perm[kBX];
    __shared__ int ptmp[kBX];
    __shared__ int rowsrc[kBX];
    __shared__ int moved[2 * kNB];
    __shared__ int wcnt[kLUT / 64];
    __shared__ int nmoved;
    __shared__ int sing;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int node = blockIdx.x;
    double* M = a.M + (size_t)node * n * n;
    int* piv = a.piv + (size_t)node * n;
    if (tid == 0) sing = 0;
    for (int i = tid; i < n; i += nt) rowsrc[i] = i;
    for (int kb0 = 0; kb0 < n; kb0 += kNB) {
        const int nb = min(kNB, n - kb0), r = n - kb0;
        __syncthreads();
        batched<16>(r * kNB,
                    [&](int t) {
                        const int i = t >> 5, j = t & (kNB - 1);
                        return j < nb ? M[(size_t)(kb0 + i) * n + kb0 + j] : 0.0;
                    },
                    [&](int t, double v) { Pn[(t >> 5) * PL + (t & (kNB - 1))] = v; });
        __syncthreads();
        for (int j = 0; j < nb; ++j) {
            const int cand = r - j;
            if (tid < ((cand + 63) & ~63)) {
                double v = tid < cand ? fabs(Pn[(j + tid) * PL + j]) : -1.0;
                int idx = j + tid;
                for (int off = 32; off > 0; off >>= 1) {
                    const double ov = __shfl_xor(v, off);
                    const int oi = __shfl_xor(idx, off);
                    if (ov > v || (ov == v && oi < idx)) {
                        v = ov;
                        idx = oi;
                    }
                }
                if (lane == 0) {
                    rv[wave] = v;
                    ri[wave] = idx;
                }
            }
            __syncthreads();
            if (tid == 0) {
                const int nw = (cand + 63) / 64;
                double bv = rv[0];
                int bi = ri[0];
                for (int w = 1; w < nw; ++w)
                    if (rv[w] > bv || (rv[w] == bv && ri[w] < bi)) {
                        bv = rv[w];
                        bi = ri[w];
                    }
                pl[j] = bi;
                if (!(bv > 0.0)) sing = 1;
            }
            __syncthreads();
            const int p = pl[j];
            if (p != j && tid < nb) {
                const double t0 = Pn[j * PL + tid];
                Pn[j * PL + tid] = Pn[p * PL + tid];
                Pn[p * PL + tid] = t0;
            }
            __syncthreads();
            const double d = Pn[j * PL + j];
            const double inv = d != 0.0 ? 1.0 / d : 0.0;
            for (int i = j + 1 + tid; i < r; i += nt) Pn[i * PL + j] *= inv;
            __syncthreads();
            {
                const int c = tid & (kNB - 1);
                if (c > j && c < nb) {
                    const double pjc = Pn[j * PL + c];
                    for (int i = j + 1 + (tid >> 5); i < r; i += kLUT / kNB)
                        Pn[i * PL + c] -= Pn[i * PL + j] * pjc;
                }
            }
            __syncthreads();
        }
        for (int t = tid; t < r * nb; t += nt) {
            const int i = t / nb, j = t % nb;
            M[(size_t)(kb0 + i) * n + kb0 + j] = Pn[i * PL + j];
        }
        // The panel's interchanges compose to one permutation of rows
        // kb0..n-1 that moves at most 2 nb rows; apply it to the columns
        // outside the panel with independent loads, then stores.
        for (int i = tid; i < r; i += nt) perm[i] = i;
        if (tid == 0) nmoved = 0;
        __syncthreads();
        if (tid == 0)
            for (int j = 0; j < nb; ++j) {
                const int p = pl[j];
                const int t0 = perm[j];
                perm[j] = perm[p];
                perm[p] = t0;
            }
        __syncthreads();
        // moved rows, listed in increasing order (ballot per wave)
        for (int i0 = 0; i0 < r; i0 += nt) {
            const int i = i0 + tid;
            const bool mv = i < r && perm[i] != i;
            const unsigned long long bal = __ballot(mv);
            const int before = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) wcnt[wave] = __popcll(bal);
            __syncthreads();
            int off = nmoved;
            for (int w = 0; w < wave; ++w) off += wcnt[w];
            if (mv) moved[off + before] = i;
            __syncthreads();
            if (tid == 0) {
                int s = 0;
                for (int w = 0; w < nt / 64; ++w) s += wcnt[w];
                nmoved += s;
            }
            __syncthreads();
        }
        // row of the original matrix now held by each row
        for (int i = tid; i < r; i += nt) ptmp[i] = rowsrc[kb0 + perm[i]];
        __syncthreads();
        for (int i = tid; i < r; i += nt) rowsrc[kb0 + i] = ptmp[i];
        __syncthreads();
        {
            // at most 2 kNB moved rows x (kBX - kNB) columns
            constexpr int kIt = 2 * kNB * (kBX - kNB) / kLUT;
            const int nm = nmoved, ncol = n - nb;
            double vals[kIt];
#pragma unroll
            for (int it = 0; it < kIt; ++it) {
                const int t = tid + it * kLUT;
                vals[it] = 0.0;
                if (t < nm * ncol) {
                    const int q = t / ncol, cc = t % ncol;
                    const int c = cc < kb0 ? cc : cc + nb;
                    vals[it] = M[(size_t)(kb0 + perm[moved[q]]) * n + c];
                }
            }
            __syncthreads();
#pragma unroll
            for (int it = 0; it < kIt; ++it) {
                const int t = tid + it * kLUT;
                if (t < nm * ncol) {
                    const int q = t / ncol, cc = t % ncol;
                    const int c = cc < kb0 ? cc : cc + nb;
                    M[(size_t)(kb0 + moved[q]) * n + c] = vals[it];
                }
            }
        }
        __syncthreads();
        const int C = n - kb0 - nb;
        if (C <= 0) continue;
        // block row of U: unit-lower solve with the panel's L11, in LDS
        batched<16>(nb * C, [&](int t) { return M[(size_t)(kb0 + t / C) * n + kb0 + nb + t % C]; },
                    [&](int t, double v) { Us[t] = v; });
        __syncthreads();
        // one column of U12 per thread (columns are independent: no barrier)
        for (int cc = tid; cc < C; cc += nt)
            for (int jj = 0; jj < nb - 1; ++jj) {
                const double xj = Us[jj * C + cc];
                for (int i = jj + 1; i < nb; ++i) Us[i * C + cc] -= Pn[i * PL + jj] * xj;
            }
        __syncthreads();
        for (int jj = 0; jj < nb; ++jj)
            for (int cc = tid; cc < C; cc += nt) M[(size_t)(kb0 + jj) * n + kb0 + nb + cc] = Us[jj * C + cc];
        __syncthreads();
        // trailing update: M[kb0+nb+i][kb0+nb+cc] -= L21 * U12, 8x4 tiles per thread
        const int R = r - nb;
        const int ty = tid >> 5, tx = tid & 31;   // 16 x 32 threads
        for (int ib = 0; ib < R; ib += 128)
            for (int jb = 0; jb < C; jb += 128) {
                double acc[8][4];
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
                for (int j = 0; j < nb; ++j) {
                    double av[8], bv[4];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int row = ib + ty + 16 * u;
                        av[u] = row < R ? Pn[(nb + row) * PL + j] : 0.0;
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int col = jb + tx + 32 * v;
                        bv[v] = col < C ? Us[j * C + col] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[u][v] += av[u] * bv[v];
                }
                double old[8][4];
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = ib + ty + 16 * u, col = jb + tx + 32 * v;
                        old[u][v] = (row < R && col < C)
                                        ? M[(size_t)(kb0 + nb + row) * n + kb0 + nb + col] : 0.0;
                    }
#pragma unroll
                for (int u = 0; u < 8; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = ib + ty + 16 * u, col = jb + tx + 32 * v;
                        if (row < R && col < C)
                            M[(size_t)(kb0 + nb + row) * n + kb0 + nb + col] = old[u][v] - acc[u][v];
                    }
            }
    }
    __syncthreads();
    // piv holds the full row permutation: row i of L U is row piv[i] of M
    for (int i = tid; i < n; i += nt) piv[i] = rowsrc[i];
    if (tid == 0 && sing) atomicOr(&a.flags[FLAG_MERGE_SINGULAR], 1);
}

// Column solves with the blocked LU factors: X[:, cols] <- M^{-1} X[:, cols].
// One workgroup per (merge, chunk of kTCW columns); 32-row blocks of L and U
// staged in LDS; diagonal blocks solved in registers by one thread per
// column, the rest as a block product.
constexpr int kTCW = 16;

constexpr int kTT = 1024;   // threads of the blocked column solve

__global__ __launch_bounds__(kTT) void k_merge_trsm(MergeArgs a, int col0, int ncol) {
    extern __shared__ double sm[];
    const int n = a.xi;
    double* xs = sm;                       // n x kTCW
    double* Bk = xs + (size_t)n * kTCW;    // n x kNB block column of L or U
    const int node = blockIdx.x;
    const int cbase = col0 + blockIdx.y * kTCW;
    const int nc = min(kTCW, col0 + ncol - cbase);
    if (nc <= 0) return;
    const double* M = a.M + (size_t)node * n * n;
    double* X = a.X + (size_t)node * n * a.ld;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int* pv = a.piv + (size_t)node * n;   // full row permutation
    batched<4>(n * kTCW,
               [&](int t) {
                   const int r = t / kTCW, c = t % kTCW;
                   return c < nc ? X[(size_t)pv[r] * a.ld + cbase + c] : 0.0;
               },
               [&](int t, double v) { xs[t] = v; });
    // forward, unit lower
    for (int kb0 = 0; kb0 < n; kb0 += kNB) {
        const int nb = min(kNB, n - kb0), rows = n - kb0;
        __syncthreads();
        {
            // rows x nb <= kBX x kNB = 8 x kTT entries, all loads issued first
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = tid + u * kTT;
                v[u] = t < rows * nb ? M[(size_t)(kb0 + t / nb) * n + kb0 + t % nb] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = tid + u * kTT;
                if (t < rows * nb) Bk[(t / nb) * kNB + t % nb] = v[u];
            }
        }
        __syncthreads();
        if (tid < kTCW) {
            double x[kNB];
#pragma unroll
            for (int j = 0; j < kNB; ++j) x[j] = j < nb ? xs[(kb0 + j) * kTCW + tid] : 0.0;
#pragma unroll
            for (int j = 0; j < kNB; ++j)
#pragma unroll
                for (int i = j + 1; i < kNB; ++i)
                    if (i < nb) x[i] -= Bk[i * kNB + j] * x[j];
#pragma unroll
            for (int j = 0; j < kNB; ++j)
                if (j < nb) xs[(kb0 + j) * kTCW + tid] = x[j];
        }
        __syncthreads();
        for (int t = tid; t < (rows - nb) * kTCW; t += nt) {
            const int i = nb + t / kTCW, c = t % kTCW;
            double s = 0.0;
            for (int j = 0; j < nb; ++j) s += Bk[i * kNB + j] * xs[(kb0 + j) * kTCW + c];
            xs[(kb0 + i) * kTCW + c] -= s;
        }
    }
    // backward, upper
    const int last = ((n - 1) / kNB) * kNB;
    for (int kb0 = last; kb0 >= 0; kb0 -= kNB) {
        const int nb = min(kNB, n - kb0), rows = kb0 + nb;
        __syncthreads();
        {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = tid + u * kTT;
                v[u] = t < rows * nb ? M[(size_t)(t / nb) * n + kb0 + t % nb] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = tid + u * kTT;
                if (t < rows * nb) Bk[(t / nb) * kNB + t % nb] = v[u];
            }
        }
        __syncthreads();
        if (tid < kTCW) {
            double x[kNB];
#pragma unroll
            for (int j = 0; j < kNB; ++j) x[j] = j < nb ? xs[(kb0 + j) * kTCW + tid] : 0.0;
#pragma unroll
            for (int j = kNB - 1; j >= 0; --j) {
                if (j < nb) {
                    x[j] /= Bk[(kb0 + j) * kNB + j];
#pragma unroll
                    for (int i = 0; i < j; ++i) x[i] -= Bk[(kb0 + i) * kNB + j] * x[j];
                }
            }
#pragma unroll
            for (int j = 0; j < kNB; ++j)
                if (j < nb) xs[(kb0 + j) * kTCW + tid] = x[j];
        }
        __syncthreads();
        for (int t = tid; t < kb0 * kTCW; t += nt) {
            const int i = t / kTCW, c = t % kTCW;
            double s = 0.0;
            for (int j = 0; j < nb; ++j) s += Bk[i * kNB + j] * xs[(kb0 + j) * kTCW + c];
            xs[i * kTCW + c] -= s;
        }
    }
    __syncthreads();
    for (int t = tid; t < n * kTCW; t += nt) {
        const int r = t / kTCW, c = t % kTCW;
        if (c < nc) X[(size_t)r * a.ld + cbase + c] = xs[t];
    }
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
    for (int s = threadIdx.x; s <= a.nslot; s += blockDim.x) {
        double v = 1.0;      // particular column
        if (s < a.nslot) {
            const int code = ss[s];
            v = code < 0 ? 0.0 : ((code & 1) ? a.glo[code >> 1] : a.ghi[code >> 1]);
        }
        dvec[s] = v;
    }
    __syncthreads();
    const int ix = node % a.nodes_x, iy = node / a.nodes_x;
    const int c1 = a.cut == 0 ? iy * (2 * a.nodes_x) + 2 * ix : (2 * iy) * a.nodes_x + ix;
    const int* ss1 = a.css + (size_t)c1 * a.cnslot;
    const double* X = a.X + (size_t)node * a.xi * a.ld;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int r = blockIdx.y * nw + wave;
    if (r >= a.xi) return;
    double s = 0.0;
    const double* xr = X + (size_t)r * a.ld;
    for (int q0 = 0; q0 < a.ld; q0 += 256) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * 64 + lane;
            v[u] = q < a.ld ? xr[q] * dvec[q] : 0.0;
        }
        s += (v[0] + v[1]) + (v[2] + v[3]);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) {
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
    a.pin = (d == 0 && !c->any_dirichlet) ? 1 : 0;
    return a;
}

static constexpr int kCW = 16;

// Generic column solve (any xi, factors read from global memory step by step).
static hipError_t solve_cols_generic(rmrcm_ctx* c, const MergeArgs& a, int col0, int ncol) {
    const int nchunk = (ncol + kCW - 1) / kCW;
    const size_t lds = sizeof(double) * (size_t)a.xi * kCW;
    hipError_t e = hipFuncSetAttribute((const void*)k_merge_solve<kCW>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_solve<kCW>, dim3(a.nnodes, nchunk), dim3(256), lds, c->stream, a,
                       col0, ncol);
    return hipGetLastError();
}

static hipError_t solve_cols_blocked(rmrcm_ctx* c, const MergeArgs& a, int col0, int ncol) {
    const int nchunk = (ncol + kTCW - 1) / kTCW;
    const size_t lds = sizeof(double) * (size_t)a.xi * (kTCW + kNB);
    hipError_t e = hipFuncSetAttribute((const void*)k_merge_trsm,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_trsm, dim3(a.nnodes, nchunk), dim3(kTT), lds, c->stream, a, col0,
                       ncol);
    return hipGetLastError();
}

static hipError_t lu_blocked(rmrcm_ctx* c, const MergeArgs& a) {
    const size_t lds = sizeof(double) * ((size_t)a.xi * (kNB + 1) + (size_t)kNB * (a.xi - kNB));
    hipError_t e = hipFuncSetAttribute((const void*)k_merge_lu_blocked,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_lu_blocked, dim3(a.nnodes), dim3(kLUT), lds, c->stream, a);
    return hipGetLastError();
}

hipError_t launch_merge_setup(rmrcm_ctx* c, int d) {
    MergeArgs a = make_args(c, d);
    if (d == 0) a.Tp = nullptr;
    if (a.xi <= kSX) {
        hipLaunchKernelGGL(k_merge_small, dim3(a.nnodes), dim3(256), 0, c->stream, a, 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_merge_assemble, dim3(a.nnodes, (a.xi * a.xi + 255) / 256), dim3(256), 0,
                       c->stream, a);
    hipError_t e;
    if (a.xi <= kBX) {
        e = lu_blocked(c, a);
    } else {
        hipLaunchKernelGGL(k_merge_lu, dim3(a.nnodes), dim3(256), 0, c->stream, a);
        e = hipGetLastError();
    }
    if (e != hipSuccess || d == 0) return e;     // the root has no boundary columns
    hipLaunchKernelGGL(k_merge_rhs, dim3(a.nnodes, (a.xi * a.nslot + 255) / 256), dim3(256), 0,
                       c->stream, a, 0, a.nslot);
    e = a.xi <= kBX ? solve_cols_blocked(c, a, 0, a.nslot) : solve_cols_generic(c, a, 0, a.nslot);
    if (e != hipSuccess) return e;
    const size_t tot = (size_t)a.nslot * a.nslot;
    hipLaunchKernelGGL(k_merge_trace, dim3(a.nnodes, (unsigned)((tot + 255) / 256)), dim3(256), 0,
                       c->stream, a, 0, a.nslot);
    return hipGetLastError();
}

hipError_t launch_merge_particular(rmrcm_ctx* c, int d) {
    MergeArgs a = make_args(c, d);
    if (d == 0) a.Tp = nullptr;
    if (a.xi <= kSX) {
        hipLaunchKernelGGL(k_merge_small, dim3(a.nnodes), dim3(256), 0, c->stream, a, 1);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_merge_rhs, dim3(a.nnodes, (a.xi + 255) / 256), dim3(256), 0, c->stream, a,
                       a.nslot, 1);
    hipError_t e = a.xi <= kBX ? solve_cols_blocked(c, a, a.nslot, 1)
                               : solve_cols_generic(c, a, a.nslot, 1);
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
    hipLaunchKernelGGL(k_down, dim3(P.nnodes, (P.xi + 3) / 4), dim3(256), lds, c->stream, a);
    return hipGetLastError();
}

}  // namespace rmrcm
