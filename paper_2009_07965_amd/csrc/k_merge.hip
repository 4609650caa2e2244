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
// M is factored once and kept with X for the downward pass (the Remark of
// Section 3.2: coefficients are tracked back to the finest level instead of
// storing coarse basis functions).  Every merge uses the pivot-free
// quasi-definite form below: gamma blocks of up to 128 segments in
// registers, longer ones in global memory.

#include <algorithm>
#include <vector>
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
    const int* gseg;            // [nnodes][g] global segment of gamma segment t
    double* M;                  // [nnodes][4 g^2]: D^{-1}, E, S^{-1}, B
    double* X;                  // [nnodes][xi][ld]
    double* Tp;                 // [nnodes][nslot][ld] (null at the root)
    const double* beta;
    const double* seglen;
    int* flags;
    int pin;                    // 1 at the root of an all-Neumann problem
    double* work;               // scratch of merges with g > 128 (see kBigWork)
    const unsigned char* tflag; // [nnodes][ntiles]: 64-slot tiles holding an active slot
    int ntiles;                 // (the particular column nslot counts as active)
    const int* run;             // null, or a device flag: the kernel does nothing while it is 0
};

// The launch does nothing when its run flag is given and 0 (the interface
// refinement's chain, skipped on the device when it is not needed).
#define RMRCM_RUN_GUARD(flag)            \
    do {                                 \
        if ((flag) && !*(flag)) return;  \
    } while (0)

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


// ---------------------------------------------------------------------------
// Pivot-free elimination in sum/difference variables.
//
// With s = (y1 + y2) / 2 and d = (y2 - y1) / 2 (the interface pressure and
// beta times the interface flux density of each gamma segment), the system
//     (T1gg + W) y1 - W y2 = r1,   -W y1 + (T2gg + W) y2 = r2
// becomes
//     [ N  B ] [s]   [r1 + r2]      N = T1gg + T2gg
//     [ B  D ] [d] = [r2 - r1],     B = T2gg - T1gg,   D = T1gg + T2gg + 4W.
// Every trace matrix is the Robin-to-flux map of a passive TPFA network with
// a series resistance beta on its Robin faces, so -diag(|f|/(rho+beta))
// summed per segment <= T <= 0, hence T + 2W > 0 on gamma: D is symmetric
// positive definite and S = N - B D^{-1} B negative definite (singular only
// at the top of an all-Neumann problem, whose null vector is a constant s).
// Such a quasi-definite system needs no pivoting.  Stored per merge, four
// g x g blocks: D^{-1}, E = D^{-1} B, S^{-1}, B; then
//     t = D^{-1}(r2 - r1),  s = S^{-1}(r1 + r2 - B t),  d = t - E s,
//     y1 = s - d,  y2 = s + d.
// The all-Neumann top pins s of the last gamma segment to zero.
//
// Factor, on the matrix cores (v_mfma_f64_16x16x4f64), one workgroup of
// GT/16 waves per merge.
//
// Each g x g block is padded to GT x GT and split into 16 x 16 tiles; wave w
// owns block column w and keeps its tiles in registers in the accumulator
// layout: lane l, register v holds row l/16 + 4v, column l%16 of the tile.
// That layout is also the B operand of the next product (k-slice s = v), so
// the tiles a wave owns never leave its registers.
//
// Inversion: blocked Gauss-Jordan without pivoting, one 16-wide pivot block K
// per step:  P = M_KK^{-1},  R_J = P M_KJ,  M_IJ -= M_IK R_J (I, J != K),
// M_IK = -M_IK P,  M_KK = P.  The owner of block column K publishes it to LDS
// (one barrier per step); every wave forms P itself from the symmetric block
// by an LDL^T factorisation without pivoting, with L^{-1} built alongside:
// P = L^{-T} diag(1/d) L^{-1}.  It needs only nonzero pivots (the blocks of D
// and S are definite; those of a learned trace need not be).  Padding rows
// and columns are identity rows and columns.  The products E = D^{-1} B and
// N - B E take the shared operand block column by block column through LDS
// panels, the next panel's loads in flight during the current one's MFMAs.
typedef double v4d __attribute__((ext_vector_type(4)));
__device__ inline v4d mfma_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int GT>
struct QdM {
    static constexpr int T = GT / 16;            // tiles per dimension = waves
    static constexpr int NT = 64 * T;
    static constexpr int CPL = 17;               // row stride of a column panel
    static constexpr int LTL = 20;               // row stride of a wave's L^{-1}
};

// Orders this wave's LDS writes before its later LDS reads by other lanes.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double readlane_d(double v, int l) {
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffu), l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// 1/d: the hardware estimate (relative error below 2^-24 on this part) and
// two Newton-Raphson steps y <- y + y (1 - d y), each squaring the error
// (one step leaves about 2^-48, which the recursive inverses of long
// interfaces amplify beyond the FP64 accuracy of the method).
__device__ inline double rcp_refined(double d) {
    double y = __builtin_amdgcn_rcp(d);
    y = fma(y, fma(-d, y, 1.0), y);
    y = fma(y, fma(-d, y, 1.0), y);
    return y;
}

// P = M_KK^{-1} of the symmetric 16 x 16 block at rows 16K.. of the column
// panel cpk (row stride CPL), returned in the accumulator layout.  lt, ls:
// this wave's two 16 x LTL scratch blocks.  Lanes 0-15 hold the columns of
// M_KK, lanes 16-31 the identity; eliminating below each pivot (multipliers
// from the pivot row, by symmetry) leaves L^{-1} in lanes 16-31.  kmax: the
// rows and columns from kmax on are identity ones, whose elimination steps
// change nothing and are skipped.  EARLY: row k of the result is stored as
// soon as pivot k is done (it is final then), so no reciprocal is held to
// the end: fewer vector registers, but where the caller's own registers are
// many the compiler then spills scalar ones, so only the fused small merge
// takes it; both forms store the same numbers.
template <bool EARLY = false>
__device__ __forceinline__ v4d qd_pivot_inverse(const double* cpk, int K, double* lt, double* ls,
                                                 int* bad, int kmax = 16) {
    typedef QdM<16> Q;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const bool scol = lane < 16, icol = lane >= 16 && lane < 32;
    double a[16], rd[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        a[i] = scol ? cpk[(16 * K + i) * Q::CPL + li] : ((icol && i == li) ? 1.0 : 0.0);
    int sing = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k >= kmax) {
            rd[k] = 1.0;
            if (EARLY && icol) {
                lt[li * Q::LTL + k] = a[k];
                ls[li * Q::LTL + k] = a[k];
            }
            continue;
        }
        // a zero or non-finite pivot is flagged (the inverse is then not
        // used); the test stays off the pivot chain
        const double d = readlane_d(a[k], k);
        sing |= !(d != 0.0 && isfinite(d));
        rd[k] = rcp_refined(d);
        const double lrow = a[k] * rd[k];          // row k of L^T
#pragma unroll
        for (int i = k + 1; i < 16; ++i) a[i] = fma(-readlane_d(lrow, i), a[k], a[i]);
        if (EARLY && icol) {
            lt[li * Q::LTL + k] = a[k];
            ls[li * Q::LTL + k] = lrow;
        }
    }
    if (sing && lane == 0) *bad = 1;
    if (!EARLY && icol) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            lt[li * Q::LTL + i] = a[i];             // row c = column c of L^{-1}
            ls[li * Q::LTL + i] = a[i] * rd[i];     // the same scaled by 1/d_i
        }
    }
    wave_lds_sync();
    // P[r][c] = sum_i L^{-1}[i][r] (1/d_i) L^{-1}[i][c], on the vector units
    // (the matrix cores are busy with the other waves' updates), in the
    // accumulator layout: lane l forms rows l/16 + 4v of column l%16
    v4d P = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
        P = mfma_f64(lt[li * Q::LTL + 4 * s + lk], ls[li * Q::LTL + 4 * s + lk], P);
    return P;
}

// In-place inversion of the register-resident matrix m (block column w of
// the wave).  cp: two column panels, pt: two 16 x 17 tiles for P.  Step K,
// two barriers: first every wave updates its block column with P_K (the
// owner of block column K + 1 publishes it), then the owner of block column
// K inverts the next pivot block, P_{K+1}, alone: run beside the other
// waves' matrix-core updates the pivot chain takes more than twice as long.
template <int GT>
__device__ __forceinline__ void qd_publish(const v4d (&m)[QdM<GT>::T], double* c) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int I = 0; I < QdM<GT>::T; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) c[(16 * I + lk + 4 * v) * QdM<GT>::CPL + li] = m[I][v];
    wave_lds_sync();
}

template <int GT>
__device__ void qd_gj_mfma(v4d (&m)[QdM<GT>::T], double* cp, double* pt, double* lt, double* ls,
                           int* bad) {
    typedef QdM<GT> Q;
    constexpr int T = Q::T, CPL = Q::CPL;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    if (w == 0) {
        qd_publish<GT>(m, cp);
        const v4d P = qd_pivot_inverse(cp, 0, lt, ls, bad);
#pragma unroll
        for (int v = 0; v < 4; ++v) pt[(lk + 4 * v) * 17 + li] = P[v];
    }
    __syncthreads();
    for (int K = 0; K < T; ++K) {
        const double* c = cp + (K & 1) * GT * CPL;
        const double* pk = pt + (K & 1) * 16 * 17;
        double* cn = cp + ((K + 1) & 1) * GT * CPL;
        v4d P;
        double pa[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) P[v] = pk[(lk + 4 * v) * 17 + li];     // B operand layout
#pragma unroll
        for (int s = 0; s < 4; ++s) pa[s] = pk[li * 17 + 4 * s + lk];      // A operand layout
        if (w == K) {
            // pivot block column: M_IK = -M_IK P, M_KK = P
#pragma unroll
            for (int I = 0; I < T; ++I) {
                v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    acc = mfma_f64(-c[(16 * I + li) * CPL + 4 * s + lk], P[s], acc);
                m[I] = (I == K) ? P : acc;
            }
        } else {
            // R_J = P M_KJ, M_IJ -= M_IK R_J (I != K), M_KJ = R_J
            v4d mk = m[0];
#pragma unroll
            for (int I = 1; I < T; ++I)
                if (I == K) mk = m[I];
            v4d R = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s) R = mfma_f64(pa[s], mk[s], R);
#pragma unroll
            for (int I = 0; I < T; ++I) {
                if (I == K) {
                    m[I] = R;
                    continue;
                }
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    m[I] = mfma_f64(-c[(16 * I + li) * CPL + 4 * s + lk], R[s], m[I]);
            }
            if (w == K + 1) qd_publish<GT>(m, cn);
        }
        __syncthreads();
        if (w == K && K + 1 < T) {
            const v4d Pn = qd_pivot_inverse(cn, K + 1, lt, ls, bad);
            double* pn = pt + ((K + 1) & 1) * 16 * 17;
#pragma unroll
            for (int v = 0; v < 4; ++v) pn[(lk + 4 * v) * 17 + li] = Pn[v];
        }
        __syncthreads();
    }
}

// Stores the wave's tiles (rows and columns below g) to the row-major g x g
// block X; pin: the all-Neumann top's pinned entry is stored as zero.
template <int GT>
__device__ void qd_store(const v4d (&m)[QdM<GT>::T], int g, double* X, bool pin) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int I = 0; I < QdM<GT>::T; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + lk + 4 * v, j = 16 * w + li;
            if (i < g && j < g) X[(size_t)i * g + j] = (pin && i == g - 1 && j == g - 1) ? 0.0 : m[I][v];
        }
}

// Block column K of the row-major g x g block X (zero outside g x g): four
// entries per thread, consecutive threads on consecutive columns.
template <int GT>
__device__ inline void qd_panel_load(const double* X, int g, int K, double (&r)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + QdM<GT>::NT * q, row = e >> 4, col = 16 * K + (e & 15);
        r[q] = (row < g && col < g) ? X[(size_t)row * g + col] : 0.0;
    }
}
template <int GT>
__device__ inline void qd_panel_put(double* pn, const double (&r)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + QdM<GT>::NT * q;
        pn[(e >> 4) * QdM<GT>::CPL + (e & 15)] = r[q];
    }
}

// phase 0: the whole factorisation; 1: up to D^{-1} (B and N stored);
// 2: S^{-1} from S in Sg (the products in between by k_qd_es_mfma).
template <int GT>
__global__ __launch_bounds__(QdM<GT>::NT) void k_qd_factor_mfma(MergeArgs a, int phase) {
    RMRCM_RUN_GUARD(a.run);
    typedef QdM<GT> Q;
    constexpr int T = Q::T, CPL = Q::CPL;
    // up to 64 segments the products between the inversions take D^{-1} and
    // B from LDS and B, N, E from registers (beyond, from global memory)
    constexpr bool LP = GT <= 64;
    constexpr int DLD = GT + 1;
    __shared__ double DL[LP ? GT * DLD : 1], BL[LP ? GT * DLD : 1];
    __shared__ double cp[2 * GT * CPL];
    __shared__ double lts[2 * T * 16 * Q::LTL];
    __shared__ double pt[2 * 16 * 17];
    __shared__ double wv[GT];
    __shared__ int gi1[GT], gi2[GT];
    __shared__ int bad;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int node = blockIdx.x, g = a.g;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    if (tid == 0) bad = 0;
    for (int t = tid; t < g; t += Q::NT) {
        gi1[t] = a.gmap[t];
        gi2[t] = a.gmap[g + t];
        const int e = a.gseg[(size_t)node * g + t];
        wv[t] = a.seglen[e] / (2.0 * a.beta[e]);
    }
    __syncthreads();
    const size_t gg = (size_t)g * g;
    double* Dg = a.M + (size_t)node * 4 * gg;
    double* Eg = Dg + gg;
    double* Sg = Eg + gg;
    double* Bg = Sg + gg;
    double* lt = lts + 2 * w * 16 * Q::LTL;
    double* ls = lt + 16 * Q::LTL;
    const int j = 16 * w + li;                   // the column this lane holds
    v4d m[T];
    v4d Bm[LP ? T : 1], Nm[LP ? T : 1];
    if (phase == 2) {
        // S (identity outside g x g)
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + lk + 4 * v;
                m[I][v] = (i < g && j < g) ? Sg[(size_t)i * g + j] : (i == j ? 1.0 : 0.0);
            }
    } else {
    // the gamma blocks of both children: B and N to global memory, D in
    // registers (four tiles' loads in flight at a time)
    constexpr int CI = T;
#pragma unroll
    for (int I0 = 0; I0 < T; I0 += CI) {
        double t1[CI][4], t2[CI][4];
#pragma unroll
        for (int u = 0; u < CI; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * (I0 + u) + lk + 4 * v;
                const bool in = i < g && j < g;
                t1[u][v] = in ? T1[(size_t)gi1[i] * a.cld + gi1[j]] : 0.0;
                t2[u][v] = in ? T2[(size_t)gi2[i] * a.cld + gi2[j]] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < CI; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * (I0 + u) + lk + 4 * v;
                const double nv = t1[u][v] + t2[u][v];
                const bool in = i < g && j < g;
                if (in) {
                    Bg[(size_t)i * g + j] = t2[u][v] - t1[u][v];
                    if (!LP) Sg[(size_t)i * g + j] = nv;         // N, parked until the Schur step
                    m[I0 + u][v] = nv + (i == j ? 4.0 * wv[i] : 0.0);
                } else {
                    m[I0 + u][v] = (i == j) ? 1.0 : 0.0;
                }
                if constexpr (LP) {
                    Bm[I0 + u][v] = in ? t2[u][v] - t1[u][v] : 0.0;
                    Nm[I0 + u][v] = in ? nv : (i == j ? 1.0 : 0.0);
                }
            }
    }
    qd_gj_mfma<GT>(m, cp, pt, lt, ls, &bad);              // D^{-1}
    qd_store<GT>(m, g, Dg, false);
    if (phase == 1) {
        if (tid == 0 && bad) atomicOr(&a.flags[FLAG_MERGE_SINGULAR], 1);
        return;
    }
    if constexpr (LP) {
        // D^{-1} and B to LDS, then E = D^{-1} B and S = N - B E for block
        // column w (B_KJ, N_IJ and E_KJ the wave's own tiles)
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + lk + 4 * v;
                DL[i * DLD + j] = m[I][v];
                BL[i * DLD + j] = Bm[I][v];
            }
        __syncthreads();
#pragma unroll
        for (int I = 0; I < T; ++I) {
            v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int K = 0; K < T; ++K)
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    acc = mfma_f64(DL[(16 * I + li) * DLD + 16 * K + 4 * s + lk], Bm[K][s], acc);
            m[I] = acc;
        }
        qd_store<GT>(m, g, Eg, false);
#pragma unroll
        for (int I = 0; I < T; ++I) {
            v4d acc = Nm[I];
#pragma unroll
            for (int K = 0; K < T; ++K)
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    acc = mfma_f64(-BL[(16 * I + li) * DLD + 16 * K + 4 * s + lk], m[K][s], acc);
            Bm[I] = acc;
        }
#pragma unroll
        for (int I = 0; I < T; ++I) m[I] = Bm[I];
    } else {
    __syncthreads();                                       // D^{-1}, B, N visible to the workgroup
    // E = D^{-1} B (block column w): block column K of D^{-1} staged in LDS
    // (the next one in flight meanwhile), B_KJ from global memory
    {
        double r[4], bcur[4], bnext[4];
        qd_panel_load<GT>(Dg, g, 0, r);
        qd_panel_put<GT>(cp, r);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = 4 * s + lk;
            bcur[s] = (k < g && j < g) ? Bg[(size_t)k * g + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int I = 0; I < T; ++I) m[I] = v4d{0.0, 0.0, 0.0, 0.0};
        for (int K = 0; K < T; ++K) {
            const double* pn = cp + (K & 1) * GT * CPL;
            if (K + 1 < T) {
                qd_panel_load<GT>(Dg, g, K + 1, r);
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int k = 16 * (K + 1) + 4 * s + lk;
                    bnext[s] = (k < g && j < g) ? Bg[(size_t)k * g + j] : 0.0;
                }
            }
#pragma unroll
            for (int I = 0; I < T; ++I)
#pragma unroll
                for (int s = 0; s < 4; ++s) m[I] = mfma_f64(pn[(16 * I + li) * CPL + 4 * s + lk], bcur[s], m[I]);
            if (K + 1 < T) {
                qd_panel_put<GT>(cp + ((K + 1) & 1) * GT * CPL, r);
#pragma unroll
                for (int s = 0; s < 4; ++s) bcur[s] = bnext[s];
            }
            __syncthreads();
        }
    }
    qd_store<GT>(m, g, Eg, false);
    // S = N - B E (block column w; E_KJ is the wave's own tile m[K]): block
    // column K of B staged in LDS
    {
        v4d acc[T];
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + lk + 4 * v;
                acc[I][v] = (i < g && j < g) ? Sg[(size_t)i * g + j] : (i == j ? 1.0 : 0.0);
            }
        double r[4];
        qd_panel_load<GT>(Bg, g, 0, r);
        qd_panel_put<GT>(cp, r);
        __syncthreads();
#pragma unroll
        for (int K = 0; K < T; ++K) {
            const double* pn = cp + (K & 1) * GT * CPL;
            if (K + 1 < T) qd_panel_load<GT>(Bg, g, K + 1, r);
#pragma unroll
            for (int I = 0; I < T; ++I)
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    acc[I] = mfma_f64(-pn[(16 * I + li) * CPL + 4 * s + lk], m[K][s], acc[I]);
            if (K + 1 < T) qd_panel_put<GT>(cp + ((K + 1) & 1) * GT * CPL, r);
            __syncthreads();
        }
#pragma unroll
        for (int I = 0; I < T; ++I) m[I] = acc[I];
    }
    }
    }
    if (a.pin) {
        // all-Neumann top: s of the last gamma segment is pinned
#pragma unroll
        for (int I = 0; I < T; ++I)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + lk + 4 * v;
                if (i == g - 1 || j == g - 1) m[I][v] = (i == j) ? 1.0 : 0.0;
            }
    }
    qd_gj_mfma<GT>(m, cp, pt, lt, ls, &bad);              // S^{-1}
    qd_store<GT>(m, g, Sg, a.pin);
    if (tid == 0 && bad) atomicOr(&a.flags[FLAG_MERGE_SINGULAR], 1);
}

// The two products between the inversions of k_qd_factor_mfma, E = D^{-1} B
// and S = N - B E, spread over workgroups: block column w = blockIdx.y of
// one merge per workgroup (S's block column needs only E's), wave r forming
// row tile r of E's block column, shared in LDS, then of S's; for merges
// that are few and large (one workgroup per merge would leave the chip
// idle).
template <int GT>
__device__ __forceinline__ void qd_load_tile(int g, const double* __restrict__ A, double (&av)[GT / 4]);

template <int GT>
__global__ __launch_bounds__(QdM<GT>::NT) void k_qd_es_mfma(MergeArgs a) {
    RMRCM_RUN_GUARD(a.run);
    constexpr int T = QdM<GT>::T;
    __shared__ double Es[GT * 17];
    const int tid = threadIdx.x, lane = tid & 63, r = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int node = blockIdx.x, w = blockIdx.y, g = a.g;
    const size_t gg = (size_t)g * g;
    const double* Dg = a.M + (size_t)node * 4 * gg;
    double* Eg = a.M + (size_t)node * 4 * gg + gg;
    double* Sg = Eg + gg;
    const double* Bg = Sg + gg;
    const int j = 16 * w + li, ia = 16 * r + li;
    // every operand of a product is loaded before the product runs (the
    // loads in flight together), B's row tile for S before the barrier; the
    // k-slices as in qd_load_tile (slice q: k = 16 (q / 4) + 4 lk + q % 4, a
    // lane's row entries read four at a time)
    double av[4 * T], bv[4 * T], b2[4 * T];
    qd_load_tile<GT>(g, Dg, av);
    qd_load_tile<GT>(g, Bg, b2);
#pragma unroll
    for (int q = 0; q < 4 * T; ++q) {
        const int ka = 16 * (q >> 2) + 4 * lk + (q & 3);
        bv[q] = (ka < g && j < g) ? Bg[(size_t)ka * g + j] : 0.0;
    }
    (void)ia;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4 * T; ++q) acc = mfma_f64(av[q], bv[q], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 16 * r + lk + 4 * v;
        Es[i * 17 + li] = acc[v];
        if (i < g && j < g) Eg[(size_t)i * g + j] = acc[v];
    }
    __syncthreads();
    v4d sc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 16 * r + lk + 4 * v;
        sc[v] = (i < g && j < g) ? Sg[(size_t)i * g + j] : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < 4 * T; ++q)
        sc = mfma_f64(-b2[q], Es[(16 * (q >> 2) + 4 * lk + (q & 3)) * 17 + li], sc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 16 * r + lk + 4 * v;
        if (i < g && j < g) Sg[(size_t)i * g + j] = sc[v];
    }
}

// Gamma coefficients of columns [col0, col0 + ncol): X = -M^{-1} R through
// the stored blocks, on the matrix cores, 16 NCT columns per workgroup: each
// of the four products is A (g x g, row-major in global memory) times a
// g x 16 NCT block held in LDS (rows padded to GT, leading dimension
// 16 NCT + 1); wave w forms row tiles I = w, w + NW, .. with every k-slice
// of A for the tile loaded at once and used for all NCT column tiles.
template <int GT>
__host__ __device__ constexpr int qd_apply_waves() { return GT / 16 > 4 ? GT / 16 : 4; }

// The row tile w of A (g x g, row-major) as MFMA A operands: k-slice
// q = 4u + h of lane l holds k = 16u + 4(l/16) + h, so that a lane loads four
// consecutive entries of its row at once (the sum over k is taken in this
// order on both operands).  Zero outside g x g and for waves without a tile.
template <int GT>
__device__ __forceinline__ void qd_load_tile(int g, const double* __restrict__ A, double (&av)[GT / 4]) {
    constexpr int KS = GT / 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int i = 16 * w + li;
    if ((g & 3) == 0 && i < g) {
        const double* Ai = A + (size_t)i * g;
#pragma unroll
        for (int u = 0; u < KS / 4; ++u) {
            const int k0 = 16 * u + 4 * lk;
            const double4 v = k0 < g ? *(const double4*)(Ai + k0) : double4{0.0, 0.0, 0.0, 0.0};
            av[4 * u] = v.x;
            av[4 * u + 1] = v.y;
            av[4 * u + 2] = v.z;
            av[4 * u + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const int k = 16 * (q >> 2) + 4 * lk + (q & 3);
            av[q] = (i < g && k < g) ? A[(size_t)i * g + k] : 0.0;
        }
    }
}

// out (=, or -= when sub) A in for the row tile of this wave, A given as
// loaded by qd_load_tile; in and out g x 16 NCT blocks in LDS.
template <int GT, int NCT>
__device__ __forceinline__ void qd_prod_mfma(const double (&av)[GT / 4], const double* in, double* out,
                                             bool sub) {
    constexpr int T = GT / 16, KS = GT / 4, AL = 16 * NCT + 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    if (w < T) {
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < KS; ++q)
                acc = mfma_f64(av[q], in[(16 * (q >> 2) + 4 * lk + (q & 3)) * AL + 16 * ct + li], acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e = (16 * w + lk + 4 * v) * AL + 16 * ct + li;
                out[e] = sub ? out[e] - acc[v] : acc[v];
            }
        }
    }
    __syncthreads();
}

template <int GT, int NCT>
__global__ __launch_bounds__(64 * qd_apply_waves<GT>()) void k_qd_apply_mfma(MergeArgs a, int col0,
                                                                             int ncol) {
    RMRCM_RUN_GUARD(a.run);
    constexpr int CT = 16 * NCT, AL = CT + 1, NT = 64 * qd_apply_waves<GT>();
    __shared__ double rs[GT * AL], rd[GT * AL], tt[GT * AL];
    const int node = blockIdx.x, g = a.g;
    const int cb = col0 + blockIdx.y * CT;
    const int nc = min(CT, col0 + ncol - cb);
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    const int* g1 = a.gmap;
    const int* g2 = a.gmap + g;
    const size_t gg = (size_t)g * g;
    const double* Dg = a.M + (size_t)node * 4 * gg;
    const double* Eg = Dg + gg;
    const double* Sg = Eg + gg;
    const double* Bg = Sg + gg;
    double av[GT / 4], an[GT / 4];
    qd_load_tile<GT>(g, Dg, av);                     // in flight during the gathers
    qd_load_tile<GT>(g, Bg, an);
    // r1, r2 of the columns (zero outside g x nc), as r1 + r2 and r2 - r1;
    // four entries per thread in flight
    for (int t0 = 0; t0 < GT * CT; t0 += 4 * NT) {
        double v1[4], v2[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * NT + threadIdx.x;
            const int i = t / CT, cc = t % CT, col = cb + cc;
            v1[u] = 0.0;
            v2[u] = 0.0;
            if (t < GT * CT && cc < nc && i < g) {
                if (col == a.nslot) {
                    v1[u] = T1[(size_t)g1[i] * a.cld + a.cld - 1];
                    v2[u] = T2[(size_t)g2[i] * a.cld + a.cld - 1];
                } else {
                    const int pm = a.pmap[col], off = pm & 0xffffff;
                    if ((pm >> 24) == 0) v1[u] = T1[(size_t)g1[i] * a.cld + off];
                    else v2[u] = T2[(size_t)g2[i] * a.cld + off];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * NT + threadIdx.x;
            if (t < GT * CT) {
                const int e = (t / CT) * AL + t % CT;
                rs[e] = v1[u] + v2[u];
                rd[e] = v2[u] - v1[u];
            }
        }
    }
    __syncthreads();
    // the four products; each block's tile is loaded while the previous
    // product runs
    qd_prod_mfma<GT, NCT>(av, rd, tt, false);       // t = D^{-1} (r2 - r1)
#pragma unroll
    for (int q = 0; q < GT / 4; ++q) av[q] = an[q];
    qd_load_tile<GT>(g, Sg, an);
    qd_prod_mfma<GT, NCT>(av, tt, rs, true);        // u = r1 + r2 - B t
#pragma unroll
    for (int q = 0; q < GT / 4; ++q) av[q] = an[q];
    qd_load_tile<GT>(g, Eg, an);
    qd_prod_mfma<GT, NCT>(av, rs, rd, false);       // s = S^{-1} u
    qd_prod_mfma<GT, NCT>(an, rd, tt, true);        // d = t - E s
    double* X = a.X + (size_t)node * a.xi * a.ld;
    for (int t = threadIdx.x; t < g * CT; t += NT) {
        const int i = t / CT, cc = t % CT;
        if (cc >= nc) continue;
        const double s = rd[i * AL + cc], d = tt[i * AL + cc];
        X[(size_t)i * a.ld + cb + cc] = -(s - d);
        X[(size_t)(g + i) * a.ld + cb + cc] = -(s + d);
    }
}

// Column apply and parent traces of one 16-column tile of a merge in
// workgroups of eight waves, for interfaces of 32 and 64 segments (as two
// launches, each is bound by its own load latency and the traces wait for X
// to reach memory).  The first waves apply the factorisation as
// k_qd_apply_mfma does; X stays in LDS for the traces, whose row tiles the
// gridDim.z workgroups of the tile share (each repeats the apply, the first
// writes X), eight waves each.  The trace operands (the child trace rows
// against gamma and the direct terms) of a row tile are loaded at its start;
// the gamma maps are staged in LDS and X is read from LDS at each use, so
// that two workgroups fit a compute unit.
template <int GT>
__global__ __launch_bounds__(512) void k_qd_cols_mfma(MergeArgs a, int col0, int ncol) {
    RMRCM_RUN_GUARD(a.run);
    constexpr int CT = 16, AL = CT + 1, NT = 512, NW = NT / 64, KS = GT / 4;
    __shared__ double rs[GT * AL], rd[GT * AL], tt[GT * AL];
    __shared__ int gms[2 * GT];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int node = blockIdx.x, g = a.g, nslot = a.nslot;
    const int cb = col0 + blockIdx.y * CT;
    const int nc = min(CT, col0 + ncol - cb);
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    const int* g1 = a.gmap;
    const int* g2 = a.gmap + g;
    const size_t gg = (size_t)g * g;
    const double* Dg = a.M + (size_t)node * 4 * gg;
    const double* Eg = Dg + gg;
    const double* Sg = Eg + gg;
    const double* Bg = Sg + gg;
    // trace operands: this lane's column, gamma columns of both children,
    // and a row tile's child trace rows and direct terms
    const int col = cb + li;
    const bool cin = li < nc;
    const int pc = (cin && col < nslot) ? a.pmap[col] : -1;
    const int nrt = (nslot + 15) / 16, ot0 = w + NW * blockIdx.z, ots = NW * gridDim.z;
    // the gamma maps of both children in LDS (read by the trace operand
    // loads; registers are the occupancy bound here)
    for (int t = tid; t < 2 * GT; t += NT) {
        const int k = t / GT, i = t % GT;
        gms[t] = i < g ? (k ? g2[i] : g1[i]) : 0;
    }
    __syncthreads();
    auto load_rows = [&](int ot, double (&av)[KS], double (&dr)[4], int& ka) {
        const int oa = 16 * ot + li;
        const int pa = (ot < nrt && oa < nslot) ? a.pmap[oa] : -1;
        ka = pa >= 0 ? (pa >> 24) : -1;
        const double* ta = (ka == 1 ? T2 : T1) + (size_t)(pa >= 0 ? (pa & 0xffffff) : 0) * a.cld;
        const int* gk = gms + (ka == 1 ? GT : 0);
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const int i = 4 * q + lk;
            av[q] = (ka >= 0 && i < g) ? ta[gk[i]] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = 16 * ot + lk + 4 * v;
            double d = 0.0;
            if (ot < nrt && o < nslot && cin) {
                const int pm = a.pmap[o], k = pm >> 24;
                const double* tr = (k ? T2 : T1) + (size_t)(pm & 0xffffff) * a.cld;
                if (col == nslot) d = tr[a.cld - 1];
                else if ((pc >> 24) == k) d = tr[pc & 0xffffff];
            }
            dr[v] = d;
        }
    };
    // ---- the apply (k_qd_apply_mfma with one column tile)
    double av[GT / 4], an[GT / 4];
    qd_load_tile<GT>(g, Dg, av);
    qd_load_tile<GT>(g, Bg, an);
    for (int t0 = 0; t0 < GT * CT; t0 += 4 * NT) {
        double v1[4], v2[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * NT + tid;
            const int i = t / CT, cc = t % CT, cl = cb + cc;
            v1[u] = 0.0;
            v2[u] = 0.0;
            if (t < GT * CT && cc < nc && i < g) {
                if (cl == nslot) {
                    v1[u] = T1[(size_t)g1[i] * a.cld + a.cld - 1];
                    v2[u] = T2[(size_t)g2[i] * a.cld + a.cld - 1];
                } else {
                    const int pm = a.pmap[cl], off = pm & 0xffffff;
                    if ((pm >> 24) == 0) v1[u] = T1[(size_t)g1[i] * a.cld + off];
                    else v2[u] = T2[(size_t)g2[i] * a.cld + off];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * NT + tid;
            if (t < GT * CT) {
                const int e = (t / CT) * AL + t % CT;
                rs[e] = v1[u] + v2[u];
                rd[e] = v2[u] - v1[u];
            }
        }
    }
    __syncthreads();
    qd_prod_mfma<GT, 1>(av, rd, tt, false);       // t = D^{-1} (r2 - r1)
#pragma unroll
    for (int q = 0; q < GT / 4; ++q) av[q] = an[q];
    qd_load_tile<GT>(g, Sg, an);
    qd_prod_mfma<GT, 1>(av, tt, rs, true);        // u = r1 + r2 - B t
#pragma unroll
    for (int q = 0; q < GT / 4; ++q) av[q] = an[q];
    qd_load_tile<GT>(g, Eg, an);
    qd_prod_mfma<GT, 1>(av, rs, rd, false);       // s = S^{-1} u
    qd_prod_mfma<GT, 1>(an, rd, tt, true);        // d = t - E s
    double* X = a.X + (size_t)node * a.xi * a.ld;
    if (blockIdx.z == 0) {
        for (int t = tid; t < g * CT; t += NT) {
            const int i = t / CT, cc = t % CT;
            if (cc >= nc) continue;
            const double sv = rd[i * AL + cc], dv = tt[i * AL + cc];
            X[(size_t)i * a.ld + cb + cc] = -(sv - dv);
            X[(size_t)(g + i) * a.ld + cb + cc] = -(sv + dv);
        }
    }
    // ---- parent traces of the tile: T_p[o, col] = direct + A_k(o) X_k[:, col],
    // the B operands X_1 = -(s - d), X_2 = -(s + d) formed from s and d in
    // LDS at each use; each row tile's operands loaded at its start (another
    // workgroup on the compute unit covers the latency: registers bound the
    // occupancy, and holding the next tile's operands would halve it)
    auto xb = [&](int k, int q) -> double {
        const int i = 4 * q + lk;
        const double sv = rd[i * AL + li], dv = tt[i * AL + li];
        const bool in = i < g && cin;
        return in ? (k ? -(sv + dv) : -(sv - dv)) : 0.0;
    };
    double* Tp = a.Tp + (size_t)node * nslot * a.ld;
    for (int ot = ot0; ot < nrt; ot += ots) {
        double av0[KS], dr0[4];
        int ka0;
        load_rows(ot, av0, dr0, ka0);
        // a child's half is skipped when none of the tile's rows is its
        // (all-zero A rows: the sum is unchanged bit for bit); most tiles
        // lie on one child's sides
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        if (__ballot(ka0 == 0) != 0ull) {
#pragma unroll
            for (int q = 0; q < KS; ++q) acc = mfma_f64(ka0 == 0 ? av0[q] : 0.0, xb(0, q), acc);
        }
        if (__ballot(ka0 == 1) != 0ull) {
#pragma unroll
            for (int q = 0; q < KS; ++q) acc = mfma_f64(ka0 == 1 ? av0[q] : 0.0, xb(1, q), acc);
        }
        if (cin) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 16 * ot + lk + 4 * v;
                if (o < nslot) Tp[(size_t)o * a.ld + col] = dr0[v] + acc[v];
            }
        }
    }
}

// The particular column alone (the top's, where one merge is one workgroup)
// as matrix-vector products on the vector units: the same four products as
// k_qd_apply_mfma, t = D^{-1} (r2 - r1), u = r1 + r2 - B t, s = S^{-1} u,
// d = t - E s.  Row i of a g x g block is summed by 8 consecutive threads,
// thread c8 taking entries c8, c8 + 8, ... (each load reads runs of 8
// consecutive entries), and the partial sums added across those lanes; the
// next block's entries are loaded while the current product is reduced.
template <int GT>
__device__ __forceinline__ void qd_vec_load(const double* A, int g, int i, int c8, double (&r)[GT / 8]) {
    constexpr int CW = GT / 8;
#pragma unroll
    for (int q = 0; q < CW; ++q) {
        const int j = c8 + 8 * q;
        r[q] = (i < g && j < g) ? A[(size_t)i * g + j] : 0.0;
    }
}
template <int GT>
__device__ __forceinline__ double qd_vec_dot(const double (&r)[GT / 8], const double* x, int c8) {
    constexpr int CW = GT / 8;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < CW; ++q) s = fma(r[q], x[c8 + 8 * q], s);
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 4, 64);
    return s;
}

// With glo non-null the kernel also does the root's step of the downward
// pass: every slot of the root lies on the domain boundary (datum 0), so
// the gamma data are the particular column itself, written to the Robin
// datum of each row's side of its segment.
template <int GT>
__global__ __launch_bounds__(8 * GT) void k_qd_apply_vec(MergeArgs a, int col, double* glo, double* ghi) {
    RMRCM_RUN_GUARD(a.run);
    __shared__ double rs[GT], rd[GT], tt[GT], uu[GT];
    const int node = blockIdx.x, g = a.g;
    const int tid = threadIdx.x, i = tid >> 3, c8 = tid & 7;
    int c1, c2;
    children(a, node, &c1, &c2);
    const size_t gg = (size_t)g * g;
    const double* Dg = a.M + (size_t)node * 4 * gg;
    const double* Eg = Dg + gg;
    const double* Sg = Eg + gg;
    const double* Bg = Sg + gg;
    double ra[GT / 8], rb[GT / 8];
    qd_vec_load<GT>(Dg, g, i, c8, ra);                 // in flight during the gathers
    qd_vec_load<GT>(Bg, g, i, c8, rb);
    if (tid < GT) {
        double v1 = 0.0, v2 = 0.0;
        if (tid < g) {
            const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
            const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
            if (col == a.nslot) {
                v1 = T1[(size_t)a.gmap[tid] * a.cld + a.cld - 1];
                v2 = T2[(size_t)a.gmap[g + tid] * a.cld + a.cld - 1];
            } else {
                const int pm = a.pmap[col], off = pm & 0xffffff;
                if ((pm >> 24) == 0) v1 = T1[(size_t)a.gmap[tid] * a.cld + off];
                else v2 = T2[(size_t)a.gmap[g + tid] * a.cld + off];
            }
        }
        rs[tid] = v1 + v2;
        rd[tid] = v2 - v1;
    }
    __syncthreads();
    const double t = qd_vec_dot<GT>(ra, rd, c8);      // t = D^{-1} (r2 - r1)
    if (c8 == 0) tt[i] = t;
    qd_vec_load<GT>(Sg, g, i, c8, ra);
    __syncthreads();
    const double u = rs[i] - qd_vec_dot<GT>(rb, tt, c8);   // u = r1 + r2 - B t
    if (c8 == 0) uu[i] = u;
    qd_vec_load<GT>(Eg, g, i, c8, rb);
    __syncthreads();
    const double sv = qd_vec_dot<GT>(ra, uu, c8);     // s = S^{-1} u
    if (c8 == 0) rs[i] = sv;
    __syncthreads();
    const double d = tt[i] - qd_vec_dot<GT>(rb, rs, c8);   // d = t - E s
    if (c8 == 0 && i < g) {
        double* X = a.X + (size_t)node * a.xi * a.ld;
        X[(size_t)i * a.ld + col] = -(sv - d);
        X[(size_t)(g + i) * a.ld + col] = -(sv + d);
        if (glo) {
            const int e = a.css[(size_t)c1 * a.cnslot + a.gmap[i]] >> 1;
            glo[e] = -(sv - d);
            ghi[e] = -(sv + d);
        }
    }
}

// Parent traces on the matrix cores: T_p[o][col] = direct(o, col)
// + sum_i A_1[o][i] X_1[i][col] + sum_i A_2[o][i] X_2[i][col], with A_k[o][i]
// = T_k[o, gamma_k(i)] on the rows o that child k owns and zero on the
// others (an MFMA's B operand is shared by all rows of the tile).  Wave w of
// a workgroup forms the 16 x 16 tile of rows 16 (4 y + w).., columns 16 z..
template <int GT>
__global__ __launch_bounds__(256) void k_qd_trace_mfma(MergeArgs a, int col0, int ncol) {
    RMRCM_RUN_GUARD(a.run);
    constexpr int KS = GT / 4;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int node = blockIdx.x, g = a.g;
    const int o0 = 16 * (4 * blockIdx.y + w), cb = col0 + 16 * blockIdx.z;
    if (o0 >= a.nslot) return;
    const int ce = col0 + ncol;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* Tk[2] = {a.Tc + (size_t)c1 * a.cnslot * a.cld, a.Tc + (size_t)c2 * a.cnslot * a.cld};
    const double* X = a.X + (size_t)node * a.xi * a.ld;
    // the A row of this lane
    const int oa = o0 + li;
    const int pa = oa < a.nslot ? a.pmap[oa] : -1;
    const int ka = pa >= 0 ? (pa >> 24) : -1;
    const double* ta = pa >= 0 ? Tk[ka] + (size_t)(pa & 0xffffff) * a.cld : nullptr;
    const int col = cb + li;
    // the direct terms of this lane's outputs, loaded with the operands
    const int pc = col < a.nslot ? a.pmap[col] : -1;
    double dr[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int o = o0 + lk + 4 * v;
        double d = 0.0;
        if (o < a.nslot && col < ce) {
            const int pm = a.pmap[o], k = pm >> 24;
            const double* tr = Tk[k] + (size_t)(pm & 0xffffff) * a.cld;
            if (col == a.nslot) d = tr[a.cld - 1];
            else if ((pc >> 24) == k) d = tr[pc & 0xffffff];
        }
        dr[v] = d;
    }
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double av[KS], bv[KS];
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            const int i = 4 * q + lk;
            av[q] = (ka == k && i < g) ? ta[a.gmap[k * g + i]] : 0.0;
            bv[q] = (i < g && col < ce) ? X[(size_t)(k * g + i) * a.ld + col] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < KS; ++q) acc = mfma_f64(av[q], bv[q], acc);
    }
    if (col >= ce) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int o = o0 + lk + 4 * v;
        if (o >= a.nslot) continue;
        a.Tp[(size_t)node * a.nslot * a.ld + (size_t)o * a.ld + col] = dr[v] + acc[v];
    }
}

// ---------------------------------------------------------------- g <= 16
// Merges below the root whose gamma block is one 16 x 16 tile: factor,
// column apply and parent traces in one workgroup per merge, one wave per
// 16-column tile (at least four).  At these sizes every step is bound by
// load latency, so the kernel keeps the dependent global round trips to
// two before the factorisation: the level's maps and the gamma segments'
// numbers, then everything else at once.  Wave 0 gathers the gamma blocks
// and factors them in registers (the pivot chains stopping at g); the other
// waves stage in LDS the right-hand sides of every column (r1 + r2 and
// r2 - r1) and the child trace entries of every parent slot against gamma
// (the left operand of the trace product).  After the factorisation each
// wave issues the loads of the direct terms of its columns' parent traces
// (held for at most 16 MAXRT parent slots; not live during the pivot
// chains, whose registers bound the occupancy), applies the factorisation
// to its column tile in registers (a result in the accumulator layout is
// the next product's B operand), writes X and forms the parent traces of
// its columns.  Layouts as in the tiers above: accumulator lane l, register
// v = row l/16 + 4v, column l%16.
__host__ __device__ inline int small_cw(int ncol) { return 16 * ((ncol + 15) / 16) + 1; }
__host__ __device__ inline int small_ns16(int nslot) { return 16 * ((nslot + 15) / 16); }
__host__ __device__ inline int small_waves(int ncol) { return max(4, (ncol + 15) / 16); }
__host__ __device__ inline size_t small_lds_bytes(int ncol, int nslot) {
    const size_t nd = (size_t)32 * small_cw(ncol) + (size_t)small_ns16(nslot) * 17 + 5 * 272 + 2 * 16 * 20;
    return nd * sizeof(double) + (size_t)(48 + small_ns16(nslot) + 1) * sizeof(int);
}

template <int MAXRT>
__global__ __launch_bounds__(512) void k_qd_small(MergeArgs a, int ncol) {
    RMRCM_RUN_GUARD(a.run);
    extern __shared__ double sm[];
    const int CW = small_cw(ncol), NS16 = small_ns16(a.nslot), CT = (ncol + 15) / 16, NRT = NS16 / 16;
    double* rs = sm;                 // [16][CW]  r1 + r2
    double* rd = rs + 16 * CW;       // [16][CW]  r2 - r1
    double* ar = rd + 16 * CW;       // [NS16][17] T_k(o)[o, gamma_k(i)]
    double* dl = ar + NS16 * 17;     // D^{-1}, B, E, S^{-1}: [16][17] each
    double* bl = dl + 272;
    double* el = bl + 272;
    double* sl = el + 272;
    double* cp = sl + 272;           // the block being inverted
    double* lt = cp + 272;
    double* ls = lt + 16 * 20;
    int* gi1 = (int*)(ls + 16 * 20);
    int* gi2 = gi1 + 16;
    int* ge = gi2 + 16;              // global segment of gamma segment i
    int* pms = ge + 16;              // [NS16] parent slot map
    int* bad = pms + NS16;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int nt = blockDim.x, node = blockIdx.x, g = a.g, nslot = a.nslot;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    if (tid < 16) {
        gi1[tid] = tid < g ? a.gmap[tid] : 0;
        gi2[tid] = tid < g ? a.gmap[g + tid] : 0;
        ge[tid] = tid < g ? a.gseg[(size_t)node * g + tid] : 0;
    }
    if (tid >= 16)
        for (int o = tid - 16; o < NS16; o += nt - 16) pms[o] = o < nslot ? a.pmap[o] : -1;
    if (tid == 0) *bad = 0;
    __syncthreads();
    // this wave's column tile and the direct terms of its parent traces:
    // T_k[o, col] where slot o and column col belong to the same child k
    // (the particular column: T_k's own)
    const int col = 16 * w + li;
    const bool cin = col < ncol;
    double dv[MAXRT][4];
    auto load_direct = [&]() {
        const int pc = (cin && col < nslot) ? pms[col] : -1;
#pragma unroll
        for (int ot = 0; ot < MAXRT; ++ot)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = 16 * ot + lk + 4 * v;
                double x = 0.0;
                if (ot < NRT && o < nslot && cin) {
                    const int pm = pms[o], k = pm >> 24;
                    const double* tr = (k ? T2 : T1) + (size_t)(pm & 0xffffff) * a.cld;
                    if (col == nslot) x = tr[a.cld - 1];
                    else if ((pc >> 24) == k) x = tr[pc & 0xffffff];
                }
                dv[ot][v] = x;
            }
    };
    const size_t gg = (size_t)g * g;
    double* Dg = a.M + (size_t)node * 4 * gg;
    double* Eg = Dg + gg;
    double* Sg = Eg + gg;
    double* Bg = Sg + gg;
    if (w == 0) {
        // D = N + 4W, B = T2gg - T1gg, N = T1gg + T2gg (identity / zero padding)
        double t1[4], t2[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = lk + 4 * v;
            const bool in = i < g && li < g;
            t1[v] = in ? T1[(size_t)gi1[i] * a.cld + gi1[li]] : 0.0;
            t2[v] = in ? T2[(size_t)gi2[i] * a.cld + gi2[li]] : 0.0;
        }
        const int eg = ge[li];
        const double wl = li < g ? a.seglen[eg] / (2.0 * a.beta[eg]) : 0.0;
        v4d Dm, Nm, Bm;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = lk + 4 * v;
            const bool in = i < g && li < g;
            Nm[v] = t1[v] + t2[v];
            Bm[v] = t2[v] - t1[v];
            Dm[v] = in ? Nm[v] + (i == li ? 4.0 * wl : 0.0) : (i == li ? 1.0 : 0.0);
            cp[i * 17 + li] = Dm[v];
            bl[i * 17 + li] = Bm[v];
        }
        wave_lds_sync();
        const v4d Dinv = qd_pivot_inverse<true>(cp, 0, lt, ls, bad, g);
#pragma unroll
        for (int v = 0; v < 4; ++v) dl[(lk + 4 * v) * 17 + li] = Dinv[v];
        wave_lds_sync();
        // E = D^{-1} B, S = N - B E
        v4d E = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s) E = mfma_f64(dl[li * 17 + 4 * s + lk], Bm[s], E);
        v4d S = Nm;
#pragma unroll
        for (int s = 0; s < 4; ++s) S = mfma_f64(-bl[li * 17 + 4 * s + lk], E[s], S);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = lk + 4 * v;
            const bool in = i < g && li < g;
            el[i * 17 + li] = E[v];
            cp[i * 17 + li] = in ? S[v] : (i == li ? 1.0 : 0.0);
        }
        wave_lds_sync();
        const v4d Sinv = qd_pivot_inverse<true>(cp, 0, lt, ls, bad, g);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = lk + 4 * v;
            sl[i * 17 + li] = Sinv[v];
            if (i < g && li < g) {
                const size_t e = (size_t)i * g + li;
                Dg[e] = Dinv[v];
                Eg[e] = E[v];
                Sg[e] = Sinv[v];
                Bg[e] = Bm[v];
            }
        }
        if (lane == 0 && *bad) atomicOr(&a.flags[FLAG_MERGE_SINGULAR], 1);
    } else {
        // right-hand sides of the columns, four loads in flight per thread
        const int t2 = tid - 64, ns = nt - 64, CC = 16 * CT;
        for (int t0 = 0; t0 < 16 * CC; t0 += 4 * ns) {
            double v1[4], v2[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + ns * u + t2, i = t / CC, cc = t % CC;
                v1[u] = 0.0;
                v2[u] = 0.0;
                if (t < 16 * CC && i < g && cc < ncol) {
                    if (cc == nslot) {
                        v1[u] = T1[(size_t)gi1[i] * a.cld + a.cld - 1];
                        v2[u] = T2[(size_t)gi2[i] * a.cld + a.cld - 1];
                    } else {
                        const int pm = pms[cc], off = pm & 0xffffff;
                        if ((pm >> 24) == 0) v1[u] = T1[(size_t)gi1[i] * a.cld + off];
                        else v2[u] = T2[(size_t)gi2[i] * a.cld + off];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + ns * u + t2;
                if (t < 16 * CC) {
                    const int e = (t / CC) * CW + t % CC;
                    rs[e] = v1[u] + v2[u];
                    rd[e] = v2[u] - v1[u];
                }
            }
        }
        // the trace product's left operand: row o, gamma segment i of the
        // child that owns slot o
        for (int t0 = 0; t0 < 16 * NS16; t0 += 4 * ns) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + ns * u + t2, o = t >> 4, i = t & 15;
                v[u] = 0.0;
                if (t < 16 * NS16 && o < nslot && i < g) {
                    const int pm = pms[o], k = pm >> 24;
                    const double* tr = (k ? T2 : T1) + (size_t)(pm & 0xffffff) * a.cld;
                    v[u] = tr[k ? gi2[i] : gi1[i]];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + ns * u + t2;
                if (t < 16 * NS16) ar[(t >> 4) * 17 + (t & 15)] = v[u];
            }
        }
    }
    __syncthreads();
    if (w >= CT) return;
    double DA[4], BA[4], SA[4], EA[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int e = li * 17 + 4 * s + lk;
        DA[s] = dl[e];
        BA[s] = bl[e];
        SA[s] = sl[e];
        EA[s] = el[e];
    }
    load_direct();
    // t = D^{-1} (r2 - r1), u = r1 + r2 - B t, s = S^{-1} u, d = t - E s
    v4d t = {0.0, 0.0, 0.0, 0.0}, u, sv = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) t = mfma_f64(DA[s], rd[(4 * s + lk) * CW + col], t);
#pragma unroll
    for (int v = 0; v < 4; ++v) u[v] = rs[(lk + 4 * v) * CW + col];
#pragma unroll
    for (int s = 0; s < 4; ++s) u = mfma_f64(-BA[s], t[s], u);
#pragma unroll
    for (int s = 0; s < 4; ++s) sv = mfma_f64(SA[s], u[s], sv);
    v4d dd = t;
#pragma unroll
    for (int s = 0; s < 4; ++s) dd = mfma_f64(-EA[s], sv[s], dd);
    v4d x1, x2;
    double* X = a.X + (size_t)node * a.xi * a.ld;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        x1[v] = -(sv[v] - dd[v]);
        x2[v] = -(sv[v] + dd[v]);
        const int i = lk + 4 * v;
        if (i < g && cin) {
            X[(size_t)i * a.ld + col] = x1[v];
            X[(size_t)(g + i) * a.ld + col] = x2[v];
        }
    }
    // T_p[o, col] = direct + sum_i A_1[o][i] X_1[i][col] + A_2[o][i] X_2[i][col]
    double* Tp = a.Tp + (size_t)node * nslot * a.ld;
#pragma unroll
    for (int ot = 0; ot < MAXRT; ++ot) {
        if (ot >= NRT) break;
        const int o = 16 * ot + li;
        const int ko = o < nslot ? (pms[o] >> 24) : -1;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double val = ar[o * 17 + 4 * q + lk];
            acc = mfma_f64(ko == 0 ? val : 0.0, x1[q], acc);
            acc = mfma_f64(ko == 1 ? val : 0.0, x2[q], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int oo = 16 * ot + lk + 4 * v;
            if (oo < nslot && cin) Tp[(size_t)oo * a.ld + col] = dv[ot][v] + acc[v];
        }
    }
}

// The fused merge above serves a level when its gamma fits one tile, it is
// not the root, and the staged operands fit 64 KiB of LDS.
static bool small_merge_ok(const MergeArgs& a, int d, int ncol) {
    return d > 0 && a.g <= 16 && !a.pin && a.nslot <= 127 && ncol <= 128 &&
           small_lds_bytes(ncol, a.nslot) <= 64 * 1024;
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
    const int* run;
};

__global__ __launch_bounds__(256) void k_down(DownArgs a) {
    RMRCM_RUN_GUARD(a.run);
    extern __shared__ double dvec[];   // nslot + 1
    constexpr int EMAX = 12;           // X row entries per lane held in registers
    const int node = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int r = blockIdx.y * nw + wave;
    const bool row = r < a.xi;
    const int ix = node % a.nodes_x, iy = node / a.nodes_x;
    const int c1 = a.cut == 0 ? iy * (2 * a.nodes_x) + 2 * ix : (2 * iy) * a.nodes_x + ix;
    // loads that do not need the data vector, in flight during its gather:
    // this wave's row of X and the segment its result goes to
    const double* xr = a.X + ((size_t)node * a.xi + (row ? r : 0)) * a.ld;
    double xv[EMAX];
#pragma unroll
    for (int u = 0; u < EMAX; ++u) {
        const int q = u * 64 + lane;
        xv[u] = (row && q < a.ld) ? xr[q] : 0.0;
    }
    int e = 0;
    if (row && lane == 0) e = a.css[(size_t)c1 * a.cnslot + a.gmap[r % a.g]] >> 1;
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
    if (!row) return;
    double sum = 0.0;
#pragma unroll
    for (int u = 0; u < EMAX; ++u) {
        const int q = u * 64 + lane;
        if (q < a.ld) sum = fma(xv[u], dvec[q], sum);
    }
    for (int q = EMAX * 64 + lane; q < a.ld; q += 64) sum = fma(xr[q], dvec[q], sum);
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
    if (lane == 0) {
        if (r < a.g) a.glo[e] = sum;
        else a.ghi[e] = sum;
    }
}

// ---------------------------------------------------------------- g > 128
// Merges whose gamma blocks exceed the register-resident inversion (one
// workgroup holds at most 128 x 128 in registers): the same quasi-definite
// elimination with the blocks in global memory.  D^{-1} and S^{-1} by
// blocked Gauss-Jordan over 128-wide panels (qd_big_inverse: the pivot
// block's inverse in registers on one workgroup per merge, the rest as
// products over many workgroups); E = D^{-1} B and S = N - B E, the four
// products of the column apply, and the parent traces, as matrix products
// on the FP64 matrix cores, batched over the level's merges.

// C = beta C + alpha A B for untransposed row-major operands, one 64 x 64
// tile of C per workgroup and batch entry blockIdx.z, four waves of 32 x 32
// (2 x 2 matrix-core tiles), K in steps of 32 through LDS with the next
// step's operands loaded into registers while the current step's products
// run (one load latency per step hidden behind 32 products per wave).  Each
// load instruction reads whole rows of a tile (32 consecutive doubles of A,
// 64 of B per group of lanes).  Optional tile flags skip the tiles of C whose
// rows (rflag[z][tile row]) or columns (cflag[z][tile column]) are known to
// be zero in A or B: the inactive boundary slots of a merge, whose trace
// rows and columns are zero; such a tile is left as it is, or zeroed when
// beta = 0.  With kpm, the parent traces' product (A: row o = parent slot o,
// columns [0, kh) the first child's gamma segments, [kh, 2 kh) the
// second's, zero outside the half of the child that owns the slot): the
// workgroup reads its rows' owners from the slot map and runs K only over
// the halves of the children present (the skipped products are exact
// zeros, so the sums are those of the full range).
struct GemmNN {
    int m, n, k;
    const double* A;
    long long lda, sa;
    const double* B;
    long long ldb, sb;
    double* C;
    long long ldc, sc;
    double alpha, beta;
    const unsigned char* rflag;   // [batch][rfs] or null
    const unsigned char* cflag;   // [batch][cfs] or null
    int rfs, cfs;
    int skr0, skr1;               // row tiles [skr0, skr1) skipped in every batch entry
    const int* run;
    const int* kpm;               // slot map (owner child in bits 24..) or null
    int kh;                       // gamma segments of one child (K = 2 kh) with kpm
};

constexpr int kGemmKT = 32;

// One 64 x 64 tile of the product A B into acc (wave w: rows 32 (w / 2)..,
// columns 32 (w % 2).., 2 x 2 matrix-core tiles): load_a(q, kk) gives the
// entry of A at the tile's row (tid / 32) + 8 q and column kk (zero outside
// the valid rows), Bb points at the tile's first column of B (row stride
// ldb, nc columns valid), K over [kbeg, kend) in steps of kGemmKT through the
// LDS tiles As and Bs, the next step's operands loaded into registers while
// the current step's products run.  Entries outside the valid columns and
// the K range are zero.
template <typename LoadA>
__device__ __forceinline__ void nn_tile(LoadA load_a, const double* __restrict__ Bb, long long ldb, int nc,
                                        int kbeg, int kend, double* As, double* Bs, v4d (&acc)[2][2]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
    // loader roles: A rows (tid / 32) + 8 q, column tid % 32; B rows
    // (tid / 64) + 4 q, column tid % 64
    const int ar = tid >> 5, ak = tid & 31, br = tid >> 6, bc = tid & 63;
    (void)ar;
    double ra[8], rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int kk = k0 + ak;
            ra[q] = kk < kend ? load_a(q, kk) : 0.0;
            const int kb = k0 + br + 4 * q;
            rb[q] = (kb < kend && bc < nc) ? Bb[(size_t)kb * ldb + bc] : 0.0;
        }
    };
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += kGemmKT) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            As[(ar + 8 * q) * (kGemmKT + 1) + ak] = ra[q];
            Bs[(br + 4 * q) * 65 + bc] = rb[q];
        }
        __syncthreads();
        if (k0 + kGemmKT < kend) load(k0 + kGemmKT);
#pragma unroll
        for (int s4 = 0; s4 < kGemmKT / 4; ++s4) {
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[(wr + 16 * a + li) * (kGemmKT + 1) + 4 * s4 + lk];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[(4 * s4 + lk) * 65 + wc + 16 * b + li];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f64(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
}

// A operand of nn_tile from a dense row-major block: Ab the tile's first
// row, row stride lda, mr rows valid.
struct DenseA {
    const double* __restrict__ Ab;
    long long lda;
    int mr;
    __device__ double operator()(int q, int kk) const {
        const int r = (int)(threadIdx.x >> 5) + 8 * q;
        return r < mr ? Ab[(size_t)r * lda + kk] : 0.0;
    }
};

__global__ __launch_bounds__(256) void k_gemm_nn_f64(GemmNN g) {
    RMRCM_RUN_GUARD(g.run);
    __shared__ double As[64 * (kGemmKT + 1)];
    __shared__ double Bs[kGemmKT * 65];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int bm = blockIdx.y * 64, bn = blockIdx.x * 64, z = blockIdx.z;
    double* C = g.C + (size_t)z * g.sc;
    const bool skip = (g.rflag && !g.rflag[(size_t)z * g.rfs + blockIdx.y]) ||
                      (g.cflag && !g.cflag[(size_t)z * g.cfs + blockIdx.x]) ||
                      ((int)blockIdx.y >= g.skr0 && (int)blockIdx.y < g.skr1);
    if (skip) {
        if (g.beta == 0.0)
            for (int t = tid; t < 64 * 64; t += 256) {
                const int r = bm + t / 64, cc = bn + t % 64;
                if (r < g.m && cc < g.n) C[(size_t)r * g.ldc + cc] = 0.0;
            }
        return;
    }
    const double* A = g.A + (size_t)z * g.sa;
    const double* B = g.B + (size_t)z * g.sb;
    const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
    int kbeg = 0, kend = g.k;
    if (g.kpm) {
        const int r = bm + (tid & 63);
        const int own = (tid < 64 && r < g.m) ? (g.kpm[r] >> 24) : -1;
        const int has0 = __syncthreads_or(own == 0), has1 = __syncthreads_or(own == 1);
        if (!has0) kbeg = g.kh;
        if (!has1) kend = g.kh;
    }
    v4d acc[2][2];
    nn_tile(DenseA{A + (size_t)bm * g.lda, g.lda, g.m - bm}, B + bn, g.ldb, g.n - bn, kbeg, kend, As, Bs, acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = bm + wr + 16 * a + lk + 4 * v, cc = bn + wc + 16 * b + li;
                if (r < g.m && cc < g.n) {
                    double* cp = C + (size_t)r * g.ldc + cc;
                    *cp = g.beta == 0.0 ? g.alpha * acc[a][b][v] : g.beta * *cp + g.alpha * acc[a][b][v];
                }
            }
}

static hipError_t gemm(rmrcm_ctx* c, int batch, int m, int n, int k, int ta, const double* A,
                       long long lda, long long sa, int tb, const double* B, long long ldb, long long sb,
                       double* C, long long ldc, long long sc, double alpha, double beta,
                       const unsigned char* rflag = nullptr, int rfs = 0,
                       const unsigned char* cflag = nullptr, int cfs = 0, int skr0 = 0, int skr1 = 0,
                       const int* kpm = nullptr, int kh = 0) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (!ta && !tb) {
        GemmNN g{m, n, k, A, lda, sa, B, ldb, sb, C, ldc, sc, alpha, beta, rflag, cflag, rfs, cfs, skr0, skr1,
                 c->run_ptr, kpm, kh};
        hipLaunchKernelGGL(k_gemm_nn_f64, dim3((n + 63) / 64, (m + 63) / 64, batch), dim3(256), 0, c->stream, g);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;             // every product here has untransposed operands
}

// Inverse of the n x n block (n <= 128) at src (row stride lds) into dst
// (row stride ldd; dst = src: in place) by one workgroup of QdM<128>::NT
// threads, blocked Gauss-Jordan in registers as in k_qd_factor_mfma.
__device__ __forceinline__ void invert_block128(const double* src, long long lds, double* dst, long long ldd,
                                                int n, int* flags) {
    typedef QdM<128> Q;
    constexpr int T = Q::T;
    __shared__ double cp[2 * 128 * Q::CPL];
    __shared__ double lts[2 * T * 16 * Q::LTL];
    __shared__ double pt[2 * 16 * 17];
    __shared__ int bad;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    if (tid == 0) bad = 0;
    const int j = 16 * w + li;
    v4d m[T];
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + lk + 4 * v;
            m[I][v] = (i < n && j < n) ? src[(size_t)i * lds + j] : (i == j ? 1.0 : 0.0);
        }
    __syncthreads();
    double* lt = lts + 2 * w * 16 * Q::LTL;
    qd_gj_mfma<128>(m, cp, pt, lt, lt + 16 * Q::LTL, &bad);
#pragma unroll
    for (int I = 0; I < T; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * I + lk + 4 * v;
            if (i < n && j < n) dst[(size_t)i * ldd + j] = m[I][v];
        }
    if (tid == 0 && bad) atomicOr(&flags[FLAG_MERGE_SINGULAR], 1);
}

// In-place inverse of the n x n block (n <= 128) at X (row stride ld, batch
// stride sx).
__global__ __launch_bounds__(QdM<128>::NT) void k_qd_invert_mfma(double* X, long long ld, long long sx,
                                                                  int n, int* flags) {
    double* Xb = X + (size_t)blockIdx.x * sx;
    invert_block128(Xb, ld, Xb, ld, n, flags);
}

// D, B and N of every merge of the level (one thread per entry; D to the D
// block, N parked in the S block).
__global__ __launch_bounds__(256) void k_qd_gather_big(MergeArgs a) {
    RMRCM_RUN_GUARD(a.run);
    const int node = blockIdx.y, g = a.g;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= g * g) return;
    const int i = t / g, j = t % g;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    const int gi = a.gmap[i], gj = a.gmap[j];
    const double t1 = T1[(size_t)gi * a.cld + gj];
    const double t2 = T2[(size_t)a.gmap[g + i] * a.cld + a.gmap[g + j]];
    const size_t gg = (size_t)g * g;
    double* Dg = a.M + (size_t)node * 4 * gg;
    double* Sg = Dg + 2 * gg;
    double* Bg = Dg + 3 * gg;
    const double nv = t1 + t2;
    double dv = nv;
    if (i == j) {
        const int e = a.css[(size_t)c1 * a.cnslot + gi] >> 1;
        dv = nv + 4.0 * (a.seglen[e] / (2.0 * a.beta[e]));
    }
    Bg[t] = t2 - t1;
    Sg[t] = nv;
    Dg[t] = dv;
}

// Blocks of the inverse from W (128 x r): X[0:128][128:] = -W and
// X[128:][0:128] = -W^T; mode 1: the all-Neumann top's pinned row and column
// of S set to the identity (before the inversion), mode 2: its pinned entry
// stored as zero (after).
__global__ __launch_bounds__(256) void k_qd_big_fix(double* X, long long ld, long long sx,
                                                    const double* W, long long sw, int r, int mode,
                                                    int g) {
    double* Xb = X + (size_t)blockIdx.y * sx;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (mode == 0) {
        if (t >= 128 * r) return;
        const int i = t / r, q = t % r;
        const double v = -W[(size_t)blockIdx.y * sw + t];
        Xb[(size_t)i * ld + 128 + q] = v;
        Xb[(size_t)(128 + q) * ld + i] = v;
    } else if (mode == 1) {
        if (t >= g) return;
        Xb[(size_t)(g - 1) * ld + t] = t == g - 1 ? 1.0 : 0.0;
        Xb[(size_t)t * ld + g - 1] = t == g - 1 ? 1.0 : 0.0;
    } else if (t == 0) {
        Xb[(size_t)(g - 1) * ld + g - 1] = 0.0;
    }
}

// Scratch of the inverse of order n: the column panel (n x 128), the pivot
// block (128 x 128) and the row panel (128 x n) of a Gauss-Jordan step.
__host__ inline size_t big_inv_work(int n) { return 2 * 128 * (size_t)n + 128 * 128; }

// Gauss-Jordan step at columns k0 .. k0 + kb - 1 of the n x n block X (row
// stride ld, merge stride sx), first launch: workgroup 0 of each merge
// inverts the pivot block X[k0:k0+kb, k0:k0+kb] into Pw (row stride kb),
// the others copy the column panel C = X[:, k0:k0+kb] into the merge's
// scratch (row stride kb).
__global__ __launch_bounds__(QdM<128>::NT) void k_gj_pivot(const double* X, long long ld, long long sx, int n,
                                                            int k0, int kb, double* W, long long sw, int* flags) {
    const double* Xb = X + (size_t)blockIdx.y * sx;
    double* C = W + (size_t)blockIdx.y * sw;
    double* Pw = C + (size_t)n * 128;
    if (blockIdx.x == 0) {
        invert_block128(Xb + (size_t)k0 * ld + k0, ld, Pw, kb, kb, flags);
        return;
    }
    const long long t = (long long)(blockIdx.x - 1) * QdM<128>::NT + threadIdx.x;
    if (t >= (long long)n * kb) return;
    const int i = (int)(t / kb), j = (int)(t % kb);
    C[(size_t)i * kb + j] = Xb[(size_t)i * ld + k0 + j];
}

// Last launch of the step (after R = Pw X[k0:k0+kb, :] into Rw, row stride
// n), one 64 x 64 tile of X per workgroup: the panel's rows take R and the
// pivot block Pw; the panel's columns -C Pw; every other tile X - C R.  The
// products are those of k_gemm_nn_f64 on the same operands.
__global__ __launch_bounds__(256) void k_gj_update(double* X, long long ld, long long sx, int n, int k0,
                                                   int kb, const double* W, long long sw) {
    __shared__ double As[64 * (kGemmKT + 1)];
    __shared__ double Bs[kGemmKT * 65];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
    double* Xb = X + (size_t)blockIdx.z * sx;
    const double* Cw = W + (size_t)blockIdx.z * sw;
    const double* Pw = Cw + (size_t)n * 128;
    const double* Rw = Pw + 128 * 128;
    if (bm >= k0 && bm < k0 + kb) {
        for (int t = tid; t < 64 * 64; t += 256) {
            const int r = bm + t / 64, cc = bn + t % 64;
            if (r < k0 + kb && cc < n)
                Xb[(size_t)r * ld + cc] = (cc >= k0 && cc < k0 + kb) ? Pw[(size_t)(r - k0) * kb + (cc - k0)]
                                                                      : Rw[(size_t)(r - k0) * n + cc];
        }
        return;
    }
    const bool colk = bn >= k0 && bn < k0 + kb;
    v4d acc[2][2];
    const DenseA ca{Cw + (size_t)bm * kb, kb, n - bm};
    if (colk) nn_tile(ca, Pw + (bn - k0), kb, k0 + kb - bn, 0, kb, As, Bs, acc);
    else nn_tile(ca, Rw + bn, n, n - bn, 0, kb, As, Bs, acc);
    const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = bm + wr + 16 * a + lk + 4 * v, cc = bn + wc + 16 * b + li;
                if (r < n && cc < n && (!colk || cc < k0 + kb)) {
                    double* cp = Xb + (size_t)r * ld + cc;
                    *cp = colk ? -1.0 * acc[a][b][v] : 1.0 * *cp + -1.0 * acc[a][b][v];
                }
            }
}

// In-place inverse of the n x n block at X (row stride ld, merge stride sx)
// of every merge, by blocked Gauss-Jordan without pivoting (the blocks of D
// and S are definite, so their leading blocks and Schur complements are), in
// panels of 128: per step K with pivot block P = X_KK^{-1} (registers, one
// workgroup per merge),
//     R = P X_K,:      X_I,: -= X_IK R  (I != K)      X_IK = -X_IK P      X_K,: = R, X_KK = P
// with the old column panel X_:,K kept in scratch, in three launches per
// step: the pivot block's inverse beside the copy of the column panel
// (k_gj_pivot), R, and every tile's share of the rest (k_gj_update).  Every
// product has K = 128 (short chains over many workgroups); scratch per
// merge from Wb (stride sw).
static hipError_t qd_big_inverse(rmrcm_ctx* c, const MergeArgs& a, double* X, int n, long long ld,
                                 long long sx, double* Wb, long long sw) {
    const int nb = a.nnodes;
    if (n <= 128) {
        hipLaunchKernelGGL(k_qd_invert_mfma, dim3(nb), dim3(QdM<128>::NT), 0, c->stream, X, ld, sx, n, a.flags);
        return hipGetLastError();
    }
    double* Pw = Wb + (size_t)n * 128;       // kb x kb; the column panel C (n x kb) before it
    double* Rw = Pw + 128 * 128;             // kb x n
    hipError_t e;
    const unsigned tiles = (unsigned)((n + 63) / 64);
    for (int k0 = 0; k0 < n; k0 += 128) {
        const int kb = n - k0 < 128 ? n - k0 : 128;
        const unsigned blocks = 1 + (unsigned)(((long long)n * kb + QdM<128>::NT - 1) / QdM<128>::NT);
        hipLaunchKernelGGL(k_gj_pivot, dim3(blocks, nb), dim3(QdM<128>::NT), 0, c->stream, (const double*)X, ld,
                           sx, n, k0, kb, Wb, sw, a.flags);
        // R = P X_K,:  (the pivot block's own columns give P X_KK = I, replaced by P)
        if ((e = gemm(c, nb, kb, n, kb, 0, Pw, kb, sw, 0, X + (size_t)k0 * ld, ld, sx, Rw, n, sw, 1.0, 0.0)))
            return e;
        hipLaunchKernelGGL(k_gj_update, dim3(tiles, tiles, nb), dim3(256), 0, c->stream, X, ld, sx, n, k0, kb,
                           (const double*)Wb, sw);
    }
    return hipGetLastError();
}

// Scratch per merge with g > 128: the inverses', three g x (nslot + 1) column
// blocks of the apply, and the gathered trace rows (nslot x 2g).
__host__ inline size_t big_work(int g, int nslot) {
    return big_inv_work(g) + 3 * (size_t)g * (nslot + 1) + (size_t)nslot * 2 * g;
}

// Scratch per merge with g > 128 (merge stride big_work): Y and W of the
// inverses, then three g x (nslot + 1) column blocks of the apply.
static hipError_t qd_factor_big(rmrcm_ctx* c, const MergeArgs& a) {
    const int g = a.g, nb = a.nnodes;
    const long long gg = (long long)g * g, sx = 4 * gg, sw = (long long)big_work(g, a.nslot);
    double* D = a.M;
    double* E = a.M + gg;
    double* S = a.M + 2 * gg;
    double* B = a.M + 3 * gg;
    hipLaunchKernelGGL(k_qd_gather_big, dim3((g * g + 255) / 256, nb), dim3(256), 0, c->stream, a);
    hipError_t e;
    if ((e = qd_big_inverse(c, a, D, g, g, sx, a.work, sw))) return e;
    // E = D^{-1} B;  S = N - B E
    if ((e = gemm(c, nb, g, g, g, 0, D, g, sx, 0, B, g, sx, E, g, sx, 1.0, 0.0))) return e;
    if ((e = gemm(c, nb, g, g, g, 0, B, g, sx, 0, E, g, sx, S, g, sx, -1.0, 1.0))) return e;
    if (a.pin)
        hipLaunchKernelGGL(k_qd_big_fix, dim3((g + 255) / 256, nb), dim3(256), 0, c->stream, S, (long long)g, sx,
                           (const double*)nullptr, 0LL, 0, 1, g);
    if ((e = qd_big_inverse(c, a, S, g, g, sx, a.work, sw))) return e;
    if (a.pin)
        hipLaunchKernelGGL(k_qd_big_fix, dim3(1, nb), dim3(256), 0, c->stream, S, (long long)g, sx,
                           (const double*)nullptr, 0LL, 0, 2, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// General interface spaces: U_H constant on segments of mu pieces and P_H on
// segments of mp pieces (one of the two counts is 1; the gamma pieces of a
// segment are consecutive, the first at a multiple of the count).  The
// merge system of the pieces in the variables (P, V) (V = beta U, sum and
// difference of the one-sided data) is
//     [N B; B D] (P; V) = -(r1 + r2; r2 - r1)
// and the general spaces restrict it to P = F Ph, V = E Vh (E, F: 0/1
// expansions from segments to pieces) with the equations summed over the
// same segments (eq. 13.2 tested on P-segments, eq. 14.2 on U-segments):
//     [F^T N F  F^T B E; E^T B F  E^T D E] (Ph; Vh) = -(F^T (r1 + r2); E^T (r2 - r1)).
// Its elimination (Dh = E^T D E, Sh = F^T (N - B E Dh^-1 E^T B) F) gives
//     P = F Sh^-1 F^T (rs - B t),   t = E Dh^-1 E^T rd,   V = t - (E Dh^-1 E^T B) P,
// the column formulas of the pieces' merge with D^-1 -> E Dh^-1 E^T and
// S^-1 -> F Sh^-1 F^T; stored so expanded, the column kernels of every tier
// apply the general merge unchanged.  Dh is definite (D is) and Sh is the
// Schur complement of the restricted quasi-definite system.
__global__ __launch_bounds__(256) void k_gs_restrict(const double* __restrict__ X, long long sx, int g, int m,
                                                     double* __restrict__ Y, long long sy) {
    const int n = g / m;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)n * n) return;
    const int a = (int)(t / n), b = (int)(t % n);
    const double* Xb = X + (size_t)blockIdx.y * sx;
    double v = 0.0;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) v += Xb[(size_t)(a * m + i) * g + b * m + j];
    Y[(size_t)blockIdx.y * sy + t] = v;
}

__global__ __launch_bounds__(256) void k_gs_expand(const double* __restrict__ Y, long long sy, int g, int m,
                                                   double* __restrict__ X, long long sx) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)g * g) return;
    const int i = (int)(t / g), j = (int)(t % g), n = g / m;
    X[(size_t)blockIdx.y * sx + t] = Y[(size_t)blockIdx.y * sy + (size_t)(i / m) * n + j / m];
}

static bool general_spaces(const rmrcm_ctx* c) { return c->geo.mu > 1 || c->geo.mp > 1; }

// Factor of a general-spaces merge: the blocks of the pieces (as for the
// long interfaces), Dh and Sh restricted, inverted and expanded into the
// D^-1, E and S^-1 slots.  Scratch: big_work per merge (the inverses' and
// the apply's), then the restricted block of every merge (g^2 each).
static hipError_t gs_factor(rmrcm_ctx* c, const MergeArgs& a) {
    const int g = a.g, nb = a.nnodes, mu = c->geo.mu, mp = c->geo.mp;
    const int gu = g / mu, gp = g / mp;
    const long long gg = (long long)g * g, sx = 4 * gg, sw = (long long)big_work(g, a.nslot);
    double* D = a.M;
    double* E = a.M + gg;
    double* S = a.M + 2 * gg;
    double* B = a.M + 3 * gg;
    double* H = a.work + (size_t)nb * big_work(g, a.nslot);
    const long long sh = gg;
    const dim3 full((unsigned)((gg + 255) / 256), nb);
    hipLaunchKernelGGL(k_qd_gather_big, full, dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_gs_restrict, dim3((unsigned)(((long long)gu * gu + 255) / 256), nb), dim3(256), 0,
                       c->stream, (const double*)D, sx, g, mu, H, sh);
    hipError_t e;
    if ((e = qd_big_inverse(c, a, H, gu, gu, sh, a.work, sw))) return e;
    hipLaunchKernelGGL(k_gs_expand, full, dim3(256), 0, c->stream, (const double*)H, sh, g, mu, D, sx);
    // E = (E Dh^-1 E^T) B;  S = N - B E
    if ((e = gemm(c, nb, g, g, g, 0, D, g, sx, 0, B, g, sx, E, g, sx, 1.0, 0.0))) return e;
    if ((e = gemm(c, nb, g, g, g, 0, B, g, sx, 0, E, g, sx, S, g, sx, -1.0, 1.0))) return e;
    hipLaunchKernelGGL(k_gs_restrict, dim3((unsigned)(((long long)gp * gp + 255) / 256), nb), dim3(256), 0,
                       c->stream, (const double*)S, sx, g, mp, H, sh);
    // all-Neumann top: the last P-segment's pressure pinned
    if (a.pin)
        hipLaunchKernelGGL(k_qd_big_fix, dim3((gp + 255) / 256, nb), dim3(256), 0, c->stream, H, (long long)gp, sh,
                           (const double*)nullptr, 0LL, 0, 1, gp);
    if ((e = qd_big_inverse(c, a, H, gp, gp, sh, a.work, sw))) return e;
    if (a.pin)
        hipLaunchKernelGGL(k_qd_big_fix, dim3(1, nb), dim3(256), 0, c->stream, H, (long long)gp, sh,
                           (const double*)nullptr, 0LL, 0, 2, gp);
    hipLaunchKernelGGL(k_gs_expand, full, dim3(256), 0, c->stream, (const double*)H, sh, g, mp, S, sx);
    return hipGetLastError();
}

// r1 + r2 and r2 - r1 of columns [col0, col0 + ncol) (row stride ncol), and
// the coefficients X from s and d.
__global__ __launch_bounds__(256) void k_qd_rhs_big(MergeArgs a, int col0, int ncol, double* RS,
                                                    double* RD, long long sw) {
    RMRCM_RUN_GUARD(a.run);
    const int node = blockIdx.y, g = a.g;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= g * ncol) return;
    const int i = t / ncol, cc = t % ncol, col = col0 + cc;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* T1 = a.Tc + (size_t)c1 * a.cnslot * a.cld;
    const double* T2 = a.Tc + (size_t)c2 * a.cnslot * a.cld;
    double v1 = 0.0, v2 = 0.0;
    if (col == a.nslot) {
        v1 = T1[(size_t)a.gmap[i] * a.cld + a.cld - 1];
        v2 = T2[(size_t)a.gmap[g + i] * a.cld + a.cld - 1];
    } else {
        const int pm = a.pmap[col], off = pm & 0xffffff;
        if ((pm >> 24) == 0) v1 = T1[(size_t)a.gmap[i] * a.cld + off];
        else v2 = T2[(size_t)a.gmap[g + i] * a.cld + off];
    }
    RS[(size_t)node * sw + t] = v1 + v2;
    RD[(size_t)node * sw + t] = v2 - v1;
}

__global__ __launch_bounds__(256) void k_qd_x_big(MergeArgs a, int col0, int ncol, const double* Sv,
                                                  const double* Dv, long long sw) {
    RMRCM_RUN_GUARD(a.run);
    const int node = blockIdx.y, g = a.g;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= g * ncol) return;
    const int i = t / ncol, cc = t % ncol;
    const double s = Sv[(size_t)node * sw + t], d = Dv[(size_t)node * sw + t];
    double* X = a.X + (size_t)node * a.xi * a.ld;
    X[(size_t)i * a.ld + col0 + cc] = -(s - d);
    X[(size_t)(g + i) * a.ld + col0 + cc] = -(s + d);
}

// Parent traces of merges beyond 128 gamma segments as a matrix product:
// Tp = direct + A X with A[o][k g + i] = T_k[o's slot in child k][gamma_k(i)]
// for the child k that owns slot o (zero in the other child's half), the
// terms and their sum being those of k_qd_trace_mfma.
__global__ __launch_bounds__(256) void k_qd_trace_rows_big(MergeArgs a, double* Ar, long long sw) {
    RMRCM_RUN_GUARD(a.run);
    const int node = blockIdx.y, g = a.g;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)a.nslot * 2 * g) return;
    const int o = (int)(t / (2 * g)), q = (int)(t % (2 * g)), k = q / g, i = q % g;
    int c1, c2;
    children(a, node, &c1, &c2);
    const int pm = a.pmap[o];
    double v = 0.0;
    if ((pm >> 24) == k) {
        const double* Tk = a.Tc + (size_t)(k == 0 ? c1 : c2) * a.cnslot * a.cld;
        v = Tk[(size_t)(pm & 0xffffff) * a.cld + a.gmap[k * g + i]];
    }
    Ar[(size_t)node * sw + t] = v;
}

__global__ __launch_bounds__(256) void k_qd_trace_direct_big(MergeArgs a, int col0, int ncol) {
    RMRCM_RUN_GUARD(a.run);
    const int node = blockIdx.y;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)a.nslot * ncol) return;
    const int o = (int)(t / ncol), col = col0 + (int)(t % ncol);
    int c1, c2;
    children(a, node, &c1, &c2);
    const int pm = a.pmap[o], k = pm >> 24;
    const double* tr = a.Tc + (size_t)(k == 0 ? c1 : c2) * a.cnslot * a.cld + (size_t)(pm & 0xffffff) * a.cld;
    const int pc = col < a.nslot ? a.pmap[col] : -1;
    const double d = col == a.nslot ? tr[a.cld - 1] : ((pc >> 24) == k ? tr[pc & 0xffffff] : 0.0);
    a.Tp[(size_t)node * a.nslot * a.ld + (size_t)o * a.ld + col] = d;
}

// The same parent traces in one launch, one 64 x 64 tile of Tp per
// workgroup (columns [col0, col0 + ncol)): the left operand is gathered
// from the owning child's trace row through the slot map and the gamma map
// (staged in LDS for the tile's K range), the direct term is added in the
// epilogue, tiles of inactive slots
// take the direct terms alone, and K runs over the halves of the children
// present in the tile's rows, as in k_gemm_nn_f64 with kpm: the operands and
// sums of k_qd_trace_rows_big, k_qd_trace_direct_big and k_gemm_nn_f64.
__host__ __device__ inline size_t trace_gemm_lds(int g) {
    return sizeof(double) * (64 * (kGemmKT + 1) + kGemmKT * 65) + sizeof(int) * 2 * (size_t)g;
}

__global__ __launch_bounds__(256) void k_qd_trace_gemm(MergeArgs a, int col0, int ncol) {
    RMRCM_RUN_GUARD(a.run);
    extern __shared__ double tgs[];
    double* As = tgs;
    double* Bs = As + 64 * (kGemmKT + 1);
    int* gms = reinterpret_cast<int*>(Bs + kGemmKT * 65);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int node = blockIdx.z, g = a.g, nslot = a.nslot;
    const int bm = blockIdx.y * 64, bn = blockIdx.x * 64;
    int c1, c2;
    children(a, node, &c1, &c2);
    const double* Tk[2] = {a.Tc + (size_t)c1 * a.cnslot * a.cld, a.Tc + (size_t)c2 * a.cnslot * a.cld};
    double* Tp = a.Tp + (size_t)node * nslot * a.ld + col0;
    const double* X = a.X + (size_t)node * a.xi * a.ld + col0;
    const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
    const bool skip = a.tflag && (!a.tflag[(size_t)node * a.ntiles + blockIdx.y] ||
                                  (col0 == 0 && !a.tflag[(size_t)node * a.ntiles + blockIdx.x]));
    v4d acc[2][2];
    if (skip) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    } else {
        int kbeg = 0, kend = 2 * g;
        {
            const int r = bm + (tid & 63);
            const int own = (tid < 64 && r < nslot) ? (a.pmap[r] >> 24) : -1;
            const int has0 = __syncthreads_or(own == 0), has1 = __syncthreads_or(own == 1);
            if (!has0) kbeg = g;
            if (!has1) kend = g;
        }
        for (int t = tid; t < kend - kbeg; t += 256) gms[t] = a.gmap[kbeg + t];
        // this thread's A rows (tid / 32) + 8 q: owner and trace row
        int own[8];
        const double* trow[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int o = bm + (tid >> 5) + 8 * q;
            const int pm = o < nslot ? a.pmap[o] : -1;
            own[q] = pm >= 0 ? (pm >> 24) : -1;
            trow[q] = Tk[own[q] == 1 ? 1 : 0] + (size_t)(pm >= 0 ? (pm & 0xffffff) : 0) * a.cld;
        }
        __syncthreads();
        auto load_a = [&](int q, int kk) -> double {
            return own[q] == (kk >= g ? 1 : 0) ? trow[q][gms[kk - kbeg]] : 0.0;
        };
        nn_tile(load_a, X + bn, a.ld, ncol - bn, kbeg, kend, As, Bs, acc);
    }
    // direct terms of this lane's outputs (rows wr + 16 i + lk + 4 v,
    // columns wc + 16 j + li of the tile), loaded after the products so
    // that they hold no registers across them
    double dr[2][2][4];
    {
        int pc[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = col0 + bn + wc + 16 * j + li;
            pc[j] = col < nslot ? a.pmap[col] : -1;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = bm + wr + 16 * i + lk + 4 * v;
                const int pm = o < nslot ? a.pmap[o] : 0, k = pm >> 24;
                const double* tr = Tk[k & 1] + (size_t)(pm & 0xffffff) * a.cld;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int cc = bn + wc + 16 * j + li, col = col0 + cc;
                    double d = 0.0;
                    if (o < nslot && cc < ncol)
                        d = col == nslot ? tr[a.cld - 1] : ((pc[j] >> 24) == k ? tr[pc[j] & 0xffffff] : 0.0);
                    dr[i][j][v] = d;
                }
            }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int o = bm + wr + 16 * i + lk + 4 * v, cc = bn + wc + 16 * j + li;
                if (o < nslot && cc < ncol) {
                    const double r = skip ? dr[i][j][v] : 1.0 * dr[i][j][v] + 1.0 * acc[i][j][v];
                    Tp[(size_t)o * a.ld + cc] = r;
                }
            }
}

static hipError_t qd_trace_big(rmrcm_ctx* c, const MergeArgs& a, int col0, int ncol) {
    const int g = a.g, nb = a.nnodes;
    if (trace_gemm_lds(g) <= 64 * 1024) {
        hipLaunchKernelGGL(k_qd_trace_gemm, dim3((ncol + 63) / 64, (a.nslot + 63) / 64, nb), dim3(256),
                           trace_gemm_lds(g), c->stream, a, col0, ncol);
        return hipGetLastError();
    }
    const long long sw = (long long)big_work(g, a.nslot);
    double* Ar = a.work + big_inv_work(g) + 3 * (size_t)g * (a.nslot + 1);
    const long long nr = (long long)a.nslot * 2 * g, nd = (long long)a.nslot * ncol;
    hipLaunchKernelGGL(k_qd_trace_rows_big, dim3((unsigned)((nr + 255) / 256), nb), dim3(256), 0, c->stream, a, Ar, sw);
    hipLaunchKernelGGL(k_qd_trace_direct_big, dim3((unsigned)((nd + 255) / 256), nb), dim3(256), 0, c->stream, a,
                       col0, ncol);
    // rows of inactive parent slots are zero in Ar, columns of inactive slots
    // zero in X
    return gemm(c, nb, a.nslot, ncol, 2 * g, 0, Ar, 2 * g, sw, 0, a.X + col0, a.ld, (long long)a.xi * a.ld,
                a.Tp + col0, a.ld, (long long)a.nslot * a.ld, 1.0, 1.0, a.tflag, a.ntiles,
                col0 == 0 ? a.tflag : nullptr, a.ntiles, 0, 0, a.pmap, g);
}

// y = alpha A x + beta y for the g x g block A of every merge (row-major,
// merge stride sa) and vectors x, y (merge strides sv): one wave per row,
// lane l summing the entries l, l + 64, ... (each load instruction reads 64
// consecutive entries of the row), the lane sums added by shuffles.  The
// long interfaces' single-column apply (the particular column of the root
// in a step), where a tiled product would leave most of the chip idle.
__global__ __launch_bounds__(256) void k_matvec_big(int g, const double* __restrict__ A, long long sa,
                                                    const double* __restrict__ x, double* y, long long sv,
                                                    double alpha, double beta, const int* run) {
    RMRCM_RUN_GUARD(run);
    const int lane = threadIdx.x & 63, row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= g) return;
    const double* Ar = A + (size_t)blockIdx.y * sa + (size_t)row * g;
    const double* xv = x + (size_t)blockIdx.y * sv;
    double s = 0.0;
    for (int j = lane; j < g; j += 64) s = fma(Ar[j], xv[j], s);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) {
        double* yr = y + (size_t)blockIdx.y * sv + row;
        *yr = beta == 0.0 ? alpha * s : beta * *yr + alpha * s;
    }
}

static hipError_t qd_apply_big(rmrcm_ctx* c, const MergeArgs& a, int col0, int ncol) {
    const int g = a.g, nb = a.nnodes;
    const long long gg = (long long)g * g, sx = 4 * gg;
    const size_t per = big_work(g, a.nslot);
    if ((size_t)ncol > (size_t)a.nslot + 1) return hipErrorInvalidValue;
    // per merge: RS, RD, TT of g x ncol each, after the inverses' scratch
    double* RS = a.work + big_inv_work(g);
    double* RD = RS + (size_t)g * (a.nslot + 1);
    double* TT = RD + (size_t)g * (a.nslot + 1);
    const long long sw = (long long)per;
    const double* D = a.M;
    const double* E = a.M + gg;
    const double* S = a.M + 2 * gg;
    const double* B = a.M + 3 * gg;
    const dim3 grid((g * ncol + 255) / 256, nb);
    hipLaunchKernelGGL(k_qd_rhs_big, grid, dim3(256), 0, c->stream, a, col0, ncol, RS, RD, sw);
    hipError_t e;
    // columns of inactive slots are zero in every right-hand side block
    const unsigned char* cf = col0 == 0 ? a.tflag : nullptr;
    const int cs = a.ntiles;
    if (ncol == 1) {
        const dim3 mg((g + 3) / 4, nb);
        const struct { const double *A, *x; double* y; double alpha, beta; } mv[4] = {
            {D, RD, TT, 1.0, 0.0}, {B, TT, RS, -1.0, 1.0}, {S, RS, RD, 1.0, 0.0}, {E, RD, TT, -1.0, 1.0}};
        for (const auto& m : mv) {
            hipLaunchKernelGGL(k_matvec_big, mg, dim3(256), 0, c->stream, g, m.A, sx, m.x, m.y, sw, m.alpha,
                               m.beta, c->run_ptr);
            if ((e = hipGetLastError())) return e;
        }
        hipLaunchKernelGGL(k_qd_x_big, grid, dim3(256), 0, c->stream, a, col0, ncol, (const double*)RD,
                           (const double*)TT, sw);
        return hipGetLastError();
    }
    if ((e = gemm(c, nb, g, ncol, g, 0, D, g, sx, 0, RD, ncol, sw, TT, ncol, sw, 1.0, 0.0, nullptr, 0, cf, cs))) return e;   // t
    if ((e = gemm(c, nb, g, ncol, g, 0, B, g, sx, 0, TT, ncol, sw, RS, ncol, sw, -1.0, 1.0, nullptr, 0, cf, cs))) return e;  // u
    if ((e = gemm(c, nb, g, ncol, g, 0, S, g, sx, 0, RS, ncol, sw, RD, ncol, sw, 1.0, 0.0, nullptr, 0, cf, cs))) return e;   // s
    if ((e = gemm(c, nb, g, ncol, g, 0, E, g, sx, 0, RD, ncol, sw, TT, ncol, sw, -1.0, 1.0, nullptr, 0, cf, cs))) return e;  // d
    hipLaunchKernelGGL(k_qd_x_big, grid, dim3(256), 0, c->stream, a, col0, ncol, (const double*)RD,
                       (const double*)TT, sw);
    return hipGetLastError();
}

// One depth of the downward pass as k_down_sub takes it: that depth's merge
// grid, gamma length, interface and slot counts, and X.
struct DownLevel {
    int nodes_x, nodes_y, g, xi, nslot, ld;
    const double* X;
};
static constexpr int kDownSubMax = 6;     // depths per launch
static constexpr int kDownZero = -1;      // source codes of data-vector entries
static constexpr int kDownPart = -0x7fffffff;
struct DownSubArgs {
    DownLevel lv[kDownSubMax];
    int toff[kDownSubMax], roff[kDownSubMax];
    int n, entries, results;
    const int* tab;     // [subtrees][entries]
    double* glo;
    double* ghi;
    const int* run;
};

// The downward pass of n consecutive depths with short interfaces for the
// subtree of one merge of the first of them per workgroup.  A merge's gamma
// data depend on its ancestors only, so the depths follow one another inside
// the workgroup, and the data an ancestor in the subtree produced are taken
// from LDS: a table built at setup gives every entry of every depth's data
// vectors its source (an earlier depth's result in LDS, the subtree
// boundary's Robin datum in global memory, zero on the domain boundary, 1
// for the particular column) and every result its segment.  Every global
// load is issued at the start: the table, the boundary data and, for every
// depth, this lane's entries of its row of X (each (merge, gamma row) pair of
// a depth is one group of lpr consecutive lanes, each lane holding every
// lpr-th entry of the row).  Then per depth the LDS-sourced entries are
// copied, the partial dot products summed across each group, and the results
// written to LDS and to the Robin datum of the row's side of its segment.
static constexpr int kDownSubThreads = 512;
static constexpr int kDownSubEntries = 12;   // X row entries per lane and depth held in registers

__global__ __launch_bounds__(kDownSubThreads) void k_down_sub(DownSubArgs A) {
    RMRCM_RUN_GUARD(A.run);
    extern __shared__ double sm[];
    constexpr int EMAX = kDownSubEntries;
    double* dall = sm;                 // [entries] data vectors of every depth
    double* res = dall + A.entries;    // [results] gamma data of every depth
    int* src = (int*)(res + A.results);
    int* dst = src + A.entries;        // [results] segment of every result
    const int tid = threadIdx.x, nt = blockDim.x;
    const int rx0 = A.lv[0].nodes_x, ry0 = A.lv[0].nodes_y;
    const int ix0 = blockIdx.x % rx0, iy0 = blockIdx.x / rx0;
    const int* tab = A.tab + (size_t)blockIdx.x * (A.entries + A.results);
    // this lane's group at depth l: lanes per row, lane in the row, merge, row
    auto lanes = [&](int l, int& lpr, int& j, int& k, int& r, bool& act) {
        const DownLevel a = A.lv[l];
        const int R = (a.nodes_x / rx0) * (a.nodes_y / ry0) * a.xi;
        lpr = 64;
        while (lpr > 1 && lpr * R > nt) lpr >>= 1;
        const int p = tid / lpr;
        j = tid % lpr;
        act = p < R;
        k = act ? p / a.xi : 0;
        r = act ? p % a.xi : 0;
    };
    auto row_ptr = [&](int l, int k, int r) {
        const DownLevel a = A.lv[l];
        const int fx = a.nodes_x / rx0, fy = a.nodes_y / ry0;
        const int node = (iy0 * fy + k / fx) * a.nodes_x + ix0 * fx + k % fx;
        return a.X + ((size_t)node * a.xi + r) * a.ld;
    };
    double xv[kDownSubMax][EMAX];
#pragma unroll
    for (int l = 0; l < kDownSubMax; ++l) {
        if (l < A.n) {
            int lpr, j, k, r;
            bool act;
            lanes(l, lpr, j, k, r, act);
            const double* xr = row_ptr(l, k, r);
            const int ld = A.lv[l].ld;
#pragma unroll
            for (int u = 0; u < EMAX; ++u) {
                const int q = j + u * lpr;
                xv[l][u] = (act && q < ld) ? xr[q] : 0.0;
            }
        }
    }
    for (int t = tid; t < A.entries; t += nt) {
        const int sc = tab[t];
        double v = 0.0;
        if (sc == kDownPart) v = 1.0;
        else if (sc <= -2) {
            const int code = -2 - sc;
            v = (code & 1) ? A.glo[code >> 1] : A.ghi[code >> 1];
        }
        src[t] = sc;
        dall[t] = v;
    }
    for (int t = tid; t < A.results; t += nt) dst[t] = tab[A.entries + t];
    __syncthreads();
#pragma unroll
    for (int l = 0; l < kDownSubMax; ++l) {
        if (l >= A.n) break;
        const DownLevel a = A.lv[l];
        const int w = a.nslot + 1, ne = (a.nodes_x / rx0) * (a.nodes_y / ry0) * w;
        for (int t = A.toff[l] + tid; t < A.toff[l] + ne; t += nt) {
            const int sc = src[t];
            if (sc >= 0) dall[t] = res[sc];
        }
        __syncthreads();
        int lpr, j, k, r;
        bool act;
        lanes(l, lpr, j, k, r, act);
        const double* dv = dall + A.toff[l] + (size_t)k * w;
        double sum = 0.0;
#pragma unroll
        for (int u = 0; u < EMAX; ++u) {
            const int q = j + u * lpr;
            if (act && q < a.ld) sum = fma(xv[l][u], dv[q], sum);
        }
        if (act && j + EMAX * lpr < a.ld) {
            const double* xr = row_ptr(l, k, r);
            for (int q = j + EMAX * lpr; q < a.ld; q += lpr) sum = fma(xr[q], dv[q], sum);
        }
        for (int off = lpr >> 1; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        if (act && j == 0) {
            const int o = A.roff[l] + k * a.xi + r;
            res[o] = sum;
            if (r < a.g) A.glo[dst[o]] = sum;
            else A.ghi[dst[o]] = sum;
        }
        __syncthreads();
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
    a.gseg = P.gseg;
    a.M = P.M;
    a.X = P.X;
    a.Tp = P.T;
    a.beta = c->beta;
    a.seglen = c->seglen;
    a.flags = c->flags;
    a.pin = (d == 0 && !c->any_dirichlet) ? 1 : 0;
    a.work = P.work;
    a.tflag = P.tflag;
    a.ntiles = (P.nslot + 1 + 63) / 64;
    a.run = c->run_ptr;
    return a;
}


// Size class of the merge: register-resident tiers up to 128; 256 stands for
// every larger gamma (the blocks in global memory).
static int qd_tier(int g) { return g <= 16 ? 16 : g <= 32 ? 32 : g <= 64 ? 64 : g <= 128 ? 128 : 256; }

// ct: columns per workgroup, 16 or 32 (0: 16).
template <int GT>
static hipError_t qd_apply(rmrcm_ctx* c, const MergeArgs& a, int col0, int ncol, int ct) {
    const dim3 block(64 * qd_apply_waves<GT>());
    if (ct == 32 && ncol > 16)
        hipLaunchKernelGGL((k_qd_apply_mfma<GT, 2>), dim3(a.nnodes, (ncol + 31) / 32), block, 0,
                           c->stream, a, col0, ncol);
    else
        hipLaunchKernelGGL((k_qd_apply_mfma<GT, 1>), dim3(a.nnodes, (ncol + 15) / 16), block, 0,
                           c->stream, a, col0, ncol);
    return hipGetLastError();
}

// Levels whose column apply and parent traces run fused (k_qd_cols_mfma).
static bool cols_fused(const MergeArgs& a, bool trace) {
    return trace && a.g > 16 && a.g <= 64 && a.nslot <= 512;
}

template <int GT>
static hipError_t qd_columns(rmrcm_ctx* c, const MergeArgs& a, int col0, int ncol, bool trace, int ct) {
    if constexpr (GT == 32 || GT == 64) {
        if (cols_fused(a, trace)) {
            // at most one row tile per wave (up to four workgroups per tile)
            const int z = std::min(4, ((a.nslot + 15) / 16 + 7) / 8);
            hipLaunchKernelGGL(k_qd_cols_mfma<GT>, dim3(a.nnodes, (ncol + 15) / 16, std::max(z, 1)), dim3(512), 0,
                               c->stream, a, col0, ncol);
            return hipGetLastError();
        }
    }
    hipError_t e = qd_apply<GT>(c, a, col0, ncol, ct);
    if (e != hipSuccess) return e;
    if (trace)
        hipLaunchKernelGGL(k_qd_trace_mfma<GT>, dim3(a.nnodes, (a.nslot + 63) / 64, (ncol + 15) / 16),
                           dim3(256), 0, c->stream, a, col0, ncol);
    return hipGetLastError();
}

template <int GT>
static hipError_t qd_factor_mfma(rmrcm_ctx* c, const MergeArgs& a) {
    if (GT == 128) {
        // the largest tier (the top merges): the products between the two
        // inversions on T workgroups per merge
        hipLaunchKernelGGL(k_qd_factor_mfma<GT>, dim3(a.nnodes), dim3(QdM<GT>::NT), 0, c->stream, a, 1);
        hipLaunchKernelGGL(k_qd_es_mfma<GT>, dim3(a.nnodes, QdM<GT>::T), dim3(QdM<GT>::NT), 0, c->stream, a);
        hipLaunchKernelGGL(k_qd_factor_mfma<GT>, dim3(a.nnodes), dim3(QdM<GT>::NT), 0, c->stream, a, 2);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_qd_factor_mfma<GT>, dim3(a.nnodes), dim3(QdM<GT>::NT), 0, c->stream, a, 0);
    return hipGetLastError();
}

static hipError_t qd_factor_any(rmrcm_ctx* c, const MergeArgs& a) {
    switch (qd_tier(a.g)) {
        case 256: return qd_factor_big(c, a);
        case 16: return qd_factor_mfma<16>(c, a);
        case 32: return qd_factor_mfma<32>(c, a);
        case 64: return qd_factor_mfma<64>(c, a);
        case 128: return qd_factor_mfma<128>(c, a);
    }
    return hipErrorInvalidValue;
}

static hipError_t qd_columns_any(rmrcm_ctx* c, const MergeArgs& a, int col0, int ncol, bool trace,
                                 int ct) {
    switch (qd_tier(a.g)) {
        case 16: return qd_columns<16>(c, a, col0, ncol, trace, ct);
        case 32: return qd_columns<32>(c, a, col0, ncol, trace, ct);
        case 64: return qd_columns<64>(c, a, col0, ncol, trace, ct);
        case 128:
            // long parent columns: the products over many workgroups (the
            // blocks are stored as for the longer interfaces)
            if (a.work) {
                hipError_t e = qd_apply_big(c, a, col0, ncol);
                if (e != hipSuccess || !trace) return e;
                return qd_trace_big(c, a, col0, ncol);
            }
            return qd_columns<128>(c, a, col0, ncol, trace, ct);
        case 256: {
            hipError_t e = qd_apply_big(c, a, col0, ncol);
            if (e != hipSuccess || !trace) return e;
            return qd_trace_big(c, a, col0, ncol);
        }
    }
    return hipErrorInvalidValue;
}

size_t merge_work_doubles(const rmrcm_ctx* c, const Level& L) {
    if (general_spaces(c)) return (size_t)L.nnodes * (big_work(L.g, L.nslot) + (size_t)L.g * L.g);
    return L.g >= 128 ? (size_t)L.nnodes * big_work(L.g, L.nslot) : 0;
}

bool merge_apply_tunable(rmrcm_ctx* c, int d) {
    if (!(d > 0 && d < c->D)) return false;
    const MergeArgs a = make_args(c, d);
    if (general_spaces(c)) return false;
    if (small_merge_ok(a, d, a.nslot) || small_merge_ok(a, d, a.nslot + 1)) return false;   // fused merge
    if (cols_fused(a, true)) return false;                                                    // fused columns
    return qd_tier(a.g) < 128;
}

hipError_t launch_merge_apply(rmrcm_ctx* c, int d, int ct) {
    if (!merge_apply_tunable(c, d)) return hipErrorInvalidValue;
    MergeArgs a = make_args(c, d);
    switch (qd_tier(a.g)) {
        case 16: return qd_apply<16>(c, a, 0, a.nslot, ct);
        case 32: return qd_apply<32>(c, a, 0, a.nslot, ct);
        case 64: return qd_apply<64>(c, a, 0, a.nslot, ct);
        case 128: return qd_apply<128>(c, a, 0, a.nslot, ct);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_merge_setup(rmrcm_ctx* c, int d, bool part) {
    MergeArgs a = make_args(c, d);
    if (d == 0) a.Tp = nullptr;
    const int ncol = a.nslot + (part ? 1 : 0);
    if (general_spaces(c)) {
        hipError_t e = gs_factor(c, a);
        if (e != hipSuccess || d == 0) return e;
        return qd_columns_any(c, a, 0, ncol, true, c->ct_tune[d]);
    }
    if (small_merge_ok(a, d, ncol)) {
        const int nrt = small_ns16(a.nslot) / 16;
        const dim3 grid(a.nnodes), block(64 * small_waves(ncol));
        const size_t lds = small_lds_bytes(ncol, a.nslot);
        if (nrt <= 2) hipLaunchKernelGGL(k_qd_small<2>, grid, block, lds, c->stream, a, ncol);
        else if (nrt <= 4) hipLaunchKernelGGL(k_qd_small<4>, grid, block, lds, c->stream, a, ncol);
        else hipLaunchKernelGGL(k_qd_small<8>, grid, block, lds, c->stream, a, ncol);
        return hipGetLastError();
    }
    hipError_t e = qd_factor_any(c, a);
    if (e != hipSuccess || d == 0) return e;     // the root has no boundary columns
    return qd_columns_any(c, a, 0, ncol, true, c->ct_tune[d]);
}

hipError_t launch_merge_particular(rmrcm_ctx* c, int d) {
    MergeArgs a = make_args(c, d);
    if (d == 0) a.Tp = nullptr;
    if (d == 0) {
        // the top: one merge, one column (and the root's downward step when
        // root_down_fused)
        double* gl = c->root_down_fused ? c->glo : nullptr;
        double* gh = c->root_down_fused ? c->ghi : nullptr;
        switch (qd_tier(a.g)) {
            case 16: hipLaunchKernelGGL(k_qd_apply_vec<16>, dim3(a.nnodes), dim3(128), 0, c->stream, a, a.nslot, gl, gh); return hipGetLastError();
            case 32: hipLaunchKernelGGL(k_qd_apply_vec<32>, dim3(a.nnodes), dim3(256), 0, c->stream, a, a.nslot, gl, gh); return hipGetLastError();
            case 64: hipLaunchKernelGGL(k_qd_apply_vec<64>, dim3(a.nnodes), dim3(512), 0, c->stream, a, a.nslot, gl, gh); return hipGetLastError();
            case 128: hipLaunchKernelGGL(k_qd_apply_vec<128>, dim3(a.nnodes), dim3(1024), 0, c->stream, a, a.nslot, gl, gh); return hipGetLastError();
        }
    }
    return qd_columns_any(c, a, a.nslot, 1, d != 0, 1);
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
    a.run = c->run_ptr;
    const size_t lds = sizeof(double) * (size_t)(P.nslot + 1);
    hipLaunchKernelGGL(k_down, dim3(P.nnodes, (P.xi + 3) / 4), dim3(256), lds, c->stream, a);
    return hipGetLastError();
}

// The downward pass of every depth: one launch per depth while the
// interfaces are long, then up to kDownSubMax remaining depths with
// interfaces of at most kDownSubXi unknowns in one launch (k_down_sub), if
// every depth's rows fit the workgroup and the data vectors, results and
// source table fit LDS.  Sources: the writer of every (segment, side) datum
// among the fused depths is found by the same rule k_down_sub applies.
// Builds the host table only (c->h_down_tab); the device copy is the
// caller's.
static constexpr int kDownSubXi = 32;

int build_down_sub(rmrcm_ctx* c) {
    const int D = c->D;
    c->down_ds = D;
    // the root's downward step inside the top's particular column: when
    // every root slot is on the domain boundary and the top takes the
    // register-resident column kernel
    c->root_down_fused = false;
    if (D > 0 && c->levels[0].g <= 128 && c->levels[0].nnodes == 1) {
        bool all_boundary = true;
        for (int code : c->levels[0].h_slotseg) all_boundary = all_boundary && code < 0;
        c->root_down_fused = all_boundary;
    }
    int ds = D;
    while (ds > 0 && D - ds < kDownSubMax && c->levels[ds - 1].xi <= kDownSubXi) --ds;
    if (D - ds < 2) return RMRCM_OK;
    const int n = D - ds, NS = c->levels[ds].nnodes;
    const int rx0 = c->levels[ds].nodes_x, ry0 = c->levels[ds].nodes_y;
    int E = 0, RT = 0;
    int toff[kDownSubMax], roff[kDownSubMax];
    for (int l = 0; l < n; ++l) {
        const Level& P = c->levels[ds + l];
        const int nsub = P.nnodes / NS;
        if (nsub * P.xi > kDownSubThreads) return RMRCM_OK;
        toff[l] = E;
        roff[l] = RT;
        E += nsub * (P.nslot + 1);
        RT += nsub * P.xi;
    }
    if ((size_t)(E + RT) * 12 > 48 * 1024) return RMRCM_OK;
    // writer of every (segment, side) datum: depth l, global node, row
    struct W {
        int l, node, r;
    };
    std::vector<std::pair<long long, W>> writers;
    for (int l = 0; l < n; ++l) {
        const Level& P = c->levels[ds + l];
        const Level& C = c->levels[ds + l + 1];
        for (int m = 0; m < P.nnodes; ++m) {
            const int ix = m % P.nodes_x, iy = m / P.nodes_x;
            const int c1 = P.cut == 0 ? iy * (2 * P.nodes_x) + 2 * ix : (2 * iy) * P.nodes_x + ix;
            for (int r = 0; r < P.xi; ++r) {
                const int e = C.h_slotseg[(size_t)c1 * C.nslot + P.h_gmap[r % P.g]] >> 1;
                writers.push_back({2LL * e + (r < P.g ? 1 : 0), W{l, m, r}});
            }
        }
    }
    std::sort(writers.begin(), writers.end(),
              [](const std::pair<long long, W>& x, const std::pair<long long, W>& y) { return x.first < y.first; });
    auto find = [&](long long key) -> const W* {
        auto it = std::lower_bound(writers.begin(), writers.end(), key,
                                   [](const std::pair<long long, W>& x, long long k) { return x.first < k; });
        return (it != writers.end() && it->first == key) ? &it->second : nullptr;
    };
    const size_t TW = (size_t)E + RT;      // per subtree: sources, then result segments
    std::vector<int> tab((size_t)NS * TW);
    for (int st = 0; st < NS; ++st) {
        const int ix0 = st % rx0, iy0 = st / rx0;
        for (int l = 0; l < n; ++l) {
            const Level& P = c->levels[ds + l];
            const int fx = P.nodes_x / rx0, fy = P.nodes_y / ry0, w = P.nslot + 1;
            for (int kk = 0; kk < fx * fy; ++kk) {
                const int nd = (iy0 * fy + kk / fx) * P.nodes_x + ix0 * fx + kk % fx;
                for (int sl = 0; sl < w; ++sl) {
                    int sc;
                    if (sl == P.nslot) {
                        sc = kDownPart;
                    } else {
                        const int code = P.h_slotseg[(size_t)nd * P.nslot + sl];
                        if (code < 0) {
                            sc = kDownZero;
                        } else {
                            sc = -2 - code;
                            const W* wr = find(2LL * (code >> 1) + (code & 1));
                            if (wr && wr->l < l) {
                                const Level& Q = c->levels[ds + wr->l];
                                const int qx = Q.nodes_x / rx0, qy = Q.nodes_y / ry0;
                                const int mx = wr->node % Q.nodes_x - ix0 * qx, my = wr->node / Q.nodes_x - iy0 * qy;
                                if (mx >= 0 && mx < qx && my >= 0 && my < qy)
                                    sc = roff[wr->l] + (my * qx + mx) * Q.xi + wr->r;
                            }
                        }
                    }
                    tab[(size_t)st * TW + toff[l] + kk * w + sl] = sc;
                }
            }
            // the segment of every result (row r of merge kk)
            const Level& C = c->levels[ds + l + 1];
            for (int kk = 0; kk < fx * fy; ++kk) {
                const int ix = ix0 * fx + kk % fx, iy = iy0 * fy + kk / fx;
                const int c1 = P.cut == 0 ? iy * (2 * P.nodes_x) + 2 * ix : (2 * iy) * P.nodes_x + ix;
                for (int r = 0; r < P.xi; ++r)
                    tab[(size_t)st * TW + E + roff[l] + kk * P.xi + r] =
                        C.h_slotseg[(size_t)c1 * C.nslot + P.h_gmap[r % P.g]] >> 1;
            }
        }
    }
    c->h_down_tab.swap(tab);   // the caller allocates down_tab and uploads it
    c->down_ds = ds;
    c->down_entries = E;
    c->down_results = RT;
    for (int l = 0; l < n; ++l) {
        c->down_toff[l] = toff[l];
        c->down_roff[l] = roff[l];
    }
    return RMRCM_OK;
}

hipError_t launch_down_all(rmrcm_ctx* c) {
    const int ds = c->down_ds;
    for (int d = c->root_down_fused ? 1 : 0; d < ds; ++d) {
        hipError_t e = launch_down(c, d);
        if (e != hipSuccess) return e;
    }
    if (ds == c->D) return hipSuccess;
    DownSubArgs A;
    A.n = c->D - ds;
    A.entries = c->down_entries;
    A.results = c->down_results;
    A.tab = c->down_tab;
    A.glo = c->glo;
    A.ghi = c->ghi;
    A.run = c->run_ptr;
    for (int l = 0; l < A.n; ++l) {
        const Level& P = c->levels[ds + l];
        DownLevel& a = A.lv[l];
        a.nodes_x = P.nodes_x;
        a.nodes_y = P.nodes_y;
        a.g = P.g;
        a.xi = P.xi;
        a.nslot = P.nslot;
        a.ld = P.ld;
        a.X = P.X;
        A.toff[l] = c->down_toff[l];
        A.roff[l] = c->down_roff[l];
    }
    const size_t lds = (size_t)(A.entries + A.results) * (sizeof(double) + sizeof(int));
    hipLaunchKernelGGL(k_down_sub, dim3(c->levels[ds].nnodes), dim3(kDownSubThreads), lds, c->stream, A);
    return hipGetLastError();
}

}  // namespace rmrcm
