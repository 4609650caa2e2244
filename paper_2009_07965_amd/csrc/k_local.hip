// Local Robin solves on every finest subdomain.
//
// The local problem of Section 2 (eq. 11.2-12.2) with the lowest-order
// Raviart-Thomas / lumped-mass discretisation is a symmetric positive
// definite five-point system A on the bx*by cells of a subdomain.  A Robin
// face of cell c on segment e adds |f| / (rho_c + beta_e) to the diagonal
// and, for the basis problem of that segment (Section 2.1, the basis
// problems with unit interface datum), the same amount to the right-hand
// side.
//
// Factorisation: band Cholesky with half-bandwidth bx, blocked by grid
// rows (block size = bandwidth, the blocking of LAPACK's band Cholesky).
// With cells numbered row by row, A is block tridiagonal with dense
// diagonal blocks A_jj (tridiagonal) and diagonal couplings -D_j between
// rows j and j+1.  For each block row j:
//     L_j L_j^T = S_j                      (Cholesky of the Schur complement)
//     P_j = S_j^{-1} = L_j^{-T} L_j^{-1}   (inverted diagonal block)
//     S_{j+1} = A_{j+1,j+1} - D_j P_j D_j  (trailing update)
// and the multi-RHS sweeps become products with P_j:
//     forward:  w_j = P_j (f_j + D_{j-1} w_{j-1})
//     backward: x_j = w_j + P_j D_j x_{j+1}.
// P_j is kept for every row (the factor store), so a later right-hand side
// (the particular solution at solve time) needs only the two sweeps.

#include "rmrcm_internal.h"

namespace rmrcm {

// ---------------------------------------------------------------- helpers
__device__ inline double cellK(const double* __restrict__ K, const Geo& g, int gi, int gj) {
    return K[(size_t)gj * g.nx + gi];
}

// Transmissibility of the x-face between (gi,gj) and (gi+1,gj).
__device__ inline double trans_x(const double* __restrict__ K, const Geo& g, int gi, int gj) {
    const double ra = g.hx / (2.0 * cellK(K, g, gi, gj));
    const double rb = g.hx / (2.0 * cellK(K, g, gi + 1, gj));
    return g.hy / (ra + rb);
}

// Transmissibility of the y-face between (gi,gj) and (gi,gj+1).
__device__ inline double trans_y(const double* __restrict__ K, const Geo& g, int gi, int gj) {
    const double ra = g.hy / (2.0 * cellK(K, g, gi, gj));
    const double rb = g.hy / (2.0 * cellK(K, g, gi, gj + 1));
    return g.hx / (ra + rb);
}

// Slot index of the boundary face of a subdomain cell on side s (0 W, 1 E,
// 2 S, 3 N); pos = j for W/E and i for S/N.
__device__ inline int slot_of(const Geo& g, int side, int pos) {
    const int t = pos / g.sg;
    return side == 0 ? t : side == 1 ? g.nsy + t : side == 2 ? 2 * g.nsy + t
                                                                 : 2 * g.nsy + g.nsx + t;
}

// Index of an outer boundary face in the W E S N list.
__device__ inline int outer_face(const Geo& g, int side, int gi, int gj) {
    return side == 0 ? gj : side == 1 ? g.ny + gj : side == 2 ? 2 * g.ny + gi
                                                                 : 2 * g.ny + g.nx + gi;
}

// Conductance of the subdomain-boundary face of local cell (i, j) on side
// s.  Sets *slot to the Robin slot (or -1) and *outer to the outer-face
// index (or -1).
__device__ inline double bface(const Geo& g, const double* __restrict__ K,
                               const int8_t* __restrict__ bct, const double* __restrict__ beta,
                               const int* __restrict__ ss, int I, int J, int i, int j, int side,
                               int* slot, int* outer) {
    const int gi = I * g.bx + i, gj = J * g.by + j;
    const double kc = cellK(K, g, gi, gj);
    const double area = side < 2 ? g.hy : g.hx;
    const double rho = (side < 2 ? g.hx : g.hy) / (2.0 * kc);
    const int a = slot_of(g, side, side < 2 ? j : i);
    const int code = ss[a];
    if (code >= 0) {
        *slot = a;
        *outer = -1;
        return area / (rho + beta[code >> 1]);
    }
    *slot = -1;
    const int f = outer_face(g, side, gi, gj);
    *outer = f;
    return bct[f] == RMRCM_BC_DIRICHLET ? area / rho : 0.0;
}

// ---------------------------------------------------------------- K0
// Robin parameter per segment: beta_e = alpha * Hbar_e / Keff_e with Keff
// the mean over the segment's faces of the harmonic mean of the two
// adjacent permeabilities (Section 5.1).
__global__ void k_beta(Geo g, const double* __restrict__ K, double* __restrict__ beta,
                       double* __restrict__ seglen) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.nseg) return;
    double hsum = 0.0, len;
    if (e < g.nv) {
        const int I = e / g.lines_v + 1, k = e % g.lines_v;
        const int ilo = I * g.bx - 1;
        for (int t = 0; t < g.sg; ++t) {
            const int j = k * g.sg + t;
            const double a = cellK(K, g, ilo, j), b = cellK(K, g, ilo + 1, j);
            hsum += 2.0 * a * b / (a + b);
        }
        len = g.sg * g.hy;
    } else {
        const int r = e - g.nv;
        const int J = r / g.lines_h + 1, k = r % g.lines_h;
        const int jlo = J * g.by - 1;
        for (int t = 0; t < g.sg; ++t) {
            const int i = k * g.sg + t;
            const double a = cellK(K, g, i, jlo), b = cellK(K, g, i, jlo + 1);
            hsum += 2.0 * a * b / (a + b);
        }
        len = g.sg * g.hx;
    }
    const double keff = hsum / g.sg;
    beta[e] = g.alpha * len / keff;
    seglen[e] = len;
}

// Flags a permeability that is not finite and positive.
__global__ void k_check_perm(const double* __restrict__ K, size_t n, int* __restrict__ flags) {
    bool bad = false;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x) {
        const double v = K[t];
        bad |= !(v > 0.0) || !(v <= 1.7976931348623157e308);
    }
    if (bad) atomicOr(&flags[FLAG_BAD_PERM], 1);
}

// Boundary faces of a subdomain, numbered W (by faces, bottom to top), E
// (by), S (bx faces, left to right), N (bx).  The prologue of each local
// kernel stores, per face, its conductance (Robin |f|/(rho+beta), Dirichlet
// |f|/rho, or 0 for Neumann), its Robin slot (or -1) and its outer-face
// index (or -1) in LDS.
__device__ inline void face_cell(const Geo& g, int BX, int f, int* side, int* i, int* j) {
    const int BY = g.by;
    if (f < BY) { *side = 0; *i = 0; *j = f; }
    else if (f < 2 * BY) { *side = 1; *i = BX - 1; *j = f - BY; }
    else if (f < 2 * BY + BX) { *side = 2; *i = f - 2 * BY; *j = 0; }
    else { *side = 3; *i = f - 2 * BY - BX; *j = BY - 1; }
}

__device__ inline int face_of_slot(const Geo& g, int BX, int a, int t) {
    // t-th face (0..sg-1) of slot a
    const int BY = g.by;
    if (a < g.nsy) return a * g.sg + t;
    if (a < 2 * g.nsy) return BY + (a - g.nsy) * g.sg + t;
    if (a < 2 * g.nsy + g.nsx) return 2 * BY + (a - 2 * g.nsy) * g.sg + t;
    return 2 * BY + BX + (a - 2 * g.nsy - g.nsx) * g.sg + t;
}

template <int BX>
__device__ void face_prologue(const Geo& g, const double* __restrict__ K,
                              const int8_t* __restrict__ bct, const double* __restrict__ beta,
                              const int* __restrict__ ss, int I, int J, double* cf, int* rs,
                              int* of) {
    const int NF = 2 * (BX + g.by);
    for (int f = threadIdx.x; f < NF; f += blockDim.x) {
        int side, i, j;
        face_cell(g, BX, f, &side, &i, &j);
        int sl, o;
        cf[f] = bface(g, K, bct, beta, ss, I, J, i, j, side, &sl, &o);
        rs[f] = sl;
        of[f] = o;
    }
}

__device__ inline double tpx(const Geo& g, double ka, double kb) {
    return g.hy / (g.hx / (2.0 * ka) + g.hx / (2.0 * kb));
}
__device__ inline double tpy(const Geo& g, double ka, double kb) {
    return g.hx / (g.hy / (2.0 * ka) + g.hy / (2.0 * kb));
}

// Permeabilities around cell (i, j) of the subdomain: centre, left, right,
// below, above (the neighbours outside the subdomain are not read).
template <int BX>
__device__ inline void load_kstencil(const Geo& g, const double* __restrict__ K, int I, int J,
                                     int i, int j, double kv[5]) {
    const int gi = I * BX + i, gj = J * g.by + j;
    const double* row = K + (size_t)gj * g.nx + gi;
    kv[0] = row[0];
    kv[1] = i > 0 ? row[-1] : 1.0;
    kv[2] = i < BX - 1 ? row[1] : 1.0;
    kv[3] = j > 0 ? row[-(ptrdiff_t)g.nx] : 1.0;
    kv[4] = j < g.by - 1 ? row[g.nx] : 1.0;
}

// Row coefficients of cell (i, j): diagonal, coupling to (i+1, j) and to
// (i, j+1).
template <int BX>
__device__ inline void stencil_coeffs(const Geo& g, const double kv[5], const double* cf, int i,
                                      int j, double* dg, double* txr, double* tyu) {
    const int BY = g.by;
    const double txl = i > 0 ? tpx(g, kv[1], kv[0]) : cf[j];
    const double tr = i < BX - 1 ? tpx(g, kv[0], kv[2]) : 0.0;
    const double tyd = j > 0 ? tpy(g, kv[3], kv[0]) : cf[2 * BY + i];
    const double tu = j < BY - 1 ? tpy(g, kv[0], kv[4]) : 0.0;
    *dg = txl + (i < BX - 1 ? tr : cf[BY + j]) + tyd + (j < BY - 1 ? tu : cf[2 * BY + BX + i]);
    *txr = tr;
    *tyu = tu;
}

// Adds the basis right-hand side of block row j (unit Robin datum on one
// slot per column) to F (BX x R).
template <int BX>
__device__ inline void add_basis_rhs(const Geo& g, const double* cf, const int* rs, int j, int R,
                                     double* F) {
    const int lane = threadIdx.x, BY = g.by;
    if (lane == 0 && rs[j] >= 0) F[rs[j]] += cf[j];
    if (lane == 1 && rs[BY + j] >= 0) F[(BX - 1) * R + rs[BY + j]] += cf[BY + j];
    __syncthreads();
    if ((j == 0 || j == BY - 1) && lane < BX) {
        const int f = (j == 0 ? 2 * BY : 2 * BY + BX) + lane;
        if (rs[f] >= 0) F[lane * R + rs[f]] += cf[f];   // one (row, column) per lane
    }
    __syncthreads();
}

// Value of a double held by lane l (l uniform, a compile-time constant at
// every call) as a wave-uniform scalar.
__device__ inline double readlane_d(double v, int l) {
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffull), l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

constexpr int kWPre = 16;   // basis columns prefetched per lane in the backward sweep

// ---------------------------------------------------------------- K1
// Factorisation and basis solves: one wavefront per subdomain.
//
// Lane l < 2 BX owns column l of the augmented block [S_j | I] of the
// current block row in registers.  Cholesky step k: the pivot comes from
// lane k, row k is scaled by 1/sqrt(pivot), and by symmetry of the trailing
// block the multiplier of row i > k is the scaled row-k entry held by lane
// i, read as a wave-uniform scalar.  After BX steps lanes BX..2BX-1 hold
// L_j^{-1}; P_j = L_j^{-T} L_j^{-1} is formed column by column (lane c
// computes column c, which is also row c), stored, and used for the sweep
// w_j = P_j z_j and the trailing update S_{j+1} = A_{j+1} - D_j P_j D_j.
// Global loads are issued one row ahead of their use.
template <int BX>
__global__ __launch_bounds__(64) void k_local_setup(Geo g, const double* __restrict__ K,
                                                    const int8_t* __restrict__ bct,
                                                    const double* __restrict__ beta,
                                                    const int* __restrict__ slotseg, int R,
                                                    double* __restrict__ Pstore,
                                                    double* __restrict__ Psi,
                                                    double* __restrict__ T, int ld,
                                                    int* __restrict__ flags) {
    extern __shared__ double sm[];
    constexpr int LT = BX + 1;             // padded row of L^{-T}
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    double* LTs = sm;                       // BX x LT: row c = column c of L^{-1}
    double* Z = LTs + BX * LT;              // BX x R: z_j, later D_j x_{j+1}
    double* Wl = Z + BX * R;                // BX x R: w_j, later x_j
    double* tys = Wl + BX * R;              // BY x BX: couplings D_j
    double* cf = tys + BY * BX;             // NF face conductances
    int* rs = (int*)(cf + NF);              // NF Robin slots
    int* of = rs + NF;                      // NF outer faces

    const int lane = threadIdx.x;
    const int sub = blockIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    double* Ps = Pstore + (size_t)sub * BY * BX * BX;
    double* Psub = Psi + (size_t)sub * R * n;

    const bool scol = lane < BX;                    // column of S
    const bool icol = lane >= BX && lane < 2 * BX;  // column of the identity block
    const int c = scol ? lane : (icol ? lane - BX : 0);

    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    double kv[5], kn[5];
    load_kstencil<BX>(g, K, I, J, c, 0, kv);
    for (int t = lane; t < BX * R; t += 64) Z[t] = 0.0;
    __syncthreads();

    double a[BX];
    double p[BX];
    int sing = 0;
    double dg, txr, tyu;
    stencil_coeffs<BX>(g, kv, cf, c, 0, &dg, &txr, &tyu);
    double txl = __shfl(txr, lane > 0 ? lane - 1 : 0, 64);
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        double v = 0.0;
        if (scol) v = (i == c) ? dg : (i == c + 1) ? -txr : (i + 1 == c) ? -txl : 0.0;
        else if (icol) v = (i == c) ? 1.0 : 0.0;
        a[i] = v;
    }
    add_basis_rhs<BX>(g, cf, rs, 0, R, Z);

    for (int j = 0; j < BY; ++j) {
        if (j + 1 < BY) load_kstencil<BX>(g, K, I, J, c, j + 1, kn);
        // ---- Cholesky of S_j fused with the inversion of its factor
#pragma unroll
        for (int k = 0; k < BX; ++k) {
            double d = readlane_d(a[k], k);
            if (!(d > 0.0)) {
                sing = 1;
                d = 1.0;
            }
            const double r = 1.0 / sqrt(d);
            a[k] *= r;
#pragma unroll
            for (int i = k + 1; i < BX; ++i) a[i] = fma(-readlane_d(a[k], i), a[k], a[i]);
        }
        // ---- P_j = L^{-T} L^{-1}
        if (icol) {
#pragma unroll
            for (int i = 0; i < BX; ++i) LTs[c * LT + i] = a[i];
        }
        __syncthreads();
        if (scol) {
#pragma unroll
            for (int r = 0; r < BX; ++r) p[r] = 0.0;
#pragma unroll
            for (int i = 0; i < BX; ++i) {
                const double lci = LTs[c * LT + i];
#pragma unroll
                for (int r = 0; r <= i; ++r) p[r] = fma(LTs[r * LT + i], lci, p[r]);
            }
#pragma unroll
            for (int r = 0; r < BX; ++r) Ps[(size_t)j * BX * BX + r * BX + c] = p[r];
            // w_j = P_j z_j: lane c computes row c (P symmetric)
            for (int q = 0; q < R; ++q) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < BX; ++k) s = fma(p[k], Z[k * R + q], s);
                Wl[c * R + q] = s;
                Psub[(size_t)q * n + j * BX + c] = s;
            }
            tys[j * BX + c] = tyu;    // D_j
        }
        __syncthreads();
        if (j + 1 < BY) {
            const double dc = tyu;
            stencil_coeffs<BX>(g, kn, cf, c, j + 1, &dg, &txr, &tyu);
            txl = __shfl(txr, lane > 0 ? lane - 1 : 0, 64);
#pragma unroll
            for (int i = 0; i < BX; ++i) {
                double v = 0.0;
                if (scol) {
                    v = -p[i] * (tys[j * BX + i] * dc);
                    if (i == c) v += dg;
                    else if (i == c + 1) v -= txr;
                    else if (i + 1 == c) v -= txl;
                } else if (icol) {
                    v = (i == c) ? 1.0 : 0.0;
                }
                a[i] = v;
            }
            // z_{j+1} = F_{j+1} + D_j w_j
            for (int t = lane; t < BX * R; t += 64) Z[t] = tys[j * BX + t / R] * Wl[t];
            __syncthreads();
            add_basis_rhs<BX>(g, cf, rs, j + 1, R, Z);
        }
    }
    // ---- backward sweep: x_{BY-1} = w_{BY-1}; x_j = w_j + P_j D_j x_{j+1}
    // Wl holds x_{j+1}; lane c loads row c of P_j (= column c) and its own
    // row of w_j one step ahead.
    double pn[BX];
    double wn[kWPre];
    if (scol && BY > 1) {
#pragma unroll
        for (int k = 0; k < BX; ++k) pn[k] = Ps[(size_t)(BY - 2) * BX * BX + k * BX + c];
#pragma unroll
        for (int q = 0; q < kWPre; ++q)
            wn[q] = q < R ? Psub[(size_t)q * n + (BY - 2) * BX + c] : 0.0;
    }
    for (int j = BY - 2; j >= 0; --j) {
        double wc[kWPre];
#pragma unroll
        for (int k = 0; k < BX; ++k) p[k] = pn[k];
#pragma unroll
        for (int q = 0; q < kWPre; ++q) wc[q] = wn[q];
        if (scol && j > 0) {
#pragma unroll
            for (int k = 0; k < BX; ++k) pn[k] = Ps[(size_t)(j - 1) * BX * BX + k * BX + c];
#pragma unroll
            for (int q = 0; q < kWPre; ++q)
                wn[q] = q < R ? Psub[(size_t)q * n + (j - 1) * BX + c] : 0.0;
        }
        for (int t = lane; t < BX * R; t += 64) Z[t] = tys[j * BX + t / R] * Wl[t];
        __syncthreads();
        if (scol) {
#pragma unroll
            for (int q = 0; q < kWPre; ++q) {
                if (q < R) {
                    double s = wc[q];
#pragma unroll
                    for (int k = 0; k < BX; ++k) s = fma(p[k], Z[k * R + q], s);
                    Wl[c * R + q] = s;
                    Psub[(size_t)q * n + j * BX + c] = s;
                }
            }
            for (int q = kWPre; q < R; ++q) {
                double s = Psub[(size_t)q * n + j * BX + c];
#pragma unroll
                for (int k = 0; k < BX; ++k) s = fma(p[k], Z[k * R + q], s);
                Wl[c * R + q] = s;
                Psub[(size_t)q * n + j * BX + c] = s;
            }
        }
        __syncthreads();
    }
    // ---- traces T[a][b] = sum_{f in slot a} c_f (x_b(cell f) - delta_ab)
    double* Tsub = T + (size_t)sub * R * ld;
    for (int t = lane; t < R * R; t += 64) {
        const int ar = t / R, b = t % R;
        double s = 0.0;
        if (ss[ar] >= 0 && ss[b] >= 0) {
            const double* col = Psub + (size_t)b * n;
            for (int u = 0; u < g.sg; ++u) {
                const int f = face_of_slot(g, BX, ar, u);
                int side, i, jj;
                face_cell(g, BX, f, &side, &i, &jj);
                s += cf[f] * (col[jj * BX + i] - (ar == b ? 1.0 : 0.0));
            }
        }
        Tsub[(size_t)ar * ld + b] = s;
    }
    if (lane == 0 && sing) atomicOr(&flags[FLAG_LOCAL_SINGULAR], 1);
}

// ---------------------------------------------------------------- K1p
// Particular solution (source and outer boundary data, zero Robin data)
// with the stored P_j: one wavefront per subdomain, lane c holding row c of
// P_j; writes pbar and the particular trace column.  A subdomain whose
// right-hand side vanishes has pbar = 0 and is finished at once.
template <int BX>
__device__ inline double part_rhs(const Geo& g, const double* cf, const int* of,
                                  const int8_t* __restrict__ bct, const double* __restrict__ bcv,
                                  double qv, int i, int j) {
    const int BY = g.by;
    double f = qv;
    const int faces[4] = {i == 0 ? j : -1, i == BX - 1 ? BY + j : -1, j == 0 ? 2 * BY + i : -1,
                          j == BY - 1 ? 2 * BY + BX + i : -1};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int fc = faces[s];
        if (fc < 0) continue;
        const int o = of[fc];
        if (o >= 0) f += bct[o] == RMRCM_BC_DIRICHLET ? cf[fc] * bcv[o] : -bcv[o];
    }
    return f;
}

template <int BX>
__global__ __launch_bounds__(64) void k_local_particular(
    Geo g, const double* __restrict__ K, const int8_t* __restrict__ bct,
    const double* __restrict__ beta, const int* __restrict__ slotseg, int R,
    const double* __restrict__ q, const double* __restrict__ bcv,
    const double* __restrict__ Pstore, double* __restrict__ pbar, double* __restrict__ T, int ld) {
    extern __shared__ double sm[];
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    double* fs = sm;                  // n right-hand side
    double* z = fs + n;               // BX
    double* cf = z + BX;              // NF
    int* rs = (int*)(cf + NF);
    int* of = rs + NF;
    __shared__ int nonzero;
    const int lane = threadIdx.x;
    const int sub = blockIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    const double* Ps = Pstore + (size_t)sub * BY * BX * BX;
    double* pb = pbar + (size_t)sub * n;
    double* Tsub = T + (size_t)sub * R * ld;
    const bool act = lane < BX;
    const int c = act ? lane : 0;

    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    if (lane == 0) nonzero = 0;
    __syncthreads();
    bool nz = false;
    for (int t = lane; t < n; t += 64) {
        const int i = t % BX, j = t / BX;
        const double qv = q ? q[(size_t)(J * BY + j) * g.nx + I * BX + i] : 0.0;
        const double f = part_rhs<BX>(g, cf, of, bct, bcv, qv, i, j);
        fs[t] = f;
        nz |= f != 0.0;
    }
    if (nz) nonzero = 1;
    __syncthreads();
    if (!nonzero) {
        for (int t = lane; t < n; t += 64) pb[t] = 0.0;
        for (int a = lane; a < R; a += 64) Tsub[(size_t)a * ld + ld - 1] = 0.0;
        return;
    }
    double p[BX], pn[BX];
    if (act) {
#pragma unroll
        for (int k = 0; k < BX; ++k) pn[k] = Ps[(size_t)k * BX + c];
    }
    double w = 0.0, dprev = 0.0;
    double kv[5];
    for (int j = 0; j < BY; ++j) {
#pragma unroll
        for (int k = 0; k < BX; ++k) p[k] = pn[k];
        if (act && j + 1 < BY) {
#pragma unroll
            for (int k = 0; k < BX; ++k) pn[k] = Ps[(size_t)(j + 1) * BX * BX + k * BX + c];
        }
        load_kstencil<BX>(g, K, I, J, c, j, kv);
        if (act) z[c] = fs[j * BX + c] + dprev * w;
        __syncthreads();
        if (act) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < BX; ++k) s = fma(p[k], z[k], s);
            w = s;
            fs[j * BX + c] = s;
            dprev = j + 1 < BY ? tpy(g, kv[0], kv[4]) : 0.0;
            pb[j * BX + c] = dprev;   // D_j staged in the output; overwritten at the end
        }
        __syncthreads();
    }
    // Here fs holds w_j (row by row) and pb holds D_j.
    if (act && BY > 1) {
#pragma unroll
        for (int k = 0; k < BX; ++k) pn[k] = Ps[(size_t)(BY - 2) * BX * BX + k * BX + c];
    }
    for (int j = BY - 2; j >= 0; --j) {
#pragma unroll
        for (int k = 0; k < BX; ++k) p[k] = pn[k];
        if (act && j > 0) {
#pragma unroll
            for (int k = 0; k < BX; ++k) pn[k] = Ps[(size_t)(j - 1) * BX * BX + k * BX + c];
        }
        if (act) z[c] = pb[j * BX + c] * w;
        __syncthreads();
        if (act) {
            double s = fs[j * BX + c];
#pragma unroll
            for (int k = 0; k < BX; ++k) s = fma(p[k], z[k], s);
            w = s;
            fs[j * BX + c] = s;
        }
        __syncthreads();
    }
    for (int t = lane; t < n; t += 64) pb[t] = fs[t];
    __syncthreads();
    for (int a = lane; a < R; a += 64) {
        double s = 0.0;
        if (ss[a] >= 0)
            for (int u = 0; u < g.sg; ++u) {
                const int f = face_of_slot(g, BX, a, u);
                int side, i, jj;
                face_cell(g, BX, f, &side, &i, &jj);
                s += cf[f] * fs[jj * BX + i];
            }
        Tsub[(size_t)a * ld + ld - 1] = s;
    }
}

// ---------------------------------------------------------------- launchers
template <int BX>
static hipError_t setup_bx(rmrcm_ctx* c) {
    const Level& L = c->levels[c->D];
    const int R = L.nslot, BY = c->geo.by, NF = 2 * (BX + BY);
    const size_t lds = sizeof(double) * (size_t)(BX * (BX + 1) + 2 * BX * R + BY * BX + NF) +
                       sizeof(int) * (size_t)(2 * NF);
    hipError_t e = hipFuncSetAttribute((const void*)k_local_setup<BX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL(k_local_setup<BX>, dim3(nsub), dim3(64), lds, c->stream, c->geo, c->K,
                       c->bct, c->beta, L.slotseg, R, c->Pstore, c->Psi, L.T, L.ld, c->flags);
    return hipGetLastError();
}

template <int BX>
static hipError_t part_bx(rmrcm_ctx* c) {
    const Level& L = c->levels[c->D];
    const int BY = c->geo.by, NF = 2 * (BX + BY);
    const size_t lds = sizeof(double) * (size_t)(BX * BY + BX + NF) + sizeof(int) * (size_t)(2 * NF);
    hipError_t e = hipFuncSetAttribute((const void*)k_local_particular<BX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL(k_local_particular<BX>, dim3(nsub), dim3(64), lds, c->stream, c->geo, c->K,
                       c->bct, c->beta, L.slotseg, L.nslot, c->q, c->bcv, c->Pstore, c->pbar,
                       L.T, L.ld);
    return hipGetLastError();
}

hipError_t launch_beta(rmrcm_ctx* c) {
    if (c->geo.nseg == 0) return hipSuccess;
    const int nb = (c->geo.nseg + 255) / 256;
    hipLaunchKernelGGL(k_beta, dim3(nb), dim3(256), 0, c->stream, c->geo, c->K, c->beta, c->seglen);
    return hipGetLastError();
}

hipError_t launch_check_perm(rmrcm_ctx* c) {
    const size_t n = (size_t)c->geo.nx * c->geo.ny;
    hipLaunchKernelGGL(k_check_perm, dim3(1024), dim3(256), 0, c->stream, c->K, n, c->flags);
    return hipGetLastError();
}

hipError_t launch_local_setup(rmrcm_ctx* c) {
    switch (c->geo.bx) {
        case 4: return setup_bx<4>(c);
        case 8: return setup_bx<8>(c);
        case 16: return setup_bx<16>(c);
        case 32: return setup_bx<32>(c);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_local_particular(rmrcm_ctx* c) {
    switch (c->geo.bx) {
        case 4: return part_bx<4>(c);
        case 8: return part_bx<8>(c);
        case 16: return part_bx<16>(c);
        case 32: return part_bx<32>(c);
    }
    return hipErrorInvalidValue;
}

}  // namespace rmrcm
