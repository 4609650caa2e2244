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

#include <type_traits>
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
    if (g.neumann) {
        if (g.pin && g.pin[J * g.mx + I] && side == 0 && j == 0) {
            // the gauge face: a face to a zero datum (the cell's equation
            // keeps its right-hand side)
            *slot = code >= 0 ? a : -1;
            *outer = code >= 0 ? -1 : outer_face(g, side, gi, gj);
            return area / rho;
        }
        if (code >= 0) {
            *slot = a;
            *outer = -1;
            return 0.0;
        }
    }
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
// adjacent permeabilities (Section 5.1).  With general interface spaces the
// segment is the piece's U-segment (its g.mu pieces along the line, the
// first at a multiple of g.mu); seglen is the piece's own length.
// In 3D the segment's faces are those of every layer (the mean runs over
// all of them), Hbar is its length along the line and seglen its area.
__device__ inline void beta_of(const Geo& g, const double* __restrict__ K, double* __restrict__ beta,
                               double* __restrict__ seglen, int e) {
    double hsum = 0.0, len, h;
    const int nh = g.mu * g.sg;             // faces of the U-segment along its line
    const size_t layer = (size_t)g.nx * g.ny;
    for (int kz = 0; kz < g.nz; ++kz) {
        const double* Kk = K + kz * layer;
        if (e < g.nv) {
            const int I = e / g.lines_v + 1, k = e % g.lines_v;
            const int ilo = I * g.bx - 1, k0 = k - k % g.mu;
            for (int t = 0; t < nh; ++t) {
                const int j = k0 * g.sg + t;
                const double a = cellK(Kk, g, ilo, j), b = cellK(Kk, g, ilo + 1, j);
                hsum += 2.0 * a * b / (a + b);
            }
        } else {
            const int r = e - g.nv;
            const int J = r / g.lines_h + 1, k = r % g.lines_h;
            const int jlo = J * g.by - 1, k0 = k - k % g.mu;
            for (int t = 0; t < nh; ++t) {
                const int i = k0 * g.sg + t;
                const double a = cellK(Kk, g, i, jlo), b = cellK(Kk, g, i, jlo + 1);
                hsum += 2.0 * a * b / (a + b);
            }
        }
    }
    h = e < g.nv ? g.hy : g.hx;
    len = nh * h;
    const double keff = hsum / (nh * g.nz);
    beta[e] = g.alpha * len / keff;
    seglen[e] = g.sg * h * (g.nz * g.hz);
}



// Blocks below nbc: flag a permeability that is not finite and positive
// (with copy non-null the values are also copied there); the others: the
// segment Robin parameters.  One launch, as both read only the
// permeability.
__global__ void k_check_beta(Geo g, const double* __restrict__ K, size_t n, int* __restrict__ flags,
                             double* __restrict__ copy, int nbc, double* __restrict__ beta,
                             double* __restrict__ seglen) {
    if ((int)blockIdx.x >= nbc) {
        const int e = (blockIdx.x - nbc) * blockDim.x + threadIdx.x;
        if (e < g.nseg) beta_of(g, K, beta, seglen, e);
        return;
    }
    // four independent loads in flight per thread (a strided sweep of the
    // grid), then their checks and copies
    bool bad = false;
    const size_t stride = (size_t)nbc * blockDim.x;
    for (size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t0 < n; t0 += 4 * stride) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const size_t t = t0 + u * stride;
            v[u] = t < n ? K[t] : 1.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const size_t t = t0 + u * stride;
            bad |= !(v[u] > 0.0) || !(v[u] <= 1.7976931348623157e308);
            if (copy && t < n) copy[t] = v[u];
        }
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

// Value of a register of lane l (l uniform, a compile-time constant at every
// call) as a wave-uniform scalar.
// Row coefficients of row j for a wave whose lane holds column c, from the
// permeability k of its own cell and ku of the cell above (ku unused on the
// top row).  The half-cell resistances are formed once per cell and shared
// with the neighbours: h/(2k) of the right neighbour by a lane shuffle, the
// coupling to the row below carried over from the previous row in tyd.  The
// operands and their order are those of the two-point harmonic mean above, so
// the coefficients are the same numbers.
template <int BX>
__device__ inline void row_coeffs(const Geo& g, const double* cf, int lane, int c, int j, double k,
                                  double ku, double tyd, double* dg, double* txr, double* txl,
                                  double* tyu) {
    const int BY = g.by;
    const double rx = g.hx / (2.0 * k);
    const double rxr = __shfl(rx, lane < 63 ? lane + 1 : 63, 64);
    const double tr = c < BX - 1 ? g.hy / (rx + rxr) : 0.0;
    const double tl = __shfl(tr, lane > 0 ? lane - 1 : 0, 64);
    const double tu = j < BY - 1 ? g.hx / (g.hy / (2.0 * k) + g.hy / (2.0 * ku)) : 0.0;
    const double tlc = c > 0 ? tl : cf[j];
    *dg = tlc + (c < BX - 1 ? tr : cf[BY + j]) + tyd + (j < BY - 1 ? tu : cf[2 * BY + BX + c]);
    *txr = tr;
    *txl = tl;
    *tyu = tu;
}

// The same for an elimination from the top row down: kd is the permeability
// of the cell below (unused on the bottom row), tyu the coupling to the row
// above carried from the previous step (the north boundary conductance on the
// top row), and *tyd returns the coupling to the row below, with the operands
// of the harmonic mean in the order of the upward form (lower cell first), so
// that both directions give the same numbers.
template <int BX>
__device__ inline void row_coeffs_down(const Geo& g, const double* cf, int lane, int c, int j,
                                       double k, double kd, double tyu, double* dg, double* txr,
                                       double* txl, double* tyd) {
    const int BY = g.by;
    const double rx = g.hx / (2.0 * k);
    const double rxr = __shfl(rx, lane < 63 ? lane + 1 : 63, 64);
    const double tr = c < BX - 1 ? g.hy / (rx + rxr) : 0.0;
    const double tl = __shfl(tr, lane > 0 ? lane - 1 : 0, 64);
    const double td = j > 0 ? g.hx / (g.hy / (2.0 * kd) + g.hy / (2.0 * k)) : 0.0;
    const double tlc = c > 0 ? tl : cf[j];
    *dg = tlc + (c < BX - 1 ? tr : cf[BY + j]) + (j > 0 ? td : cf[2 * BY + c]) + tyu;
    *txr = tr;
    *txl = tl;
    *tyd = td;
}

// Orders this wave's LDS writes before its later LDS reads by other lanes
// (the workgroup is this one wave).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline double readlane_s(double v, int l) {
    const unsigned long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffull), l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ inline float readlane_s(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double inv_sqrt(double d) { return 1.0 / sqrt(d); }
__device__ inline float inv_sqrt(float d) { return 1.0f / sqrtf(d); }

// 1/sqrt(d) for d > 0: the hardware estimate (relative error below 2^-24 on
// this part) refined by Newton-Raphson steps on f(y) = y^-2 - d,
// y <- y + (y / 2)(1 - d y^2), each squaring the error: two in FP64 (one
// leaves a one-sided error near 2^-48 in every pivot, which problems with
// one-face segments amplify a hundredfold), one in FP32.
__device__ inline double rsqrt_nr(double d) {
    double y = __builtin_amdgcn_rsq(d);
    y = fma(0.5 * y, fma(-d * y, y, 1.0), y);
    y = fma(0.5 * y, fma(-d * y, y, 1.0), y);
    return y;
}
__device__ inline float rsqrt_nr(float d) {
    const float y = __builtin_amdgcn_rsqf(d);
    return fmaf(0.5f * y, fmaf(-d * y, y, 1.0f), y);
}

constexpr int kWPre = 16;   // basis columns prefetched per lane in the backward sweep

// LDS carve-up helper: returns p and advances it, 16-byte aligned.
template <typename T>
__device__ inline T* carve(char*& p, size_t count) {
    T* r = (T*)p;
    p += (count * sizeof(T) + 15) & ~(size_t)15;
    return r;
}
__host__ inline size_t carve_bytes(size_t count, size_t elem) { return (count * elem + 15) & ~(size_t)15; }

// ---------------------------------------------------------------- K1
// Factorisation and basis solves: one wavefront per subdomain, in the
// compute type S (double: the FP64 path; float: the factorisation of the
// mixed-precision path, refined afterwards in FP64).
//
// Lane l < 2 BX owns column l of the augmented block [S_j | I] of the
// current block row in registers.  Cholesky step k: the pivot comes from
// lane k, row k is scaled by 1/sqrt(pivot), and by symmetry of the trailing
// block the multiplier of row i > k is the scaled row-k entry held by lane
// i, read as a wave-uniform scalar.  After BX steps lanes BX..2BX-1 hold
// L_j^{-1}; P_j = L_j^{-T} L_j^{-1} is formed column by column (lane c
// computes column c, which is also row c), stored, and used for the sweep
// w_j = P_j z_j and the trailing update S_{j+1} = A_{j+1} - D_j P_j D_j.
// Global loads are issued one row ahead of their use.  With a mask, only
// subdomains whose mask entry equals `want` are processed.
// A local factorisation that met a non-positive pivot: an error of the FP64
// factorisation; in FP32 (fbm non-null, the mixed modes) the subdomain is
// marked for the FP64 redo instead (large Robin parameters make the local
// systems too ill conditioned for FP32).
__device__ inline void report_singular(int* flags, int* fbm, int sub) {
    if (fbm) {
        fbm[sub] = 1;
        atomicAdd(&flags[FLAG_FALLBACK], 1);
    } else {
        atomicOr(&flags[FLAG_LOCAL_SINGULAR], 1);
    }
}

template <int BX, typename S>
__global__ __launch_bounds__(64) void k_local_setup(Geo g, const double* __restrict__ K,
                                                    const int8_t* __restrict__ bct,
                                                    const double* __restrict__ beta,
                                                    const int* __restrict__ slotseg, int R,
                                                    S* __restrict__ Pstore,
                                                    double* __restrict__ Psi,
                                                    double* __restrict__ T, int ld,
                                                    int* __restrict__ flags,
                                                    const int* __restrict__ mask, int want,
                                                    int do_traces, int basis, int* __restrict__ fbm) {
    const int sub = blockIdx.x;
    if (mask && mask[sub] != want) return;
    extern __shared__ __align__(16) char smem[];
    constexpr int LT = BX + 1;             // padded row of L^{-T}
    const int ncol = basis ? R : 0;        // basis = 0: factor store only
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    char* cur = smem;
    S* LTs = carve<S>(cur, BX * LT);        // row c = column c of L^{-1}
    S* Z = carve<S>(cur, BX * R);           // z_j, later D_j x_{j+1}
    S* Wl = carve<S>(cur, BX * R);          // w_j, later x_j
    S* tys = carve<S>(cur, BY * BX);        // couplings D_j
    double* cf = carve<double>(cur, NF);    // face conductances
    int* rs = carve<int>(cur, NF);          // Robin slots
    int* of = carve<int>(cur, NF);          // outer faces

    const int lane = threadIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    S* Ps = Pstore + (size_t)sub * BY * BX * BX;
    double* Psub = Psi + (size_t)sub * R * n;

    const bool scol = lane < BX;                    // column of S
    const bool icol = lane >= BX && lane < 2 * BX;  // column of the identity block
    const int c = scol ? lane : (icol ? lane - BX : 0);

    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    double kv[5], kn[5];
    load_kstencil<BX>(g, K, I, J, c, 0, kv);
    for (int t = lane; t < BX * R; t += 64) Z[t] = S(0);
    __syncthreads();

    S a[BX];
    S p[BX];
    int sing = 0;
    double dg, txr, tyu;
    stencil_coeffs<BX>(g, kv, cf, c, 0, &dg, &txr, &tyu);
    double txl = __shfl(txr, lane > 0 ? lane - 1 : 0, 64);
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        double v = 0.0;
        if (scol) v = (i == c) ? dg : (i == c + 1) ? -txr : (i + 1 == c) ? -txl : 0.0;
        else if (icol) v = (i == c) ? 1.0 : 0.0;
        a[i] = S(v);
    }
    if (lane == 0 && rs[0] >= 0) Z[rs[0]] += S(cf[0]);
    if (lane == 1 && rs[BY] >= 0) Z[(BX - 1) * R + rs[BY]] += S(cf[BY]);
    __syncthreads();
    if (lane < BX && rs[2 * BY + lane] >= 0) Z[lane * R + rs[2 * BY + lane]] += S(cf[2 * BY + lane]);
    if (BY == 1 && lane < BX && rs[2 * BY + BX + lane] >= 0)
        Z[lane * R + rs[2 * BY + BX + lane]] += S(cf[2 * BY + BX + lane]);
    __syncthreads();

    for (int j = 0; j < BY; ++j) {
        if (j + 1 < BY) load_kstencil<BX>(g, K, I, J, c, j + 1, kn);
        // ---- Cholesky of S_j fused with the inversion of its factor
#pragma unroll
        for (int k = 0; k < BX; ++k) {
            S d = readlane_s(a[k], k);
            if (!(d > S(0))) {
                sing = 1;
                d = S(1);
            }
            const S r = inv_sqrt(d);
            a[k] *= r;
#pragma unroll
            for (int i = k + 1; i < BX; ++i) a[i] = fma(-readlane_s(a[k], i), a[k], a[i]);
        }
        // ---- P_j = L^{-T} L^{-1}
        if (icol) {
#pragma unroll
            for (int i = 0; i < BX; ++i) LTs[c * LT + i] = a[i];
        }
        __syncthreads();
        if (scol) {
#pragma unroll
            for (int r = 0; r < BX; ++r) p[r] = S(0);
#pragma unroll
            for (int i = 0; i < BX; ++i) {
                const S lci = LTs[c * LT + i];
#pragma unroll
                for (int r = 0; r <= i; ++r) p[r] = fma(LTs[r * LT + i], lci, p[r]);
            }
#pragma unroll
            for (int r = 0; r < BX; ++r) Ps[(size_t)j * BX * BX + r * BX + c] = p[r];
            // w_j = P_j z_j: lane c computes row c (P symmetric)
            for (int q = 0; q < ncol; ++q) {
                S s = S(0);
#pragma unroll
                for (int k = 0; k < BX; ++k) s = fma(p[k], Z[k * R + q], s);
                Wl[c * R + q] = s;
                Psub[(size_t)q * n + j * BX + c] = (double)s;
            }
            tys[j * BX + c] = S(tyu);    // D_j
        }
        __syncthreads();
        if (j + 1 < BY) {
            const S dc = S(tyu);
            stencil_coeffs<BX>(g, kn, cf, c, j + 1, &dg, &txr, &tyu);
            txl = __shfl(txr, lane > 0 ? lane - 1 : 0, 64);
#pragma unroll
            for (int i = 0; i < BX; ++i) {
                S v = S(0);
                if (scol) {
                    v = -p[i] * (tys[j * BX + i] * dc);
                    if (i == c) v += S(dg);
                    else if (i == c + 1) v -= S(txr);
                    else if (i + 1 == c) v -= S(txl);
                } else if (icol) {
                    v = (i == c) ? S(1) : S(0);
                }
                a[i] = v;
            }
            // z_{j+1} = F_{j+1} + D_j w_j
            for (int t = lane; t < BX * ncol; t += 64) Z[t] = tys[j * BX + t / R] * Wl[t];
            __syncthreads();
            const int jn = j + 1;
            if (lane == 0 && rs[jn] >= 0) Z[rs[jn]] += S(cf[jn]);
            if (lane == 1 && rs[BY + jn] >= 0) Z[(BX - 1) * R + rs[BY + jn]] += S(cf[BY + jn]);
            __syncthreads();
            if (jn == BY - 1 && lane < BX && rs[2 * BY + BX + lane] >= 0)
                Z[lane * R + rs[2 * BY + BX + lane]] += S(cf[2 * BY + BX + lane]);
            __syncthreads();
        }
    }
    // ---- backward sweep: x_{BY-1} = w_{BY-1}; x_j = w_j + P_j D_j x_{j+1}
    // Wl holds x_{j+1}; lane c loads row c of P_j (= column c) and its own
    // row of w_j one step ahead.
    if (!basis) {
        if (lane == 0 && sing) report_singular(flags, fbm, sub);
        return;
    }
    S pn[BX];
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
                    S s = S(wc[q]);
#pragma unroll
                    for (int k = 0; k < BX; ++k) s = fma(p[k], Z[k * R + q], s);
                    Wl[c * R + q] = s;
                    Psub[(size_t)q * n + j * BX + c] = (double)s;
                }
            }
            for (int q = kWPre; q < R; ++q) {
                S s = S(Psub[(size_t)q * n + j * BX + c]);
#pragma unroll
                for (int k = 0; k < BX; ++k) s = fma(p[k], Z[k * R + q], s);
                Wl[c * R + q] = s;
                Psub[(size_t)q * n + j * BX + c] = (double)s;
            }
        }
        __syncthreads();
    }
    if (do_traces) {
        // traces T[a][b] = sum_{f in slot a} c_f (x_b(cell f) - delta_ab)
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
    }
    if (lane == 0 && sing) report_singular(flags, fbm, sub);
}

// ---------------------------------------------------------------- K1 (MFMA)
// The same factorisation and basis solves for subdomains 16 or 32 cells wide,
// with the dense products on the matrix cores (v_mfma 16x16x4, FP64 or FP32
// by the compute type S): per block row j the inverse P_j = L^{-T} L^{-1}
// (L^{-1} from the register Cholesky above, staged in LDS) and the
// multi-column sweeps w_j = P_j z_j (forward) and x_j = w_j + P_j D_j x_{j+1}
// (backward, P_j re-read from the factor store one row ahead).  Operands are
// read from LDS in the MFMA lane layout: A[i][k] from lane i + 16 k,
// B[k][j] from lane j + 16 k; rows of LDS matrices are padded by 4 to spread
// the banks.

template <typename S>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row of the 16 x 16 result held by lane l in register v (column l % 16)
    static __device__ inline int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// Pivots per block of the local Cholesky (BX: one block, multipliers by lane
// reads only; a smaller block adds rank-NB updates through an LDS buffer of
// NB x BX entries).  Chosen so that the kernel fits the 256 registers of two
// waves per SIMD without spilling.
template <int BX, typename S>
__host__ __device__ constexpr int chol_block() { return (BX > 16 && sizeof(S) == 8) ? 16 : BX; }
template <int BX, typename S>
__host__ __device__ constexpr int chol_wb_entries() {
    return chol_block<BX, S>() < BX ? chol_block<BX, S>() * BX : 0;
}

// Right-hand side of the particular problem at cell (i, j): the source plus
// the outer boundary data (Dirichlet |f|/rho g_D, Neumann -g_N).
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

// Adds the boundary right-hand side of block row j (the Robin faces of its
// W and E ends, and of the S / N sides on the first / last row) to the basis
// columns of a right-hand side block Zb (row c = cell c, ld RP); one wave.
template <int BX, typename S>
__device__ inline void add_row_forcing(const Geo& g, const double* cf, const int* rs, S* Zb, int RP,
                                       int lane, int j) {
    const int BY = g.by;
    if (lane == 0 && rs[j] >= 0) Zb[rs[j]] += S(cf[j]);
    if (lane == 1 && rs[BY + j] >= 0) Zb[(BX - 1) * RP + rs[BY + j]] += S(cf[BY + j]);
    wave_lds_sync();
    if (j == 0 && lane < BX && rs[2 * BY + lane] >= 0) Zb[lane * RP + rs[2 * BY + lane]] += S(cf[2 * BY + lane]);
    wave_lds_sync();
    if (j == BY - 1 && lane < BX && rs[2 * BY + BX + lane] >= 0)
        Zb[lane * RP + rs[2 * BY + BX + lane]] += S(cf[2 * BY + BX + lane]);
    wave_lds_sync();
}

// Cholesky of the block held in a[] (lane c < BX: column c of S_j; lane
// BX + c: column c of the identity) fused with the inversion of its factor:
// afterwards lanes BX..2BX-1 hold L^{-1} (lane BX + c: column c), and sing
// is set on a pivot that is not positive.  NB pivots at a time: inside a
// block the multipliers are read from their lanes; the rows below take the
// block's updates with the multipliers broadcast from LDS (Wb, NB x BX
// entries).  Every entry sees the same operations in the same order as
// pivot by pivot.
template <int BX, typename S>
__device__ __forceinline__ void chol_invert(S (&a)[BX], S* Wb, bool scol, int c, int& sing) {
    constexpr int NB = chol_block<BX, S>();
#pragma unroll
    for (int kb = 0; kb < BX; kb += NB) {
#pragma unroll
        for (int k = kb; k < kb + NB; ++k) {
            // a pivot that is not positive is flagged (the factor is then
            // not used); the test stays off the pivot chain
            const S d = readlane_s(a[k], k);
            sing |= !(d > S(0));
            a[k] *= rsqrt_nr(d);
#pragma unroll
            for (int i = k + 1; i < kb + NB; ++i) a[i] = fma(-readlane_s(a[k], i), a[k], a[i]);
        }
        if (kb + NB < BX) {
            if (scol) {
#pragma unroll
                for (int k = kb; k < kb + NB; ++k) Wb[(k - kb) * BX + c] = a[k];
            }
            wave_lds_sync();
            // four rows at a time: bounds the multipliers held in registers
#pragma unroll
            for (int i0 = kb + NB; i0 < BX; i0 += 4) {
#pragma unroll
                for (int i = i0; i < i0 + 4; ++i)
#pragma unroll
                    for (int k = kb; k < kb + NB; ++k) a[i] = fma(-Wb[(k - kb) * BX + i], a[k], a[i]);
                __builtin_amdgcn_sched_barrier(0);
            }
            wave_lds_sync();
        }
    }
}

// The block [S_j | I] of a row: a[i] = p[i] ms + e_i, with p the Schur term
// (column c on lane c), ms = 1 on the lanes of S (0 elsewhere), and e_i the
// tridiagonal entries of A_jj there and the identity on the lanes that carry
// it (p[i] 1 is exact, so the sums are p[i] + entry).  Selects rather than
// branches; cc is opaque to the optimiser so that the lane-dependent compares
// are formed here, not kept live across the caller's row loop.
template <int BX, typename S>
__device__ __forceinline__ void build_block(S (&a)[BX], const S (&p)[BX], double dg, double txr,
                                            double txl, bool scol, bool icol, int c) {
    int cc = c;
    asm volatile("" : "+v"(cc));
    const S ms = scol ? S(1) : S(0);
    const S od = scol ? S(dg) : (icol ? S(1) : S(0));
    const S orr = scol ? -S(txr) : S(0), ol = scol ? -S(txl) : S(0);
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        S e = (i == cc) ? od : S(0);
        e = (i == cc + 1) ? orr : e;
        e = (i + 1 == cc) ? ol : e;
        a[i] = fma(p[i], ms, e);
    }
}

// The same with the Schur term read from LDS (row-major, padded rows of
// BX + 4; t1 null on the first row of a chain) plus a second term t2 when
// not null: a[i] = (t1[i][c] + t2[i][c]) ms + e_i.
template <int BX, typename S>
__device__ __forceinline__ void build_block_lds(S (&a)[BX], const S* t1, const S* t2, double dg,
                                                double txr, double txl, bool scol, bool icol,
                                                int c) {
    constexpr int LT = BX + 4;
    int cc = c;
    asm volatile("" : "+v"(cc));
    const S ms = scol ? S(1) : S(0);
    const S od = scol ? S(dg) : (icol ? S(1) : S(0));
    const S orr = scol ? -S(txr) : S(0), ol = scol ? -S(txl) : S(0);
#pragma unroll
    for (int i = 0; i < BX; ++i) {
        S e = (i == cc) ? od : S(0);
        e = (i == cc + 1) ? orr : e;
        e = (i + 1 == cc) ? ol : e;
        S pv = t1 ? t1[i * LT + c] : S(0);
        if (t2) pv += t2[i * LT + c];
        a[i] = fma(pv, ms, e);
    }
}

// P[r][c] = sum_{i >= max(r,c)} L^{-1}[i][r] L^{-1}[i][c] on the matrix
// cores, from LTs (row c = column c of L^{-1}, rows padded to BX + 4); tile
// (tr, tc) in the accumulator layout.
template <int BX, typename S>
__device__ __forceinline__ void form_inverse(const S* LTs, int li, int lk,
                                             typename Mfma<S>::v4 (&pacc)[BX / 16][BX / 16]) {
    constexpr int LT = BX + 4, NTL = BX / 16;
#pragma unroll
    for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
        for (int tc = 0; tc < NTL; ++tc) {
            typename Mfma<S>::v4 acc = {S(0), S(0), S(0), S(0)};
            const int k0 = 16 * (tr > tc ? tr : tc);
#pragma unroll
            for (int kk = k0; kk < BX; kk += 4) {
                const S av = LTs[(16 * tr + li) * LT + kk + lk];
                const S bv = LTs[(16 * tc + li) * LT + kk + lk];
                acc = Mfma<S>::op(av, bv, acc);
            }
            pacc[tr][tc] = acc;
        }
}

template <int BX, typename S>
__global__ __launch_bounds__(128, 2) void k_local_setup_mfma(Geo g, const double* __restrict__ K,
                                                          const int8_t* __restrict__ bct,
                                                          const double* __restrict__ beta,
                                                          const int* __restrict__ slotseg, int R,
                                                          S* __restrict__ Pstore,
                                                          double* __restrict__ Psi,
                                                          double* __restrict__ T, int ld,
                                                          int* __restrict__ flags,
                                                          const int* __restrict__ mask, int want,
                                                          int do_traces, int basis, int* __restrict__ fbm) {
    static_assert(BX == 16 || BX == 32, "MFMA tiles of 16");
    typedef Mfma<S> M;
    typedef typename M::v4 v4;
    const int sub = blockIdx.x;
    if (mask && mask[sub] != want) return;
    extern __shared__ __align__(16) char smem[];
    constexpr int LT = BX + 4;              // padded row length
    constexpr int NTL = BX / 16;            // tiles per dimension
    constexpr int NB = chol_block<BX, S>(); // pivots per Cholesky block
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    const int RP = (R + 15) & ~15;          // columns padded to whole tiles
    const int nct = basis ? RP / 16 : 0;    // column tiles of the sweeps
    char* cur = smem;
    S* LTs = carve<S>(cur, BX * LT);        // wave A: row c = column c of L^{-1}, then -D P D
    S* Wb = carve<S>(cur, chol_wb_entries<BX, S>());   // wave A: multipliers of one block
    S* Z = carve<S>(cur, BX * RP);          // z_j, later D_j x_{j+1}
    S* Z2 = carve<S>(cur, BX * RP);         // the next row's z (double buffer)
    S* tys = carve<S>(cur, BY * BX);        // couplings D_j
    double* cf = carve<double>(cur, NF);
    int* rs = carve<int>(cur, NF);
    int* of = carve<int>(cur, NF);

    // wave A (w = 0) runs the factorisation chain; wave B (w = 1) the forward
    // sweep of each row one barrier behind it; both share the backward sweep
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    S* Ps = Pstore + (size_t)sub * BY * BX * BX;
    double* Psub = Psi + (size_t)sub * R * n;

    const bool scol = lane < BX;
    const bool icol = lane >= BX && lane < 2 * BX;
    const int c = scol ? lane : (icol ? lane - BX : 0);

    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    for (int t = tid; t < BX * RP; t += 128) Z[t] = S(0);
    __syncthreads();

    // permeability of column c, row by row (wave A): kq (row being set up),
    // kq1 (the row above), kq2 (two rows above, in flight during a row's work)
    const double* Kc = K + (size_t)J * BY * g.nx + (size_t)I * BX + c;
    double kq = 1.0, kq1 = 1.0, kq2 = 1.0;
    S a[BX];
    S p[BX];
    int sing = 0;
    double dg = 0.0, txr = 0.0, txl = 0.0, tyu = 0.0;
    if (w == 0) {
        kq = Kc[0];
        kq1 = BY > 1 ? Kc[g.nx] : 1.0;
        row_coeffs<BX>(g, cf, lane, c, 0, kq, kq1, cf[2 * BY + c], &dg, &txr, &txl, &tyu);
#pragma unroll
        for (int i = 0; i < BX; ++i) {
            double v = 0.0;
            if (scol) v = (i == c) ? dg : (i == c + 1) ? -txr : (i + 1 == c) ? -txl : 0.0;
            else if (icol) v = (i == c) ? 1.0 : 0.0;
            a[i] = S(v);
        }
    } else {
        if (lane == 0 && rs[0] >= 0) Z[rs[0]] += S(cf[0]);
        if (lane == 1 && rs[BY] >= 0) Z[(BX - 1) * RP + rs[BY]] += S(cf[BY]);
        wave_lds_sync();
        if (lane < BX && rs[2 * BY + lane] >= 0) Z[lane * RP + rs[2 * BY + lane]] += S(cf[2 * BY + lane]);
        if (BY == 1 && lane < BX && rs[2 * BY + BX + lane] >= 0)
            Z[lane * RP + rs[2 * BY + BX + lane]] += S(cf[2 * BY + BX + lane]);
    }

    for (int j = 0; j < BY; ++j) {
        if (w == 0) {
            if (j + 2 < BY) kq2 = Kc[(size_t)(j + 2) * g.nx];
            chol_invert<BX, S>(a, Wb, scol, c, sing);
            if (icol) {
#pragma unroll
                for (int i = 0; i < BX; ++i) LTs[c * LT + i] = a[i];
            }
            if (scol) tys[j * BX + c] = S(tyu);    // D_j
            wave_lds_sync();
            // ---- P_j[r][c] = sum_{i >= max(r,c)} L^{-1}[i][r] L^{-1}[i][c] on the
            // matrix cores, to the factor store; once every tile is formed,
            // L^{-1} is dead and its buffer takes the Schur term
            // -(D_j P_j D_j)[r][c] of the next row, row-major
            v4 pacc[NTL][NTL];
            form_inverse<BX, S>(LTs, li, lk, pacc);
            const bool trail = j + 1 < BY;
#pragma unroll
            for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
                for (int tc = 0; tc < NTL; ++tc)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * tr + M::row(lane, v), cq = 16 * tc + li;
                        const S pv = pacc[tr][tc][v];
                        Ps[(size_t)j * BX * BX + r * BX + cq] = pv;
                        if (trail) LTs[r * LT + cq] = -(pv * (tys[j * BX + r] * tys[j * BX + cq]));
                    }
        }
        __syncthreads();                   // P_j in the factor store, D_j in tys
        if (w == 1) {
            // ---- forward sweep w_j = P_j z_j (P_j as the A operand from the
            // factor store); also D_j w_j, the next row's right-hand side (for
            // the last row D_{BY-2} w_{BY-1}, the backward sweep's first)
            const int jz = (j + 1 < BY) ? j : j - 1;
            if (nct > 0) {
                S av[NTL][BX / 4];
#pragma unroll
                for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
                    for (int kq4 = 0; kq4 < BX / 4; ++kq4)
                        av[tr][kq4] = Ps[(size_t)j * BX * BX + (16 * tr + li) * BX + 4 * kq4 + lk];
                for (int ct = 0; ct < nct; ++ct) {
#pragma unroll
                    for (int tr = 0; tr < NTL; ++tr) {
                        v4 acc = {S(0), S(0), S(0), S(0)};
#pragma unroll
                        for (int kq4 = 0; kq4 < BX / 4; ++kq4)
                            acc = M::op(av[tr][kq4], Z[(4 * kq4 + lk) * RP + 16 * ct + li], acc);
                        const int q = 16 * ct + li;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int r = 16 * tr + M::row(lane, v);
                            if (jz >= 0) Z2[r * RP + q] = tys[jz * BX + r] * acc[v];
                            if (q < R) Psub[(size_t)q * n + j * BX + r] = (double)acc[v];
                        }
                    }
                }
            }
            if (j + 1 < BY) {
                // z_{j+1} = F_{j+1} + D_j w_j
                wave_lds_sync();
                const int jn = j + 1;
                if (lane == 0 && rs[jn] >= 0) Z2[rs[jn]] += S(cf[jn]);
                if (lane == 1 && rs[BY + jn] >= 0) Z2[(BX - 1) * RP + rs[BY + jn]] += S(cf[BY + jn]);
                wave_lds_sync();
                if (jn == BY - 1 && lane < BX && rs[2 * BY + BX + lane] >= 0)
                    Z2[lane * RP + rs[2 * BY + BX + lane]] += S(cf[2 * BY + BX + lane]);
                wave_lds_sync();
            }
        } else if (j + 1 < BY) {
            // ---- trailing update S_{j+1} = A_{j+1} - D_j P_j D_j (lane c: column c)
#pragma unroll
            for (int r = 0; r < BX; ++r) p[r] = LTs[r * LT + c];     // -(D_j P_j D_j), column c
            kq = kq1;
            kq1 = kq2;
            row_coeffs<BX>(g, cf, lane, c, j + 1, kq, kq1, tyu, &dg, &txr, &txl, &tyu);
            build_block<BX, S>(a, p, dg, txr, txl, scol, icol, c);
        }
        if (j + 1 < BY) {
            S* t = Z;
            Z = Z2;
            Z2 = t;
        }
    }
    __syncthreads();                       // the last forward sweep
    if (!basis) {
        if (tid == 0 && sing) report_singular(flags, fbm, sub);
        return;
    }
    // ---- backward sweep: x_{BY-1} = w_{BY-1}; x_j = w_j + P_j (D_j x_{j+1}).
    // Wave w forms row tile w (BX = 32) or wave 0 the only one (BX = 16); the
    // tile's rows of P_{j-1} and of w_{j-1} (first WCT column tiles) are
    // loaded one row ahead.
    constexpr int WCT = 2;
    const int tr = w;
    const bool act = tr < NTL;
    S pn[BX / 4];
    v4 wn[WCT];
    auto load_row = [&](int jr) {
#pragma unroll
        for (int kq4 = 0; kq4 < BX / 4; ++kq4)
            pn[kq4] = Ps[(size_t)jr * BX * BX + (16 * tr + li) * BX + 4 * kq4 + lk];
#pragma unroll
        for (int ct = 0; ct < WCT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int q = 16 * ct + li, r = 16 * tr + M::row(lane, v);
                wn[ct][v] = (ct < nct && q < R) ? S(Psub[(size_t)q * n + jr * BX + r]) : S(0);
            }
    };
    if (act && BY > 1) load_row(BY - 2);
    for (int j = BY - 2; j >= 0; --j) {
        {                       // Z = D_j x_{j+1}, written by the previous sweep
            S* t = Z;
            Z = Z2;
            Z2 = t;
        }
        S pc[BX / 4];
        v4 wc[WCT];
#pragma unroll
        for (int kq4 = 0; kq4 < BX / 4; ++kq4) pc[kq4] = pn[kq4];
#pragma unroll
        for (int ct = 0; ct < WCT; ++ct) wc[ct] = wn[ct];
        __syncthreads();
        if (act) {
            if (j > 0) load_row(j - 1);
            auto tile = [&](int ct, v4 acc) {
                const int q = 16 * ct + li;
#pragma unroll
                for (int kq4 = 0; kq4 < BX / 4; ++kq4)
                    acc = M::op(pc[kq4], Z[(4 * kq4 + lk) * RP + q], acc);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * tr + M::row(lane, v);
                    if (j > 0) Z2[r * RP + q] = tys[(j - 1) * BX + r] * acc[v];
                    if (q < R) Psub[(size_t)q * n + j * BX + r] = (double)acc[v];
                }
            };
#pragma unroll
            for (int ct = 0; ct < WCT; ++ct)
                if (ct < nct) tile(ct, wc[ct]);
            for (int ct = WCT; ct < nct; ++ct) {
                const int q = 16 * ct + li;
                v4 acc;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * tr + M::row(lane, v);
                    acc[v] = q < R ? S(Psub[(size_t)q * n + j * BX + r]) : S(0);
                }
                tile(ct, acc);
            }
        }
    }
    __syncthreads();
    if (do_traces) {
        // traces T[a][b] = sum_{f in slot a} c_f (x_b(cell f) - delta_ab)
        double* Tsub = T + (size_t)sub * R * ld;
        for (int t = tid; t < R * R; t += 128) {
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
    }
    if (tid == 0 && sing) report_singular(flags, fbm, sub);
}

// The particular column's product w = P z on the vector units, with P in the
// accumulator layout of form_inverse (P symmetric: lane l, register v of tile
// (k, r) holds P[16 r + l % 16][16 k + l / 16 + 4 v]) and z in LDS: each
// lane sums its 2 BX / 4 terms of row 16 r + l % 16, and the sums of the
// four lanes l % 16 + 16 i are added across lanes (every one of them ends
// with the same value).
template <int BX>
__device__ __forceinline__ void part_product(const typename Mfma<double>::v4 (&pacc)[BX / 16][BX / 16],
                                             const double* z, int lk, double (&out)[BX / 16]) {
    constexpr int NTL = BX / 16;
#pragma unroll
    for (int tr = 0; tr < NTL; ++tr) {
        double s = 0.0;
#pragma unroll
        for (int kt = 0; kt < NTL; ++kt)
#pragma unroll
            for (int v = 0; v < 4; ++v) s = fma(pacc[kt][tr][v], z[16 * kt + lk + 4 * v], s);
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        out[tr] = s;
    }
}

// ---------------------------------------------------------------- K1 (twisted)
// FP64 factorisation and basis solves for subdomains 16 or 32 cells wide,
// eliminated from both ends at once (a twisted block factorisation).  With
// m = by / 2, wave 0 eliminates rows 0 .. m-1 upwards as above,
//     S_0 = A_0,          S_{j+1} = A_{j+1} - D_j P_j D_j,
// and wave 1 rows by-1 .. m+1 downwards,
//     S_{by-1} = A_{by-1}, S_{j-1} = A_{j-1} - D_{j-1} P_j D_{j-1},
// each with its forward sweep (w_j = P_j z_j, the right-hand side carried
// towards row m).  Row m takes both Schur terms,
//     S_m = A_m - D_{m-1} P_{m-1} D_{m-1} - D_m P_{m+1} D_m,
//     x_m = P_m (f_m + D_{m-1} w_{m-1} + D_m w_{m+1}),
// and the backward sweeps run outwards from it, one per wave:
//     x_j = w_j + P_j D_j x_{j+1}      (j < m),
//     x_j = w_j + P_j D_{j-1} x_{j-1}  (j > m).
// The chain of dependent block rows is m + 1 long instead of by.  The factor
// store holds P_j of this elimination for every row, its 16 x 16 tiles on
// and below the diagonal only (P_j is symmetric; readers take a tile above
// the diagonal as the transpose of its mirror: a quarter less traffic at
// 32 cells), and the particular solve sweeps it the same way.  Each wave has its own L^{-1} / Schur-term
// buffer (also the multiplier buffer of the blocked Cholesky, which is used
// only while the buffer is free) and right-hand side block in LDS.  The
// forward sweep takes P_j straight from the accumulators: P_j is symmetric,
// so tile (k, r) in the accumulator layout (lane l, register v: row
// 16 k + l / 16 + 4 v, column 16 r + l % 16) is the A operand of row tile r
// and k-slices 4 k .. 4 k + 3.
//
// With PART (and basis) the particular problem (source qsrc, outer boundary
// data bcv) is solved beside the basis: a single column, so its products are
// matrix-vector products on the vector units (each lane sums its share of
// a row of P_j from the registers that hold P_j, and the four partial sums
// of a row are added across lanes), with its right-hand side as a vector in
// LDS.  Its solution goes to pbar and, with do_traces, its traces to column
// ld - 1 of T.
template <int BX, int NCT, bool PART>
__global__ __launch_bounds__(128, 2) void k_local_setup_twist(
    Geo g, const double* __restrict__ K, const int8_t* __restrict__ bct,
    const double* __restrict__ beta, const int* __restrict__ slotseg, int R,
    double* __restrict__ Pstore, double* __restrict__ Psi, double* __restrict__ T, int ld,
    int* __restrict__ flags, const int* __restrict__ mask, int want, int do_traces, int basis,
    const double* __restrict__ qsrc, const double* __restrict__ bcv, double* __restrict__ pbar) {
    static_assert(BX == 16 || BX == 32, "MFMA tiles of 16");
    typedef double S;
    typedef Mfma<S> M;
    typedef typename M::v4 v4;
    constexpr int LT = BX + 4;              // padded row length
    constexpr int NTL = BX / 16;            // tiles per dimension
    static_assert(chol_wb_entries<BX, S>() <= BX * LT, "multipliers fit the L^{-1} buffer");
    const int sub = blockIdx.x;
    if (mask && mask[sub] != want) return;
    extern __shared__ __align__(16) char smem[];
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    // NCT > 0: the column tiles of the sweeps as a constant (basis, and
    // (R + 15) / 16 == NCT), so that the memory waits after each row's
    // stores are counted rather than drained
    const int NC = basis ? R : 0;           // basis columns of the sweeps
    const int RP = (NC + 15) & ~15;         // padded to whole tiles
    const int nct = NCT > 0 ? NCT : RP / 16;
    constexpr int part = PART ? 1 : 0;
    const int m = BY / 2;                   // the row where the eliminations meet
    char* cur = smem;
    S* LTa = carve<S>(cur, 2 * BX * LT);    // per wave: L^{-1} rows, multipliers, Schur term
    S* Za = carve<S>(cur, 2 * BX * RP);     // per wave: right-hand side block
    S* tys = carve<S>(cur, BY * BX);        // couplings D_j
    S* zpa = carve<S>(cur, 2 * BX);         // per wave: right-hand side of the particular
    double* cf = carve<double>(cur, NF);
    int* rs = carve<int>(cur, NF);
    int* of = carve<int>(cur, NF);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, li = lane & 15, lk = lane >> 4;
    const bool top = w == 1;                // wave 1 starts from the top row
    const int nrow = top ? BY - 1 - m : m;  // rows of this wave's chain (m >= either)
    const int dir = top ? -1 : 1;
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    S* Ps = Pstore + (size_t)sub * BY * BX * BX;
    double* Psub = Psi + (size_t)sub * R * n;
    double* pb = pbar + (size_t)sub * n;
    S* LTs = LTa + w * BX * LT;
    S* Z = Za + w * BX * RP;
    S* zp = zpa + w * BX;

    const bool scol = lane < BX;
    const bool icol = lane >= BX && lane < 2 * BX;
    const int c = scol ? lane : (icol ? lane - BX : 0);

    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    for (int t = tid; t < 2 * BX * RP; t += 128) Za[t] = S(0);
    if (tid < 2 * BX) zpa[tid] = S(0);
    __syncthreads();
    if (part) {
        // the particular right-hand side of every cell, staged in pbar: the
        // chains read row j + 1 of it during row j, before they overwrite it
        for (int t = tid; t < n; t += 128) {
            const int i = t % BX, jj = t / BX;
            const double qv = qsrc ? qsrc[(size_t)(J * BY + jj) * g.nx + I * BX + i] : 0.0;
            pb[t] = part_rhs<BX>(g, cf, of, bct, bcv, qv, i, jj);
        }
        __syncthreads();
    }
    if (!top || nrow > 0) {                 // f of the first row of each chain
        const int jf = top ? BY - 1 : 0;
        if (nct > 0) add_row_forcing<BX>(g, cf, rs, Z, RP, lane, jf);
        if (part && scol) zp[c] = S(pb[jf * BX + c]);
    }

    // permeability of column c: kq (row being set up), kq1 (the next row of
    // the chain), kq2 (the one after, in flight during a row's work)
    const double* Kc = K + (size_t)J * BY * g.nx + (size_t)I * BX + c;
    // (rows clamped to the subdomain: every load is issued, so that the
    // compiler can count the memory operations in flight)
    auto rowc = [&](int jr) { return jr < 0 ? 0 : (jr >= BY ? BY - 1 : jr); };
    const int j0 = top ? BY - 1 : 0;
    double kq = Kc[(size_t)j0 * g.nx];
    double kq1 = Kc[(size_t)rowc(j0 + dir) * g.nx];
    double kq2 = 1.0;
    // coupling to the previous row of the chain (boundary conductance first)
    double carry = top ? cf[2 * BY + BX + c] : cf[2 * BY + c];
    S a[BX];
    int sing = 0;

    for (int t = 0; t < m; ++t) {
        if (t < nrow) {
            const int j = top ? BY - 1 - t : t;
            const int jd = top ? j - 1 : j;         // coupling to the next row of the chain
            const int jn = j + dir;
            kq2 = Kc[(size_t)rowc(jn + dir) * g.nx];
            const bool fnext = !top || jn > m;      // row m takes f from the lower chain
            const double fpn = pb[jn * BX + c];     // f of the next row (unused without part)
            double dg, txr, txl, tnx;
            if (top) row_coeffs_down<BX>(g, cf, lane, c, j, kq, kq1, carry, &dg, &txr, &txl, &tnx);
            else row_coeffs<BX>(g, cf, lane, c, j, kq, kq1, carry, &dg, &txr, &txl, &tnx);
            build_block_lds<BX, S>(a, t > 0 ? LTs : nullptr, nullptr, dg, txr, txl, scol, icol, c);
            wave_lds_sync();                        // the Schur term is read
            chol_invert<BX, S>(a, LTs, scol, c, sing);
            if (icol) {
#pragma unroll
                for (int i = 0; i < BX; ++i) LTs[c * LT + i] = a[i];
            }
            if (scol) tys[jd * BX + c] = S(tnx);
            wave_lds_sync();
            // P_j to the factor store; L^{-1} is dead once every tile is
            // formed, and its buffer takes the next row's Schur term
            // -(D P_j D)[r][c], row-major
            v4 pacc[NTL][NTL];
            form_inverse<BX, S>(LTs, li, lk, pacc);
#pragma unroll
            for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
                for (int tc = 0; tc < NTL; ++tc)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * tr + M::row(lane, v), cq = 16 * tc + li;
                        const S pv = pacc[tr][tc][v];
                        if (tr >= tc) Ps[(size_t)j * BX * BX + r * BX + cq] = pv;   // lower tiles
                        LTs[r * LT + cq] = -(pv * (tys[jd * BX + r] * tys[jd * BX + cq]));
                    }
            // forward sweep w_j = P_j z_j, then z of the next row = D w_j + f
            for (int ct = 0; ct < nct; ++ct) {
                const int q = 16 * ct + li;
                v4 acc[NTL];
#pragma unroll
                for (int tr = 0; tr < NTL; ++tr) {
                    acc[tr] = v4{S(0), S(0), S(0), S(0)};
#pragma unroll
                    for (int kq4 = 0; kq4 < BX / 4; ++kq4)
                        acc[tr] = M::op(pacc[kq4 >> 2][tr][kq4 & 3], Z[(4 * kq4 + lk) * RP + q], acc[tr]);
                }
#pragma unroll
                for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * tr + M::row(lane, v);
                        if (q < NC) Psub[(size_t)q * n + j * BX + r] = acc[tr][v];
                        Z[r * RP + q] = tys[jd * BX + r] * acc[tr][v];
                    }
            }
            if (part) {
                S wv[NTL];
                part_product<BX>(pacc, zp, lk, wv);
                wave_lds_sync();
                if (lk == 0) {
#pragma unroll
                    for (int tr = 0; tr < NTL; ++tr) {
                        const int r = 16 * tr + li;
                        pb[j * BX + r] = wv[tr];
                        zp[r] = tys[jd * BX + r] * wv[tr];
                    }
                }
            }
            if (fnext) {
                wave_lds_sync();
                if (nct > 0) add_row_forcing<BX>(g, cf, rs, Z, RP, lane, jn);
                if (part && scol) zp[c] += S(fpn);
            }
            wave_lds_sync();
            carry = tnx;
            kq = kq1;
            kq1 = kq2;
        }
    }
    __syncthreads();                        // both chains at row m
    S* Z0 = Za;
    S* Z1 = Za + BX * RP;
    const bool has_lo = m > 0, has_hi = BY - 1 - m > 0;
    if (!top) {
        // ---- row m
        double dg, txr, txl, tnx;
        row_coeffs<BX>(g, cf, lane, c, m, kq, kq1, carry, &dg, &txr, &txl, &tnx);
        build_block_lds<BX, S>(a, has_lo ? LTs : nullptr, has_hi ? LTa + BX * LT : nullptr, dg, txr,
                               txl, scol, icol, c);
        wave_lds_sync();
        chol_invert<BX, S>(a, LTs, scol, c, sing);
        if (icol) {
#pragma unroll
            for (int i = 0; i < BX; ++i) LTs[c * LT + i] = a[i];
        }
        wave_lds_sync();
        v4 pacc[NTL][NTL];
        form_inverse<BX, S>(LTs, li, lk, pacc);
#pragma unroll
        for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
            for (int tc = 0; tc < NTL; ++tc)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * tr + M::row(lane, v), cq = 16 * tc + li;
                    if (tr >= tc) Ps[(size_t)m * BX * BX + r * BX + cq] = pacc[tr][tc][v];
                }
        if (has_hi) {
            for (int t = lane; t < BX * RP; t += 64) Z0[t] += Z1[t];
            if (part && scol) zpa[c] += zpa[BX + c];
            wave_lds_sync();
        }
        if (part) {
            S xv[NTL];
            part_product<BX>(pacc, zpa, lk, xv);
            wave_lds_sync();
            if (lk == 0) {
#pragma unroll
                for (int tr = 0; tr < NTL; ++tr) {
                    const int r = 16 * tr + li;
                    pb[m * BX + r] = xv[tr];
                    if (has_lo) zpa[r] = tys[(m - 1) * BX + r] * xv[tr];
                    if (has_hi) zpa[BX + r] = tys[m * BX + r] * xv[tr];
                }
            }
        }
        if (nct > 0) {
            // x_m = P_m z_m; the backward sweeps start from D_{m-1} x_m and D_m x_m
            for (int ct = 0; ct < nct; ++ct) {
                const int q = 16 * ct + li;
                v4 acc[NTL];
#pragma unroll
                for (int tr = 0; tr < NTL; ++tr) {
                    acc[tr] = v4{S(0), S(0), S(0), S(0)};
#pragma unroll
                    for (int kq4 = 0; kq4 < BX / 4; ++kq4)
                        acc[tr] = M::op(pacc[kq4 >> 2][tr][kq4 & 3], Z0[(4 * kq4 + lk) * RP + q], acc[tr]);
                }
#pragma unroll
                for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * tr + M::row(lane, v);
                        if (q < NC) Psub[(size_t)q * n + m * BX + r] = acc[tr][v];
                        if (has_lo) Z0[r * RP + q] = tys[(m - 1) * BX + r] * acc[tr][v];
                        if (has_hi) Z1[r * RP + q] = tys[m * BX + r] * acc[tr][v];
                    }
            }
        }
    }
    __syncthreads();                        // x_m; the factor store and w_j of both chains
    if (!basis) {
        if (lane == 0 && sing) atomicOr(&flags[FLAG_LOCAL_SINGULAR], 1);
        return;
    }
    // ---- backward sweeps, outwards from row m: the rows of P_j and of w_j
    // (first WCT column tiles, and the particular) are loaded one row ahead
    constexpr int WCT = 2;
    S pn[NTL][BX / 4];
    v4 wn[NTL][WCT];
    S wpn[NTL];
    auto load_row = [&](int jr) {
#pragma unroll
        for (int tr = 0; tr < NTL; ++tr) {
#pragma unroll
            for (int kq4 = 0; kq4 < BX / 4; ++kq4)
                // tile (tr, k / 16) above the diagonal: its transpose (P_j symmetric)
                pn[tr][kq4] = (4 * kq4) / 16 > tr ? Ps[(size_t)jr * BX * BX + (4 * kq4 + lk) * BX + 16 * tr + li]
                                                  : Ps[(size_t)jr * BX * BX + (16 * tr + li) * BX + 4 * kq4 + lk];
#pragma unroll
            for (int ct = 0; ct < WCT; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int q = 16 * ct + li, r = 16 * tr + M::row(lane, v);
                    const S x = Psub[(size_t)(q < NC ? q : 0) * n + jr * BX + r];
                    wn[tr][ct][v] = q < NC ? x : S(0);
                }
            wpn[tr] = pb[jr * BX + 16 * tr + li];    // (unused without part)
        }
    };
    if (nrow > 0) load_row(top ? m + 1 : m - 1);
    for (int t = 0; t < m; ++t) {
        if (t < nrow) {
            const int j = top ? m + 1 + t : m - 1 - t;
            const int jd = top ? j : j - 1;         // coupling to the next row of the sweep
            const bool more = t + 1 < nrow;
            S pc[NTL][BX / 4];
            v4 wc[NTL][WCT];
            S wpc[NTL];
#pragma unroll
            for (int tr = 0; tr < NTL; ++tr) {
#pragma unroll
                for (int kq4 = 0; kq4 < BX / 4; ++kq4) pc[tr][kq4] = pn[tr][kq4];
#pragma unroll
                for (int ct = 0; ct < WCT; ++ct) wc[tr][ct] = wn[tr][ct];
                wpc[tr] = wpn[tr];
            }
            if (more) load_row(j - dir);
            for (int ct = 0; ct < nct; ++ct) {
                const int q = 16 * ct + li;
                v4 acc[NTL];
#pragma unroll
                for (int tr = 0; tr < NTL; ++tr) {
                    if (ct < WCT) {
#pragma unroll
                        for (int u = 0; u < WCT; ++u)
                            if (u == ct) acc[tr] = wc[tr][u];
                    } else {
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int r = 16 * tr + M::row(lane, v);
                            acc[tr][v] = q < NC ? Psub[(size_t)q * n + j * BX + r] : S(0);
                        }
                    }
#pragma unroll
                    for (int kq4 = 0; kq4 < BX / 4; ++kq4)
                        acc[tr] = M::op(pc[tr][kq4], Z[(4 * kq4 + lk) * RP + q], acc[tr]);
                }
#pragma unroll
                for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int r = 16 * tr + M::row(lane, v);
                        if (q < NC) Psub[(size_t)q * n + j * BX + r] = acc[tr][v];
                        if (more) Z[r * RP + q] = tys[jd * BX + r] * acc[tr][v];
                    }
            }
            if (part) {
                // x_j = w_j + P_j z, P_j as held for the products above
                S xv[NTL];
#pragma unroll
                for (int tr = 0; tr < NTL; ++tr) {
                    S sacc = S(0);
#pragma unroll
                    for (int kq4 = 0; kq4 < BX / 4; ++kq4) sacc = fma(pc[tr][kq4], zp[4 * kq4 + lk], sacc);
                    sacc += __shfl_xor(sacc, 16, 64);
                    sacc += __shfl_xor(sacc, 32, 64);
                    xv[tr] = wpc[tr] + sacc;
                }
                wave_lds_sync();
                if (lk == 0) {
#pragma unroll
                    for (int tr = 0; tr < NTL; ++tr) {
                        const int r = 16 * tr + li;
                        pb[j * BX + r] = xv[tr];
                        if (more) zp[r] = tys[jd * BX + r] * xv[tr];
                    }
                }
            }
            wave_lds_sync();
        }
    }
    __syncthreads();
    if (do_traces) {
        // traces T[a][b] = sum_{f in slot a} c_f (x_b(cell f) - delta_ab); the
        // particular column (no delta) to column ld - 1
        double* Tsub = T + (size_t)sub * R * ld;
        const int ncolt = R + part;
        for (int t = tid; t < R * ncolt; t += 128) {
            const int ar = t / ncolt, b = t % ncolt;
            const bool pc = b == R;
            double s = 0.0;
            if (ss[ar] >= 0 && (pc || ss[b] >= 0)) {
                const double* col = pc ? pb : Psub + (size_t)b * n;
                for (int u = 0; u < g.sg; ++u) {
                    const int f = face_of_slot(g, BX, ar, u);
                    int side, i, jj;
                    face_cell(g, BX, f, &side, &i, &jj);
                    s += cf[f] * (col[jj * BX + i] - (ar == b ? 1.0 : 0.0));
                }
            }
            Tsub[(size_t)ar * ld + (pc ? ld - 1 : b)] = s;
        }
    }
    if (lane == 0 && sing) atomicOr(&flags[FLAG_LOCAL_SINGULAR], 1);
}

// One refinement pass on the matrix cores (subdomains 16 or 32 cells wide):
// r = b - A x in FP64 for every column, the correction A32^{-1} r from the
// FP32 factor store by the two sweeps as v_mfma_f32 16x16x4 products, and
// x += correction.  resid[sub] = max over columns of |r|_inf / |b|_inf
// (measured before the correction).  The residual of row j uses lanes as
// (cell c = lane % BX, columns lane / BX + (64 / BX) t); the largest |r| and
// |b| per column are kept per lane and reduced once at the end.
template <int BX>
__global__ __launch_bounds__(64) void k_local_refine_mfma(Geo g, const double* __restrict__ K,
                                                          const int8_t* __restrict__ bct,
                                                          const double* __restrict__ beta,
                                                          const int* __restrict__ slotseg, int R,
                                                          const float* __restrict__ P32,
                                                          double* __restrict__ X, int part,
                                                          const double* __restrict__ q,
                                                          const double* __restrict__ bcv,
                                                          float* __restrict__ Wsc,
                                                          double* __restrict__ resid,
                                                          const int* __restrict__ mask, int apply,
                                                          const int* __restrict__ stop) {
    static_assert(BX == 16 || BX == 32, "MFMA tiles of 16");
    typedef Mfma<float> M;
    typedef M::v4 v4;
    constexpr int LT = BX + 4, NTL = BX / 16, PPL = BX * BX / 64, H = 64 / BX;
    constexpr int MAXC = 16;                // columns per lane kept in registers (ncol <= 16 H)
    const int sub = blockIdx.x;
    if (stop && *stop) return;                   // the refinement has converged
    if (mask && mask[sub] == 1) return;          // redone in FP64
    extern __shared__ __align__(16) char smem[];
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    const int ncol = part ? 1 : R;
    const int RP = (ncol + 15) & ~15, nct = RP / 16;
    char* cur = smem;
    double* x3 = carve<double>(cur, 3 * BX * ncol);   // rows j-1, j, j+1 of x (ring)
    float* zf = carve<float>(cur, BX * RP);           // z_j, later D_j dx_{j+1}
    float* wf = carve<float>(cur, BX * RP);           // w_j, later dx_j
    float* Pl = carve<float>(cur, BX * LT);           // P_j
    float* tys = carve<float>(cur, BY * BX);          // D_j
    double* cf = carve<double>(cur, NF);
    int* rs = carve<int>(cur, NF);
    int* of = carve<int>(cur, NF);
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    const float* Ps = P32 + (size_t)sub * BY * BX * BX;
    double* Xs = X + (size_t)sub * ncol * n;
    float* Ws = Wsc + (size_t)sub * ncol * n;
    const int c = lane % BX, h = lane / BX;           // residual mapping

    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    if (part) {
        // a particular problem with zero data has the solution 0 (set by
        // the particular solve): nothing to refine
        __syncthreads();
        bool nz = false;
        for (int j = 0; j < BY && !nz; ++j) {
            const double qv = q ? q[(size_t)(J * BY + j) * g.nx + I * BX + c] : 0.0;
            nz = part_rhs<BX>(g, cf, of, bct, bcv, qv, c, j) != 0.0;
        }
        if (__ballot(nz) == 0ull) {
            if (lane == 0) resid[sub] = 0.0;
            return;
        }
    }
    for (int t = lane; t < BX * RP; t += 64) zf[t] = 0.f, wf[t] = 0.f;
    for (int t = lane; t < BX * ncol; t += 64) {
        const int i = t % BX, qq = t / BX;
        x3[(1 * BX + i) * ncol + qq] = Xs[(size_t)qq * n + i];
        x3[(2 * BX + i) * ncol + qq] = BY > 1 ? Xs[(size_t)qq * n + BX + i] : 0.0;
    }
    float pr[PPL];
#pragma unroll
    for (int u = 0; u < PPL; ++u) pr[u] = Ps[lane + 64 * u];
    double bmax[MAXC], rmax[MAXC];
#pragma unroll
    for (int t = 0; t < MAXC; ++t) bmax[t] = 0.0, rmax[t] = 0.0;
    __syncthreads();
    double kv[5];
    for (int j = 0; j < BY; ++j) {
#pragma unroll
        for (int u = 0; u < PPL; ++u) {
            const int e = lane + 64 * u;
            Pl[(e / BX) * LT + e % BX] = pr[u];
        }
        if (j + 1 < BY) {
#pragma unroll
            for (int u = 0; u < PPL; ++u) pr[u] = Ps[(size_t)(j + 1) * BX * BX + lane + 64 * u];
        }
        load_kstencil<BX>(g, K, I, J, c, j, kv);
        double dg, txr, tyu;
        stencil_coeffs<BX>(g, kv, cf, c, j, &dg, &txr, &tyu);
        const double txl = c > 0 ? tpx(g, kv[1], kv[0]) : 0.0;
        const double tyd = j > 0 ? tpy(g, kv[3], kv[0]) : 0.0;
        const int rc = (j + 1) % 3, rp = (j + 2) % 3;  // ring slots of rows j and j+1 (j-1: j % 3)
        if (h == 0) tys[j * BX + c] = (float)tyu;
        const double qv = (part && q) ? q[(size_t)(J * BY + j) * g.nx + I * BX + c] : 0.0;
        const double bpart = part ? part_rhs<BX>(g, cf, of, bct, bcv, qv, c, j) : 0.0;
#pragma unroll
        for (int t = 0; t < MAXC; ++t) {
            const int qq = h + H * t;
            if (qq >= ncol) break;
            double b = bpart;
            if (!part) {
                if (c == 0 && rs[j] == qq) b += cf[j];
                if (c == BX - 1 && rs[BY + j] == qq) b += cf[BY + j];
                if (j == 0 && rs[2 * BY + c] == qq) b += cf[2 * BY + c];
                if (j == BY - 1 && rs[2 * BY + BX + c] == qq) b += cf[2 * BY + BX + c];
            }
            double ax = dg * x3[(rc * BX + c) * ncol + qq];
            if (c > 0) ax -= txl * x3[(rc * BX + c - 1) * ncol + qq];
            if (c < BX - 1) ax -= txr * x3[(rc * BX + c + 1) * ncol + qq];
            if (j > 0) ax -= tyd * x3[((j % 3) * BX + c) * ncol + qq];
            if (j < BY - 1) ax -= tyu * x3[(rp * BX + c) * ncol + qq];
            const double r = b - ax;
            bmax[t] = fmax(bmax[t], fabs(b));
            rmax[t] = fmax(rmax[t], fabs(r));
            // z_j = r_j + D_{j-1} w_{j-1}
            zf[c * RP + qq] = (float)r + (j > 0 ? tys[(j - 1) * BX + c] * wf[c * RP + qq] : 0.0f);
        }
        __syncthreads();
        // w_j = P_j z_j
        for (int ct = 0; ct < nct; ++ct) {
#pragma unroll
            for (int tr = 0; tr < NTL; ++tr) {
                v4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kk = 0; kk < BX; kk += 4)
                    acc = M::op(Pl[(16 * tr + li) * LT + kk + lk], zf[(kk + lk) * RP + 16 * ct + li], acc);
                const int qq = 16 * ct + li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * tr + M::row(lane, v);
                    wf[r * RP + qq] = acc[v];
                    if (qq < ncol) Ws[(size_t)qq * n + j * BX + r] = acc[v];
                }
            }
        }
        // shift the ring: row j+2 of x into the slot of row j-1
        if (j + 2 < BY)
            for (int t = lane; t < BX * ncol; t += 64) {
                const int i = t % BX, qq = t / BX;
                x3[((j % 3) * BX + i) * ncol + qq] = Xs[(size_t)qq * n + (j + 2) * BX + i];
            }
        __syncthreads();
    }
    // per-column norms: reduce over the lanes of the same column set
    double m = 0.0;
#pragma unroll
    for (int t = 0; t < MAXC; ++t) {
        double ab = bmax[t], ar = rmax[t];
#pragma unroll
        for (int off = 1; off < BX; off <<= 1) {
            ab = fmax(ab, __shfl_xor(ab, off));
            ar = fmax(ar, __shfl_xor(ar, off));
        }
        const int qq = h + H * t;
        if (qq < ncol) m = fmax(m, ab > 0.0 ? ar / ab : (ar > 0.0 ? 1.0 : 0.0));
    }
    for (int off = BX; off < 64; off <<= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane == 0) resid[sub] = m;
    if (!apply) return;
    // backward: dx_{BY-1} = w_{BY-1}; dx_j = w_j + P_j D_j dx_{j+1}; x_j += dx_j
    for (int t = lane; t < BX * ncol; t += 64) {
        const int i = t % BX, qq = t / BX;
        Xs[(size_t)qq * n + (BY - 1) * BX + i] += (double)wf[i * RP + qq];
    }
    if (BY > 1) {
#pragma unroll
        for (int u = 0; u < PPL; ++u) pr[u] = Ps[(size_t)(BY - 2) * BX * BX + lane + 64 * u];
    }
    for (int j = BY - 2; j >= 0; --j) {
        for (int t = lane; t < BX * RP; t += 64) zf[t] = tys[j * BX + t / RP] * wf[t];
#pragma unroll
        for (int u = 0; u < PPL; ++u) {
            const int e = lane + 64 * u;
            Pl[(e / BX) * LT + e % BX] = pr[u];
        }
        __syncthreads();
        if (j > 0) {
#pragma unroll
            for (int u = 0; u < PPL; ++u) pr[u] = Ps[(size_t)(j - 1) * BX * BX + lane + 64 * u];
        }
        for (int ct = 0; ct < nct; ++ct) {
            const int qq = 16 * ct + li;
            v4 acc[NTL];
#pragma unroll
            for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[tr][v] = qq < ncol ? Ws[(size_t)qq * n + j * BX + 16 * tr + M::row(lane, v)] : 0.f;
#pragma unroll
            for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
                for (int kk = 0; kk < BX; kk += 4)
                    acc[tr] = M::op(Pl[(16 * tr + li) * LT + kk + lk], zf[(kk + lk) * RP + qq], acc[tr]);
#pragma unroll
            for (int tr = 0; tr < NTL; ++tr)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * tr + M::row(lane, v);
                    wf[r * RP + qq] = acc[tr][v];
                    if (qq < ncol) Xs[(size_t)qq * n + j * BX + r] += (double)acc[tr][v];
                }
        }
        __syncthreads();
    }
}

// Traces of the basis (columns 0..R-1) or of the particular solution
// (column R) of the subdomains whose mask entry equals `want`, from the
// stored cell values.
template <int BX>
__global__ __launch_bounds__(64) void k_local_traces(Geo g, const double* __restrict__ K,
                                                     const int8_t* __restrict__ bct,
                                                     const double* __restrict__ beta,
                                                     const int* __restrict__ slotseg, int R,
                                                     const double* __restrict__ X, int part,
                                                     double* __restrict__ T, int ld,
                                                     const int* __restrict__ mask, int want) {
    const int sub = blockIdx.x;
    if (mask && mask[sub] != want) return;
    __shared__ double cf[2 * (32 + 64)];
    __shared__ int rs[2 * (32 + 64)], of[2 * (32 + 64)];
    const int lane = threadIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int n = BX * g.by;
    const int* ss = slotseg + (size_t)sub * R;
    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    __syncthreads();
    double* Tsub = T + (size_t)sub * R * ld;
    if (part) {
        const double* col = X + (size_t)sub * n;
        for (int ar = lane; ar < R; ar += 64) {
            double s = 0.0;
            if (ss[ar] >= 0)
                for (int u = 0; u < g.sg; ++u) {
                    const int f = face_of_slot(g, BX, ar, u);
                    int side, i, jj;
                    face_cell(g, BX, f, &side, &i, &jj);
                    s += cf[f] * col[jj * BX + i];
                }
            Tsub[(size_t)ar * ld + ld - 1] = s;
        }
        return;
    }
    const double* Xs = X + (size_t)sub * R * n;
    for (int t = lane; t < R * R; t += 64) {
        const int ar = t / R, b = t % R;
        double s = 0.0;
        if (ss[ar] >= 0 && ss[b] >= 0) {
            const double* col = Xs + (size_t)b * n;
            for (int u = 0; u < g.sg; ++u) {
                const int f = face_of_slot(g, BX, ar, u);
                int side, i, jj;
                face_cell(g, BX, f, &side, &i, &jj);
                s += cf[f] * (col[jj * BX + i] - (ar == b ? 1.0 : 0.0));
            }
        }
        Tsub[(size_t)ar * ld + b] = s;
    }
}

// ---------------------------------------------------------------- trace correction
// First-order correction of the traces for the rounding of the local solves.
// A trace is a linear functional of a local solution, T[a][b] = t_a . x_b
// (less the conductance of the unit datum itself when a = b), where t_a, the
// Robin conductances on the faces of slot a, is also the right-hand side e_a
// of basis problem a (Section 2.1).  The local matrix A is symmetric, so for
// the exact solution x*_b = A^{-1} e_b
//     t_a . x*_b = t_a . x_b + (A^{-1} e_a) . (e_b - A x_b)
//                = T[a][b] + Psi*_a . r_b,
// and T[a][b] += Psi_a . r_b, with the residual r_b = e_b - A x_b formed in
// FP64, gives the traces of the once-refined solutions up to terms of
// second order, without the correction sweeps (the particular column alike,
// with the particular right-hand side).  Where the local operator is stiff
// (permeability contrast, small Robin parameter) a trace is a small
// difference of cell pressures near a unit datum, and without the
// correction its rounding reaches the interface values through the merges.
//
// One workgroup of four waves per subdomain, each wave a quarter of the
// cells.  The products Psi^T R run on the matrix cores, 16 x 16 output
// tiles: for the k-slice of cells c0 .. c0 + 3, lane l = x + 16 k holds
// Psi_{16 ta + x}(c0 + k) as A operand and r_{16 tb + x}(c0 + k) as B
// operand, the residual formed from the stencil coefficients staged in LDS
// and the neighbouring basis values.  Up to 2 x 2 tiles per pass; the waves'
// partial tiles are added in a fixed order.  basis: columns 0 .. R-1;
// part: the particular column ld - 1 (source q, outer data bcv, solution
// pbar).
template <int BX>
__global__ __launch_bounds__(256) void k_trace_correct(Geo g, const double* __restrict__ K,
                                                       const int8_t* __restrict__ bct,
                                                       const double* __restrict__ beta,
                                                       const int* __restrict__ slotseg, int R,
                                                       const double* __restrict__ Psi,
                                                       const double* __restrict__ pbar,
                                                       const double* __restrict__ q,
                                                       const double* __restrict__ bcv,
                                                       double* __restrict__ T, int ld, int basis,
                                                       int part, const int* __restrict__ list) {
    typedef Mfma<double>::v4 v4;
    extern __shared__ __align__(16) char smem[];
    const int sub = list ? list[blockIdx.x] : blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    const int TT = (R + 15) / 16;                 // 16-column tiles
    const int TG = TT < 2 ? TT : 2;               // tiles per dimension and pass
    char* sp = smem;
    double* cf = carve<double>(sp, NF);
    int* rs = carve<int>(sp, NF);
    int* of = carve<int>(sp, NF);
    double* co = carve<double>(sp, 3 * n);        // per cell: diagonal, coupling right, coupling up
    double* red = carve<double>(sp, 4 * TG * TG * 256);
    double* redp = carve<double>(sp, 4 * 16 * TT);
    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    __syncthreads();
    for (int c = tid; c < n; c += 256) {
        double kv[5], dg, txr, tyu;
        load_kstencil<BX>(g, K, I, J, c % BX, c / BX, kv);
        stencil_coeffs<BX>(g, kv, cf, c % BX, c / BX, &dg, &txr, &tyu);
        co[3 * c] = dg;
        co[3 * c + 1] = txr;
        co[3 * c + 2] = tyu;
    }
    __syncthreads();
    // (A x)(c) for the column x of this subdomain
    auto apply = [&](const double* x, int c) -> double {
        const int i = c % BX, j = c / BX;
        double v = co[3 * c] * x[c];
        if (i > 0) v -= co[3 * (c - 1) + 1] * x[c - 1];
        if (i < BX - 1) v -= co[3 * c + 1] * x[c + 1];
        if (j > 0) v -= co[3 * (c - BX) + 2] * x[c - BX];
        if (j < BY - 1) v -= co[3 * c + 2] * x[c + BX];
        return v;
    };
    // right-hand side of basis problem b at cell c: the conductances of the
    // cell's faces on slot b
    auto ebasis = [&](int b, int c) -> double {
        const int i = c % BX, j = c / BX;
        double e = 0.0;
        if (i == 0 && rs[j] == b) e += cf[j];
        if (i == BX - 1 && rs[BY + j] == b) e += cf[BY + j];
        if (j == 0 && rs[2 * BY + i] == b) e += cf[2 * BY + i];
        if (j == BY - 1 && rs[2 * BY + BX + i] == b) e += cf[2 * BY + BX + i];
        return e;
    };
    const size_t nn = (size_t)n;
    const double* Ps = Psi + (size_t)sub * R * nn;
    double* Ts = T + (size_t)sub * R * ld;
    const int CW = ((n + 15) / 16) * 4;           // cells per wave, a multiple of 4
    const int cb = w * CW;
    if (basis) {
        for (int ta0 = 0; ta0 < TT; ta0 += TG)
            for (int tb0 = 0; tb0 < TT; tb0 += TG) {
                v4 acc[2][2];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v) acc[u][v] = v4{0.0, 0.0, 0.0, 0.0};
                for (int k0 = 0; k0 < CW; k0 += 4) {
                    const int c = cb + k0 + lk;
                    double bo[2], ao[2];
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        const int b = 16 * (tb0 + v) + li;
                        bo[v] = 0.0;
                        if (c < n && b < R && tb0 + v < TT) {
                            const double* xb = Ps + (size_t)b * nn;
                            bo[v] = ebasis(b, c) - apply(xb, c);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int a = 16 * (ta0 + u) + li;
                        ao[u] = (c < n && a < R && ta0 + u < TT) ? Ps[(size_t)a * nn + c] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int v = 0; v < 2; ++v) acc[u][v] = Mfma<double>::op(ao[u], bo[v], acc[u][v]);
                }
                for (int u = 0; u < TG; ++u)
                    for (int v = 0; v < TG; ++v)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            red[((w * TG + u) * TG + v) * 256 + Mfma<double>::row(lane, r) * 16 + li] =
                                acc[u][v][r];
                __syncthreads();
                for (int t = tid; t < TG * TG * 256; t += 256) {
                    const int uv = t / 256, e = t % 256;
                    const int a = 16 * (ta0 + uv / TG) + e / 16, b = 16 * (tb0 + uv % TG) + e % 16;
                    const double s = ((red[t] + red[TG * TG * 256 + t]) + red[2 * TG * TG * 256 + t]) +
                                     red[3 * TG * TG * 256 + t];
                    if (ta0 + uv / TG < TT && tb0 + uv % TG < TT && a < R && b < R && ss[a] >= 0 &&
                        ss[b] >= 0)
                        Ts[(size_t)a * ld + b] += s;
                }
                __syncthreads();
            }
    }
    if (part) {
        const double* qs = q;
        const double* pb = pbar + (size_t)sub * nn;
        for (int ta = 0; ta < TT; ++ta) {
            const int a = 16 * ta + li;
            double acc = 0.0;
            for (int k0 = 0; k0 < CW; k0 += 4) {
                const int c = cb + k0 + lk;
                if (c < n && a < R) {
                    const int i = c % BX, j = c / BX;
                    const double qv = qs[(size_t)(J * BY + j) * g.nx + I * BX + i];
                    const double rp = part_rhs<BX>(g, cf, of, bct, bcv, qv, i, j) - apply(pb, c);
                    acc += Ps[(size_t)a * nn + c] * rp;
                }
            }
            acc += __shfl_xor(acc, 16);
            acc += __shfl_xor(acc, 32);
            if (lk == 0) redp[w * 16 * TT + a] = acc;
        }
        __syncthreads();
        for (int a = tid; a < R; a += 256) {
            const double s = ((redp[a] + redp[16 * TT + a]) + redp[2 * 16 * TT + a]) + redp[3 * 16 * TT + a];
            if (ss[a] >= 0) Ts[(size_t)a * ld + ld - 1] += s;
        }
    }
}

// The same correction for at most 16 TT slots with the subdomain's columns
// staged through LDS.  The basis columns (and with part the particular
// solution and the source) are read in stages of CH consecutive cells (whole
// grid rows), each column's stage one contiguous run of 16-byte loads from
// per-thread base addresses, into a ring of four stages (a cell's neighbours
// above and below lie in the stages before and after its own; the ring's
// power-of-two length makes every neighbour position a mask).  The loads of
// stage s + 2 are issued during stage s - 1 and stored after the work of
// stage s,
// together with the stage's x- and y-transmissibilities (one per thread, the
// two-point harmonic means of the local matrix, zero where the coupling
// leaves the subdomain), while the loads of stage s + 3 are in flight in a
// second register set; that store goes to the ring slot of stage s - 2,
// which no wave reads while working on stage s or s + 1, so one barrier per
// stage suffices.  Wave w takes cells 16 w .. 16 w + 15 of each stage: its
// lanes (cell 16 w + l % 16, column group l / 16) form -A x_b for the group's
// columns b = l / 16 + 4 k from the ring and add the Robin forcing e_b on
// boundary cells, into the wave's part of a residual buffer; then the same
// wave takes those cells through the matrix cores, lane l = x + 16 k holding
// column 16 t + x at cell 16 w + 4 kk + k from the ring (the A operand) and
// from the residual buffer (the B operand).  The four waves' partial tiles
// are added in a fixed order.
template <int CH, int TT>
__host__ __device__ constexpr int tc_ring_doubles(int nc) {  // ring, or the reduction buffers after it
    return nc * (4 * CH + 4) > 4 * TT * TT * 256 + 4 * 32 ? nc * (4 * CH + 4)
                                                          : 4 * TT * TT * 256 + 4 * 32;
}

template <int BX, int TT, int CH>
__global__ __launch_bounds__(256) void k_trace_correct_lds(Geo g, const double* __restrict__ K,
                                                           const int8_t* __restrict__ bct,
                                                           const double* __restrict__ beta,
                                                           const int* __restrict__ slotseg, int R,
                                                           const double* __restrict__ Psi,
                                                           const double* __restrict__ pbar,
                                                           const double* __restrict__ q,
                                                           const double* __restrict__ bcv,
                                                           double* __restrict__ T, int ld, int basis,
                                                           int part) {
    typedef Mfma<double>::v4 v4;
    static_assert(CH == 64 && CH % BX == 0, "a stage is whole grid rows, 16 cells per wave");
    constexpr int NW = 4, RING = 4 * CH, RM = RING - 1;
    constexpr int CS = RING + 4;                           // CS = 4 mod 64: lanes x + 16 k on distinct banks
    constexpr int RS = CH + 4;                             // residual buffer row
    constexpr int G = 4;                                   // column groups (lanes per cell)
    constexpr int KC = (16 * TT + G - 1) / G;              // basis columns per lane (at most)
    constexpr int PAIRS = CH / 2;                          // 16-byte loads per column stage
    constexpr int ML = ((16 * TT + 2) * PAIRS + 255) / 256;
    typedef double d2 __attribute__((ext_vector_type(2)));
    extern __shared__ __align__(16) char smem[];
    const int sub = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    const int I = sub % g.mx, J = sub / g.mx;
    const int NC = R + (part ? 2 : 0);                     // staged columns
    const int NS = (n + CH - 1) / CH;
    const int* ss = slotseg + (size_t)sub * R;
    char* sp = smem;
    double* cf = carve<double>(sp, NF);
    int* rs = carve<int>(sp, NF);
    int* of = carve<int>(sp, NF);
    double* txa = carve<double>(sp, RING);                 // x-transmissibility to the right
    double* tya = carve<double>(sp, RING);                 // y-transmissibility upwards
    double* rb = carve<double>(sp, (size_t)(16 * TT + 1) * RS);
    const int RD = tc_ring_doubles<CH, TT>(NC);
    double* ring = carve<double>(sp, RD);
    // every position the products read holds a finite value (a neighbour
    // outside the subdomain is read and multiplied by a zero coefficient)
    for (int t = tid; t < RD; t += 256) ring[t] = 0.0;
    for (int t = tid; t < RING; t += 256) txa[t] = tya[t] = 0.0;

    const size_t nn = (size_t)n;
    // per-thread sources of the stage loads: column col, pair pr of the stage
    const double* src[ML];
    bool row_major_q[ML];
    int soff[ML];
#pragma unroll
    for (int m = 0; m < ML; ++m) {
        const int e = tid + 256 * m, col = e / PAIRS, o2 = 2 * (e % PAIRS);
        soff[m] = col < NC ? col * CS + o2 : -1;
        row_major_q[m] = col == R + 1;
        src[m] = col < R ? Psi + ((size_t)sub * R + col) * nn + o2
                 : col == R ? pbar + (size_t)sub * nn + o2
                            : q + (size_t)(J * BY + o2 / BX) * g.nx + (size_t)I * BX + o2 % BX;
    }
    // transmissibility of this thread (tid < 2 CH): x (tid < CH) or y
    const int tco = tid % CH;
    const bool tyd = tid >= CH;
    // one stage in registers: the columns' 16-byte pieces of this thread and
    // the two permeabilities of its transmissibility
    struct Stage {
        d2 v[ML];
        double ka, kb;
    };
    auto load = [&](int st, Stage& S) {
#pragma unroll
        for (int m = 0; m < ML; ++m) {
            d2 x = {0.0, 0.0};
            const int c = st * CH + (soff[m] >= 0 ? soff[m] % CS : 0);
            if (soff[m] >= 0 && c < n)
                x = *(const d2*)(src[m] + (row_major_q[m] ? (size_t)st * (CH / BX) * g.nx : (size_t)st * CH));
            S.v[m] = x;
        }
        const int c = st * CH + tco, i = c % BX, j = c / BX;
        S.ka = S.kb = 1.0;
        if (tid < 2 * CH && c < n) {
            // the neighbour's permeability by one load at a selected offset
            // (itself where there is no neighbour; the store then ignores
            // it): loads of one register on divergent paths made the compiler
            // wait for every load in flight, the prefetched stages included
            const double* kc = K + (size_t)(J * BY + j) * g.nx + (size_t)I * BX + i;
            const bool hn = tyd ? j < BY - 1 : i < BX - 1;
            S.ka = kc[0];
            S.kb = kc[hn ? (tyd ? (size_t)g.nx : 1) : 0];
        }
    };
    auto store = [&](int st, const Stage& S) {
        const int base = (st * CH) & RM;
#pragma unroll
        for (int m = 0; m < ML; ++m)
            if (soff[m] >= 0) *(d2*)&ring[soff[m] + base] = S.v[m];
        const int c = st * CH + tco, i = c % BX, j = c / BX;
        if (tid < 2 * CH && c < n) {
            if (tyd) tya[base + tco] = j < BY - 1 ? tpy(g, S.ka, S.kb) : 0.0;
            else txa[base + tco] = i < BX - 1 ? tpx(g, S.ka, S.kb) : 0.0;
        }
    };

    // stages 0 and 1 in the ring, stage 2 in flight (register set A); stage
    // s + 3 is loaded into the other set during stage s
    Stage sa, sb;
    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    load(0, sa);
    if (NS > 1) load(1, sb);
    __syncthreads();
    store(0, sa);
    if (NS > 1) store(1, sb);
    if (NS > 2) load(2, sa);
    __syncthreads();

    v4 acc[TT][TT];
#pragma unroll
    for (int u = 0; u < TT; ++u)
#pragma unroll
        for (int t = 0; t < TT; ++t) acc[u][t] = v4{0.0, 0.0, 0.0, 0.0};
    double pp[TT];
#pragma unroll
    for (int u = 0; u < TT; ++u) pp[u] = 0.0;

    // residual pass: lane on cell offset o of the stage (its wave's cells),
    // columns h + G k
    const int o = 16 * w + li, h = lk;
    const double* xh = ring + (size_t)h * CS;
    double* rh = rb + (size_t)h * RS + o;
    auto stage = [&](int s, Stage& cur, Stage& nxt) {
        if (s + 3 < NS) load(s + 3, nxt);
        {
            // a cell past the subdomain (ragged last stage) takes the first
            // cell's indices and a zero residual
            const int c0 = s * CH + o;
            const bool in = c0 < n;
            const int c = in ? c0 : s * CH;
            const int i = c % BX, j = c / BX;
            const int p = c & RM, pl = (c - 1) & RM, pr = (c + 1) & RM;
            const int pd = (c - BX) & RM, pu = (c + BX) & RM;   // the neighbour rows' stages are in the ring
            const bool hl = i > 0, hr = i < BX - 1, hd = j > 0, hu = j < BY - 1;
            const double cl = hl ? txa[pl] : 0.0, cr = txa[p];
            const double cd = hd ? tya[pd] : 0.0, cu = tya[p];
            const double d0 = (hl ? cl : cf[j]) + (hr ? cr : cf[BY + j]) + (hd ? cd : cf[2 * BY + i]) +
                              (hu ? cu : cf[2 * BY + BX + i]);
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                if (basis && h + G * k < R) {
                    const double* x = xh + G * k * CS;
                    const double av = d0 * x[p] - cl * x[pl] - cr * x[pr] - cd * x[pd] - cu * x[pu];
                    rh[G * k * RS] = in ? -av : 0.0;
                }
            }
            // the Robin forcing of the cell's boundary faces (at most two,
            // on different sides, so in different slots)
            if (in && (!hl || !hr)) {
                const int f = hl ? BY + j : j;
                const int b = rs[f];
                if (basis && b >= 0 && b % G == h) rb[b * RS + o] += cf[f];
            }
            if (in && (!hd || !hu)) {
                const int f = hd ? 2 * BY + BX + i : 2 * BY + i;
                const int b = rs[f];
                if (basis && b >= 0 && b % G == h) rb[b * RS + o] += cf[f];
            }
            if (part && R % G == h) {
                const double* x = ring + (size_t)R * CS;
                const double av = d0 * x[p] - cl * x[pl] - cr * x[pr] - cd * x[pd] - cu * x[pu];
                rb[R * RS + o] = in ? part_rhs<BX>(g, cf, of, bct, bcv, x[CS + p], i, j) - av : 0.0;
            }
        }
        wave_lds_sync();                               // the wave reads only its own cells
        const int sbase = (s * CH) & RM;
#pragma unroll
        for (int kk = 0; kk < CH / (4 * NW); ++kk) {
            const int oc = w * (CH / NW) + 4 * kk + lk;      // cell offset in the stage
            double x0[TT];
#pragma unroll
            for (int t = 0; t < TT; ++t) {
                const int b = 16 * t + li;
                x0[t] = b < R ? ring[(size_t)b * CS + sbase + oc] : 0.0;   // zero past n
            }
            if (basis) {
#pragma unroll
                for (int t = 0; t < TT; ++t) {
                    const int b = 16 * t + li;
                    const double r = b < R ? rb[b * RS + oc] : 0.0;
#pragma unroll
                    for (int u = 0; u < TT; ++u) acc[u][t] = Mfma<double>::op(x0[u], r, acc[u][t]);
                }
            }
            if (part) {
                const double r = rb[R * RS + oc];
#pragma unroll
                for (int u = 0; u < TT; ++u) pp[u] += x0[u] * r;
            }
        }
        if (s + 2 < NS) store(s + 2, cur);            // the slot of stage s - 2
        __syncthreads();
    };
    for (int s = 0; s < NS; s += 2) {
        stage(s, sa, sb);
        if (s + 1 < NS) stage(s + 1, sb, sa);
    }

    double* red = ring;                               // the ring is free after the last stage
    double* redp = ring + NW * TT * TT * 256;
    if (basis) {
#pragma unroll
        for (int u = 0; u < TT; ++u)
#pragma unroll
            for (int t = 0; t < TT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    red[((w * TT + u) * TT + t) * 256 + Mfma<double>::row(lane, r) * 16 + li] = acc[u][t][r];
    }
    if (part) {
#pragma unroll
        for (int u = 0; u < TT; ++u) {
            double a = pp[u];
            a += __shfl_xor(a, 16);
            a += __shfl_xor(a, 32);
            if (lk == 0) redp[w * 32 + 16 * u + li] = a;
        }
    }
    __syncthreads();
    double* Ts = T + (size_t)sub * R * ld;
    if (basis) {
        const int W1 = TT * TT * 256;
        for (int t = tid; t < W1; t += 256) {
            const int uv = t / 256, e = t % 256;
            const int a = 16 * (uv / TT) + e / 16, b = 16 * (uv % TT) + e % 16;
            double sm = 0.0;
            for (int ww = 0; ww < NW; ++ww) sm += red[ww * W1 + t];
            if (a < R && b < R && ss[a] >= 0 && ss[b] >= 0) Ts[(size_t)a * ld + b] += sm;
        }
    }
    if (part)
        for (int a = tid; a < R; a += 256) {
            double sm = 0.0;
            for (int ww = 0; ww < NW; ++ww) sm += redp[ww * 32 + a];
            if (ss[a] >= 0) Ts[(size_t)a * ld + ld - 1] += sm;
        }
}

// ---------------------------------------------------------------- refinement
// One step of iterative refinement of the mixed-precision local solves:
//     r = b - A x   (FP64, the five-point operator applied on the fly)
//     x += A_32^{-1} r   (the two sweeps with the stored FP32 factor)
// for the basis columns (part = 0, X = Psi) or the particular solution
// (part = 1, X = pbar).  resid[sub] receives max_q |r_q|_inf / |b_q|_inf of
// the residual before the correction.  apply = 0 only measures.
template <int BX>
__global__ __launch_bounds__(64) void k_local_refine(Geo g, const double* __restrict__ K,
                                                     const int8_t* __restrict__ bct,
                                                     const double* __restrict__ beta,
                                                     const int* __restrict__ slotseg, int R,
                                                     const float* __restrict__ P32,
                                                     double* __restrict__ X, int part,
                                                     const double* __restrict__ q,
                                                     const double* __restrict__ bcv,
                                                     float* __restrict__ Wsc,
                                                     double* __restrict__ resid,
                                                     const int* __restrict__ mask, int apply,
                                                     const int* __restrict__ stop) {
    const int sub = blockIdx.x;
    // stop: set once the refinement has converged.  mask: 0 plain, 1 redone
    // in FP64 (skipped), 2 basis taken from the surrogate as the starting
    // iterate (FP32 factor only; refined like the others)
    if (stop && *stop) return;
    if (mask && mask[sub] == 1) return;
    extern __shared__ __align__(16) char smem[];
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    const int ncol = part ? 1 : R;
    char* cur = smem;
    double* x3 = carve<double>(cur, 3 * BX * ncol);   // rows j-1, j, j+1 of x (ring)
    float* zf = carve<float>(cur, BX * ncol);         // z_j, later D_j dx_{j+1}
    float* wf = carve<float>(cur, BX * ncol);         // w_j, later dx_j
    float* tys = carve<float>(cur, BY * BX);          // D_j
    double* bn = carve<double>(cur, ncol);            // |b_q|_inf
    double* rn = carve<double>(cur, ncol);            // |r_q|_inf
    double* cf = carve<double>(cur, NF);
    int* rs = carve<int>(cur, NF);
    int* of = carve<int>(cur, NF);
    const int lane = threadIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    const float* Ps = P32 + (size_t)sub * BY * BX * BX;
    double* Xs = X + (size_t)sub * ncol * n;
    float* Ws = Wsc + (size_t)sub * ncol * n;
    const bool act = lane < BX;
    const int c = act ? lane : 0;

    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    for (int t = lane; t < ncol; t += 64) bn[t] = 0.0, rn[t] = 0.0;
    // rows 0 and 1 of x into the ring
    for (int t = lane; t < BX * ncol; t += 64) {
        const int i = t % BX, qq = t / BX;
        x3[(1 * BX + i) * ncol + qq] = Xs[(size_t)qq * n + i];
        x3[(2 * BX + i) * ncol + qq] = BY > 1 ? Xs[(size_t)qq * n + BX + i] : 0.0;
    }
    __syncthreads();
    float pr[BX], pnx[BX];
    if (act) {
#pragma unroll
        for (int k = 0; k < BX; ++k) pnx[k] = Ps[(size_t)k * BX + c];
    }
    double kv[5];
    for (int j = 0; j < BY; ++j) {
#pragma unroll
        for (int k = 0; k < BX; ++k) pr[k] = pnx[k];
        if (act && j + 1 < BY) {
#pragma unroll
            for (int k = 0; k < BX; ++k) pnx[k] = Ps[(size_t)(j + 1) * BX * BX + k * BX + c];
        }
        load_kstencil<BX>(g, K, I, J, c, j, kv);
        double dg, txr, tyu;
        stencil_coeffs<BX>(g, kv, cf, c, j, &dg, &txr, &tyu);
        const double txl = __shfl(txr, lane > 0 ? lane - 1 : 0, 64);
        const double tyd = j > 0 ? tpy(g, kv[3], kv[0]) : 0.0;
        const int rc = (j + 1) % 3, rp = (j + 2) % 3;  // ring slots of rows j and j+1 (j-1: j % 3)
        if (act) tys[j * BX + c] = (float)tyu;
        for (int qq = 0; qq < ncol; ++qq) {
            double b = 0.0, r = 0.0;
            if (act) {
                // right-hand side of cell (c, j), column qq
                if (part) {
                    const double qv = q ? q[(size_t)(J * BY + j) * g.nx + I * BX + c] : 0.0;
                    b = part_rhs<BX>(g, cf, of, bct, bcv, qv, c, j);
                } else {
                    if (c == 0 && rs[j] == qq) b += cf[j];
                    if (c == BX - 1 && rs[BY + j] == qq) b += cf[BY + j];
                    if (j == 0 && rs[2 * BY + c] == qq) b += cf[2 * BY + c];
                    if (j == BY - 1 && rs[2 * BY + BX + c] == qq) b += cf[2 * BY + BX + c];
                }
                const double xc = x3[(rc * BX + c) * ncol + qq];
                double ax = dg * xc;
                if (c > 0) ax -= txl * x3[(rc * BX + c - 1) * ncol + qq];
                if (c < BX - 1) ax -= txr * x3[(rc * BX + c + 1) * ncol + qq];
                if (j > 0) ax -= tyd * x3[((j % 3) * BX + c) * ncol + qq];
                if (j < BY - 1) ax -= tyu * x3[(rp * BX + c) * ncol + qq];
                r = b - ax;
                zf[c * ncol + qq] = (float)r + (j > 0 ? tys[(j - 1) * BX + c] * wf[c * ncol + qq] : 0.0f);
            }
            double ab = fabs(b), ar = fabs(r);
            for (int off = 32; off > 0; off >>= 1) {
                ab = fmax(ab, __shfl_xor(ab, off));
                ar = fmax(ar, __shfl_xor(ar, off));
            }
            if (lane == 0) {
                bn[qq] = fmax(bn[qq], ab);
                rn[qq] = fmax(rn[qq], ar);
            }
        }
        __syncthreads();
        // w_j = P_j z_j
        if (act)
            for (int qq = 0; qq < ncol; ++qq) {
                float s = 0.0f;
#pragma unroll
                for (int k = 0; k < BX; ++k) s = fmaf(pr[k], zf[k * ncol + qq], s);
                Ws[(size_t)qq * n + j * BX + c] = s;
                wf[c * ncol + qq] = s;
            }
        // shift the ring: load row j+2 of x into the slot of row j-1
        if (j + 2 < BY)
            for (int t = lane; t < BX * ncol; t += 64) {
                const int i = t % BX, qq = t / BX;
                x3[((j % 3) * BX + i) * ncol + qq] = Xs[(size_t)qq * n + (j + 2) * BX + i];
            }
        __syncthreads();
    }
    if (lane == 0) {
        double m = 0.0;
        for (int qq = 0; qq < ncol; ++qq)
            if (bn[qq] > 0.0) m = fmax(m, rn[qq] / bn[qq]);
            else if (rn[qq] > 0.0) m = fmax(m, 1.0);
        resid[sub] = m;
    }
    if (!apply) return;
    // backward: dx_{BY-1} = w_{BY-1}; dx_j = w_j + P_j D_j dx_{j+1}; x_j += dx_j
    if (act) {
        for (int qq = 0; qq < ncol; ++qq)
            Xs[(size_t)qq * n + (BY - 1) * BX + c] += (double)wf[c * ncol + qq];
    }
    if (act && BY > 1) {
#pragma unroll
        for (int k = 0; k < BX; ++k) pnx[k] = Ps[(size_t)(BY - 2) * BX * BX + k * BX + c];
    }
    for (int j = BY - 2; j >= 0; --j) {
#pragma unroll
        for (int k = 0; k < BX; ++k) pr[k] = pnx[k];
        if (act && j > 0) {
#pragma unroll
            for (int k = 0; k < BX; ++k) pnx[k] = Ps[(size_t)(j - 1) * BX * BX + k * BX + c];
        }
        if (act)
            for (int qq = 0; qq < ncol; ++qq) zf[c * ncol + qq] = tys[j * BX + c] * wf[c * ncol + qq];
        __syncthreads();
        if (act)
            for (int qq = 0; qq < ncol; ++qq) {
                float s = Ws[(size_t)qq * n + j * BX + c];
#pragma unroll
                for (int k = 0; k < BX; ++k) s = fmaf(pr[k], zf[k * ncol + qq], s);
                wf[c * ncol + qq] = s;
                Xs[(size_t)qq * n + j * BX + c] += (double)s;
            }
        __syncthreads();
    }
}

// Subdomains whose refinement did not reach the tolerance are redone in
// FP64: mask = 1 marks them; their number is added to flags[3].
__global__ void k_mark_fallback(int nsub, const double* __restrict__ resid, double tol,
                                int* __restrict__ fb, int* __restrict__ flags,
                                const int* __restrict__ conv) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (*conv || s >= nsub || fb[s] == 1) return;
    const int f = !(resid[s] <= tol);
    fb[s] = f;
    if (f) atomicAdd(&flags[FLAG_FALLBACK], 1);
}

// Largest residual of a refinement pass over the subdomains it refined (one
// block, fixed order), kept in the pass history; st = {converged, passes}:
// the pass count advances and converged is set once the residual measured
// before a correction is within tol.  Nothing happens after convergence.
__global__ __launch_bounds__(256) void k_max_resid(int nsub, const double* __restrict__ resid,
                                                   const int* __restrict__ mask, double tol,
                                                   int* __restrict__ st, double* __restrict__ hist,
                                                   int nhist) {
    __shared__ double s[256];
    if (st[0]) return;
    double m = 0.0;
    // a NaN residual (a diverged refinement) is kept: it must not pass
    auto mx = [](double a, double b) { return (b > a || b != b) ? b : a; };
    for (int t = threadIdx.x; t < nsub; t += 256)
        if (!mask || mask[t] != 1) m = mx(m, resid[t]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] = mx(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int k = st[1];
        if (k < nhist) hist[k] = s[0];
        st[1] = k + 1;
        if (s[0] <= tol) st[0] = 1;
    }
}

// Particular solutions whose refinement did not reach tol (only when the
// refinement as a whole did not converge): their subdomains are solved
// again in FP64 by the solve (pfb = 1, counted); subdomains already in FP64
// are skipped.
__global__ void k_mark_part_fallback(int nsub, const double* __restrict__ resid, double tol,
                                     const int* __restrict__ fb, int* __restrict__ pfb,
                                     int* __restrict__ flags, const int* __restrict__ conv) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (*conv || s >= nsub || fb[s] == 1) return;
    if (!(resid[s] <= tol)) {
        pfb[s] = 1;
        atomicAdd(&flags[FLAG_PFALLBACK], 1);
    }
}

// ---------------------------------------------------------------- K1p
// Particular solution (source and outer boundary data, zero Robin data)
// with the stored P_j: one wavefront per subdomain, lane c holding row c of
// P_j; writes pbar and (do_traces) the particular trace column.  A
// subdomain whose right-hand side vanishes has pbar = 0 and is finished at
// once.
template <int BX, typename S>
__global__ __launch_bounds__(64) void k_local_particular(
    Geo g, const double* __restrict__ K, const int8_t* __restrict__ bct,
    const double* __restrict__ beta, const int* __restrict__ slotseg, int R,
    const double* __restrict__ q, const double* __restrict__ bcv,
    const S* __restrict__ Pstore, double* __restrict__ pbar, double* __restrict__ T, int ld,
    const int* __restrict__ mask, int want, int do_traces) {
    const int sub = blockIdx.x;
    if (mask && mask[sub] != want) return;
    extern __shared__ __align__(16) char smem[];
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY);
    char* cur = smem;
    double* fs = carve<double>(cur, n);     // right-hand side, then w, then x
    S* z = carve<S>(cur, BX);
    double* cf = carve<double>(cur, NF);
    int* rs = carve<int>(cur, NF);
    int* of = carve<int>(cur, NF);
    __shared__ int nonzero;
    const int lane = threadIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    const S* Ps = Pstore + (size_t)sub * BY * BX * BX;
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
        if (do_traces)
            for (int a = lane; a < R; a += 64) Tsub[(size_t)a * ld + ld - 1] = 0.0;
        return;
    }
    S p[BX], pn[BX];
    if (act) {
#pragma unroll
        for (int k = 0; k < BX; ++k) pn[k] = Ps[(size_t)k * BX + c];
    }
    S w = S(0), dprev = S(0);
    double kv[5];
    for (int j = 0; j < BY; ++j) {
#pragma unroll
        for (int k = 0; k < BX; ++k) p[k] = pn[k];
        if (act && j + 1 < BY) {
#pragma unroll
            for (int k = 0; k < BX; ++k) pn[k] = Ps[(size_t)(j + 1) * BX * BX + k * BX + c];
        }
        load_kstencil<BX>(g, K, I, J, c, j, kv);
        if (act) z[c] = S(fs[j * BX + c]) + dprev * w;
        __syncthreads();
        if (act) {
            S s = S(0);
#pragma unroll
            for (int k = 0; k < BX; ++k) s = fma(p[k], z[k], s);
            w = s;
            fs[j * BX + c] = (double)s;
            dprev = j + 1 < BY ? S(tpy(g, kv[0], kv[4])) : S(0);
            pb[j * BX + c] = (double)dprev;   // D_j staged in the output; overwritten at the end
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
        if (act) z[c] = S(pb[j * BX + c]) * w;
        __syncthreads();
        if (act) {
            S s = S(fs[j * BX + c]);
#pragma unroll
            for (int k = 0; k < BX; ++k) s = fma(p[k], z[k], s);
            w = s;
            fs[j * BX + c] = (double)s;
        }
        __syncthreads();
    }
    for (int t = lane; t < n; t += 64) pb[t] = fs[t];
    __syncthreads();
    if (do_traces)
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

// Particular solution with the FP64 factor store of the twisted elimination
// (subdomains 16 or 32 cells wide): lanes 0..BX-1 sweep rows 0..m-1
// upwards, lanes BX..2BX-1 rows by-1..m+1 downwards (lane c of a chain
// holding row c of P_j), both meet at row m, and the backward sweeps run
// outwards from it.  Output as above.
template <int BX>
__global__ __launch_bounds__(64) void k_local_particular_twist(
    Geo g, const double* __restrict__ K, const int8_t* __restrict__ bct,
    const double* __restrict__ beta, const int* __restrict__ slotseg, int R,
    const double* __restrict__ q, const double* __restrict__ bcv,
    const double* __restrict__ Pstore, double* __restrict__ pbar, double* __restrict__ T, int ld,
    const int* __restrict__ mask, int want, int do_traces) {
    static_assert(2 * BX <= 64, "two chains of BX lanes");
    const int sub = blockIdx.x;
    if (mask && mask[sub] != want) return;
    extern __shared__ __align__(16) char smem[];
    const int BY = g.by, n = BX * BY, NF = 2 * (BX + BY), m = BY / 2;
    char* cur = smem;
    double* fs = carve<double>(cur, n);     // right-hand side, then w, then x
    double* zb = carve<double>(cur, 2 * BX);
    double* cf = carve<double>(cur, NF);
    int* rs = carve<int>(cur, NF);
    int* of = carve<int>(cur, NF);
    __shared__ int nonzero;
    const int lane = threadIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    const double* Ps = Pstore + (size_t)sub * BY * BX * BX;
    double* pb = pbar + (size_t)sub * n;
    double* Tsub = T + (size_t)sub * R * ld;
    const int h = lane / BX;                // 0: upwards from row 0, 1: downwards from the top
    const int c = lane % BX;
    const int nrow = h == 0 ? m : (h == 1 ? BY - 1 - m : 0);
    const int dir = h == 0 ? 1 : -1;

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
        if (do_traces)
            for (int a = lane; a < R; a += 64) Tsub[(size_t)a * ld + ld - 1] = 0.0;
        return;
    }
    const double* Kc = K + (size_t)J * BY * g.nx + (size_t)I * BX + c;
    double p[BX], pn[BX];
    auto load_p = [&](int jr) {
#pragma unroll
        for (int k = 0; k < BX; ++k)   // P[k][c]; above the diagonal tiles, P[c][k] (lower tiles only)
            pn[k] = k / 16 < c / 16 ? Ps[(size_t)jr * BX * BX + c * BX + k] : Ps[(size_t)jr * BX * BX + k * BX + c];
    };
    if (nrow > 0) load_p(h == 0 ? 0 : BY - 1);
    double wv = 0.0, dprev = 0.0;
    for (int t = 0; t < m; ++t) {
        const bool on = t < nrow;
        const int j = h == 0 ? t : BY - 1 - t;
        const int jd = h == 0 ? j : j - 1;      // coupling to the next row of the chain
#pragma unroll
        for (int k = 0; k < BX; ++k) p[k] = pn[k];
        if (on && t + 1 < nrow) load_p(j + dir);
        double klo = 1.0, khi = 1.0;
        if (on) {
            klo = Kc[(size_t)jd * g.nx];
            khi = Kc[(size_t)(jd + 1) * g.nx];
            zb[h * BX + c] = fs[j * BX + c] + dprev * wv;
        }
        __syncthreads();
        if (on) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < BX; ++k) s = fma(p[k], zb[h * BX + k], s);
            wv = s;
            fs[j * BX + c] = s;
            dprev = tpy(g, klo, khi);
            pb[jd * BX + c] = dprev;            // D staged in the output; overwritten at the end
        }
        __syncthreads();
    }
    // row m: z_m = f_m + D_{m-1} w_{m-1} + D_m w_{m+1}
    if (h == 1) zb[BX + c] = dprev * wv;
    if (h == 0) load_p(m);
    __syncthreads();
    if (h == 0) zb[c] = (fs[m * BX + c] + dprev * wv) + zb[BX + c];
    __syncthreads();
    if (h == 0) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < BX; ++k) s = fma(pn[k], zb[k], s);
        wv = s;
        fs[m * BX + c] = s;
    }
    __syncthreads();
    if (h == 1) wv = fs[m * BX + c];
    if (nrow > 0) load_p(m - dir);
    for (int t = 0; t < m; ++t) {
        const bool on = t < nrow;
        const int j = h == 0 ? m - 1 - t : m + 1 + t;
        const int jd = h == 0 ? j : j - 1;      // coupling to the row solved before
#pragma unroll
        for (int k = 0; k < BX; ++k) p[k] = pn[k];
        if (on && t + 1 < nrow) load_p(j - dir);
        if (on) zb[h * BX + c] = pb[jd * BX + c] * wv;
        __syncthreads();
        if (on) {
            double s = fs[j * BX + c];
#pragma unroll
            for (int k = 0; k < BX; ++k) s = fma(p[k], zb[h * BX + k], s);
            wv = s;
            fs[j * BX + c] = s;
        }
        __syncthreads();
    }
    for (int t = lane; t < n; t += 64) pb[t] = fs[t];
    __syncthreads();
    if (do_traces)
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
template <int BX, typename S>
static hipError_t setup_bx(rmrcm_ctx* c, S* P, const int* mask, int want, int do_traces, int basis,
                            int part) {
    if constexpr (BX >= 16 && std::is_same<S, double>::value) {
        const Level& L = c->levels[c->D];
        const int R = L.nslot, BY = c->geo.by, NF = 2 * (BX + BY);
        const int RP = basis ? (R + 15) & ~15 : 0;
        const size_t lds = carve_bytes(2 * BX * (BX + 4), 8) + carve_bytes(2 * BX * RP, 8) +
                           carve_bytes(BY * BX, 8) + carve_bytes(2 * BX, 8) + carve_bytes(NF, 8) +
                           2 * carve_bytes(NF, 4);
        const int nsub = c->geo.mx * c->geo.my;
        auto go = [&](auto kern) -> hipError_t {
            hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3(nsub), dim3(128), lds, c->stream, c->geo, c->K, c->bct,
                               c->beta, L.slotseg, R, P, c->Psi, L.T, L.ld, c->flags, mask, want,
                               do_traces, basis, c->q, c->bcv, c->pbar);
            return hipGetLastError();
        };
        if (part && basis) {
            switch (RP / 16) {
                case 1: return go(k_local_setup_twist<BX, 1, true>);
                case 2: return go(k_local_setup_twist<BX, 2, true>);
                default: return go(k_local_setup_twist<BX, 0, true>);
            }
        }
        switch (RP / 16) {
            case 1: return go(k_local_setup_twist<BX, 1, false>);
            case 2: return go(k_local_setup_twist<BX, 2, false>);
            default: return go(k_local_setup_twist<BX, 0, false>);
        }
    } else if constexpr (BX >= 16) {
        const Level& L = c->levels[c->D];
        const int R = L.nslot, BY = c->geo.by, NF = 2 * (BX + BY), RP = (R + 15) & ~15;
        const size_t lds = carve_bytes(BX * (BX + 4), sizeof(S)) + carve_bytes(chol_wb_entries<BX, S>(), sizeof(S)) +
                           2 * carve_bytes(BX * RP, sizeof(S)) + carve_bytes(BY * BX, sizeof(S)) +
                           carve_bytes(NF, 8) + 2 * carve_bytes(NF, 4);
        hipError_t e = hipFuncSetAttribute((const void*)k_local_setup_mfma<BX, S>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        const int nsub = c->geo.mx * c->geo.my;
        hipLaunchKernelGGL((k_local_setup_mfma<BX, S>), dim3(nsub), dim3(128), lds, c->stream, c->geo,
                           c->K, c->bct, c->beta, L.slotseg, R, P, c->Psi, L.T, L.ld, c->flags, mask,
                           want, do_traces, basis, std::is_same<S, float>::value ? c->fb : nullptr);
        return hipGetLastError();
    }
    const Level& L = c->levels[c->D];
    const int R = L.nslot, BY = c->geo.by, NF = 2 * (BX + BY);
    const size_t lds = carve_bytes(BX * (BX + 1), sizeof(S)) + 2 * carve_bytes(BX * R, sizeof(S)) +
                       carve_bytes(BY * BX, sizeof(S)) + carve_bytes(NF, 8) + 2 * carve_bytes(NF, 4);
    hipError_t e = hipFuncSetAttribute((const void*)k_local_setup<BX, S>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL((k_local_setup<BX, S>), dim3(nsub), dim3(64), lds, c->stream, c->geo, c->K,
                       c->bct, c->beta, L.slotseg, R, P, c->Psi, L.T, L.ld, c->flags, mask, want,
                       do_traces, basis, std::is_same<S, float>::value ? c->fb : nullptr);
    return hipGetLastError();
}

template <int BX, typename S>
static hipError_t part_bx(rmrcm_ctx* c, const S* P, const int* mask, int want, int do_traces) {
    const Level& L = c->levels[c->D];
    const int BY = c->geo.by, NF = 2 * (BX + BY);
    if constexpr (BX >= 16 && std::is_same<S, double>::value) {
        // the factor store of the twisted elimination
        const size_t lds = carve_bytes(BX * BY, 8) + carve_bytes(2 * BX, 8) + carve_bytes(NF, 8) +
                           2 * carve_bytes(NF, 4);
        hipError_t e = hipFuncSetAttribute((const void*)k_local_particular_twist<BX>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        const int nsub = c->geo.mx * c->geo.my;
        hipLaunchKernelGGL((k_local_particular_twist<BX>), dim3(nsub), dim3(64), lds, c->stream,
                           c->geo, c->K, c->bct, c->beta, L.slotseg, L.nslot, c->q, c->bcv, P,
                           c->pbar, L.T, L.ld, mask, want, do_traces);
        return hipGetLastError();
    }
    const size_t lds = carve_bytes(BX * BY, 8) + carve_bytes(BX, sizeof(S)) + carve_bytes(NF, 8) +
                       2 * carve_bytes(NF, 4);
    hipError_t e = hipFuncSetAttribute((const void*)k_local_particular<BX, S>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL((k_local_particular<BX, S>), dim3(nsub), dim3(64), lds, c->stream, c->geo,
                       c->K, c->bct, c->beta, L.slotseg, L.nslot, c->q, c->bcv, P, c->pbar, L.T,
                       L.ld, mask, want, do_traces);
    return hipGetLastError();
}

template <int BX>
static hipError_t refine_bx(rmrcm_ctx* c, int part, int apply) {
    const Level& L = c->levels[c->D];
    const int R = L.nslot, BY = c->geo.by, NF = 2 * (BX + BY);
    const int ncol = part ? 1 : R;
    if constexpr (BX >= 16) {
        if (ncol <= 16 * (64 / BX)) {
            const int RP = (ncol + 15) & ~15;
            const size_t lds = carve_bytes(3 * BX * ncol, 8) + 2 * carve_bytes(BX * RP, 4) +
                               carve_bytes(BX * (BX + 4), 4) + carve_bytes(BY * BX, 4) +
                               carve_bytes(NF, 8) + 2 * carve_bytes(NF, 4);
            hipError_t e = hipFuncSetAttribute((const void*)k_local_refine_mfma<BX>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            const int nsub = c->geo.mx * c->geo.my;
            hipLaunchKernelGGL(k_local_refine_mfma<BX>, dim3(nsub), dim3(64), lds, c->stream, c->geo,
                               c->K, c->bct, c->beta, L.slotseg, R, c->P32, part ? c->pbar : c->Psi,
                               part, c->q, c->bcv, c->Wsc, c->resid, c->fb, apply, c->irst + 2 * part);
            return hipGetLastError();
        }
    }
    const size_t lds = carve_bytes(3 * BX * ncol, 8) + 2 * carve_bytes(BX * ncol, 4) +
                       carve_bytes(BY * BX, 4) + 2 * carve_bytes(ncol, 8) + carve_bytes(NF, 8) +
                       2 * carve_bytes(NF, 4);
    hipError_t e = hipFuncSetAttribute((const void*)k_local_refine<BX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL(k_local_refine<BX>, dim3(nsub), dim3(64), lds, c->stream, c->geo, c->K,
                       c->bct, c->beta, L.slotseg, R, c->P32, part ? c->pbar : c->Psi, part, c->q,
                       c->bcv, c->Wsc, c->resid, c->fb, apply, c->irst + 2 * part);
    return hipGetLastError();
}

template <int BX>
static hipError_t traces_bx(rmrcm_ctx* c, int part, const int* mask, int want) {
    const Level& L = c->levels[c->D];
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL(k_local_traces<BX>, dim3(nsub), dim3(64), 0, c->stream, c->geo, c->K, c->bct,
                       c->beta, L.slotseg, L.nslot, part ? c->pbar : c->Psi, part, L.T, L.ld, mask,
                       want);
    return hipGetLastError();
}

// The correction on the subdomains of list (nsub of them; null: all).
template <int BX>
static hipError_t trace_correct_bx(rmrcm_ctx* c, int basis, int part, const int* list, int nsub) {
    const Level& L = c->levels[c->D];
    const int R = L.nslot, BY = c->geo.by, NF = 2 * (BX + BY), n = BX * BY;
    if (R <= 32) {
        const int NC = R + (part ? 2 : 0);
        auto go = [&](auto kern, int tt, int ch, int ring) -> hipError_t {
            const size_t lds = carve_bytes(NF, 8) + 2 * carve_bytes(NF, 4) + 2 * carve_bytes(4 * ch, 8) +
                               carve_bytes((size_t)(16 * tt + 1) * (ch + 4), 8) + carve_bytes(ring, 8);
            hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(kern, dim3(nsub), dim3(256), lds, c->stream, c->geo, c->K, c->bct, c->beta,
                               L.slotseg, R, c->Psi, c->pbar, c->q, c->bcv, L.T, L.ld, basis, part);
            return hipGetLastError();
        };
        if (R <= 16) return go(k_trace_correct_lds<BX, 1, 64>, 1, 64, tc_ring_doubles<64, 1>(NC));
        return go(k_trace_correct_lds<BX, 2, 64>, 2, 64, tc_ring_doubles<64, 2>(NC));
    }
    const int TT = (R + 15) / 16, TG = TT < 2 ? TT : 2;
    const size_t lds = carve_bytes(NF, 8) + 2 * carve_bytes(NF, 4) + carve_bytes(3 * n, 8) +
                       carve_bytes(4 * TG * TG * 256, 8) + carve_bytes(4 * 16 * TT, 8);
    hipError_t e = hipFuncSetAttribute((const void*)k_trace_correct<BX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_trace_correct<BX>, dim3(nsub), dim3(256), lds, c->stream, c->geo, c->K, c->bct,
                       c->beta, L.slotseg, R, c->Psi, c->pbar, c->q, c->bcv, L.T, L.ld, basis, part, list);
    return hipGetLastError();
}

hipError_t launch_check_beta(rmrcm_ctx* c, double* copy) {
    const size_t n = geo_ncell(c->geo);
    const int nbc = 2048, nbb = (c->geo.nseg + 255) / 256;
    hipLaunchKernelGGL(k_check_beta, dim3(nbc + nbb), dim3(256), 0, c->stream, c->geo, c->K, n, c->flags, copy,
                       nbc, c->beta, c->seglen);
    return hipGetLastError();
}

#define RMRCM_BX_SWITCH(call4, call8, call16, call32) \
    switch (c->geo.bx) {                              \
        case 4: return call4;                         \
        case 8: return call8;                         \
        case 16: return call16;                       \
        case 32: return call32;                       \
    }                                                 \
    return hipErrorInvalidValue;

hipError_t launch_local_setup(rmrcm_ctx* c, bool fp32, const int* mask, int want, int do_traces,
                              int basis, int part) {
    if (c->geo.three_d) return fp32 || mask || !basis ? hipErrorInvalidValue : launch_local3d(c, 1, 1, part);
    if (part && !local_setup_solves_particular(c, fp32)) return hipErrorInvalidValue;
    if (fp32) {
        RMRCM_BX_SWITCH((setup_bx<4, float>(c, c->P32, mask, want, do_traces, basis, 0)),
                        (setup_bx<8, float>(c, c->P32, mask, want, do_traces, basis, 0)),
                        (setup_bx<16, float>(c, c->P32, mask, want, do_traces, basis, 0)),
                        (setup_bx<32, float>(c, c->P32, mask, want, do_traces, basis, 0)))
    }
    RMRCM_BX_SWITCH((setup_bx<4, double>(c, c->Pstore, mask, want, do_traces, basis, 0)),
                    (setup_bx<8, double>(c, c->Pstore, mask, want, do_traces, basis, 0)),
                    (setup_bx<16, double>(c, c->Pstore, mask, want, do_traces, basis, part)),
                    (setup_bx<32, double>(c, c->Pstore, mask, want, do_traces, basis, part)))
}

bool local_setup_solves_particular(const rmrcm_ctx* c, bool fp32) {
    return !fp32 && (c->geo.three_d || c->geo.bx == 16 || c->geo.bx == 32);
}

hipError_t launch_local_particular(rmrcm_ctx* c, bool fp32, const int* mask, int want,
                                   int do_traces) {
    if (c->geo.three_d) return fp32 || mask ? hipErrorInvalidValue : launch_local3d(c, 0, 0, 1);
    if (fp32) {
        RMRCM_BX_SWITCH((part_bx<4, float>(c, c->P32, mask, want, do_traces)),
                        (part_bx<8, float>(c, c->P32, mask, want, do_traces)),
                        (part_bx<16, float>(c, c->P32, mask, want, do_traces)),
                        (part_bx<32, float>(c, c->P32, mask, want, do_traces)))
    }
    RMRCM_BX_SWITCH((part_bx<4, double>(c, c->Pstore, mask, want, do_traces)),
                    (part_bx<8, double>(c, c->Pstore, mask, want, do_traces)),
                    (part_bx<16, double>(c, c->Pstore, mask, want, do_traces)),
                    (part_bx<32, double>(c, c->Pstore, mask, want, do_traces)))
}

hipError_t launch_local_refine(rmrcm_ctx* c, int part, int apply) {
    RMRCM_BX_SWITCH((refine_bx<4>(c, part, apply)), (refine_bx<8>(c, part, apply)),
                    (refine_bx<16>(c, part, apply)), (refine_bx<32>(c, part, apply)))
}

hipError_t launch_trace_correct(rmrcm_ctx* c, int basis, int part) {
    if (c->geo.three_d) return hipSuccess;   // the 3D traces are formed from the solution directly
    const int nsub = c->geo.mx * c->geo.my;
    RMRCM_BX_SWITCH((trace_correct_bx<4>(c, basis, part, nullptr, nsub)),
                    (trace_correct_bx<8>(c, basis, part, nullptr, nsub)),
                    (trace_correct_bx<16>(c, basis, part, nullptr, nsub)),
                    (trace_correct_bx<32>(c, basis, part, nullptr, nsub)))
}

hipError_t launch_local_traces(rmrcm_ctx* c, int part, const int* mask, int want) {
    RMRCM_BX_SWITCH((traces_bx<4>(c, part, mask, want)), (traces_bx<8>(c, part, mask, want)),
                    (traces_bx<16>(c, part, mask, want)), (traces_bx<32>(c, part, mask, want)))
}

// Input features of the local-basis surrogate network for every subdomain
// (square subdomains): channel 0 the log-permeability minus its mean over
// the subdomain, channel 1 on boundary cells the mean over the cell's
// Robin faces of log(beta) + that mean (0 elsewhere).  Both are unchanged
// when K is scaled (beta scales inversely, Section 5.1), as is the basis.
// interior[sub] = 1 when every boundary slot of the subdomain is a Robin
// slot (no face on the outer boundary).
__global__ __launch_bounds__(256) void k_features(Geo g, const double* __restrict__ K,
                                                  const double* __restrict__ beta,
                                                  const int* __restrict__ slotseg, int R,
                                                  float* __restrict__ x, int* __restrict__ interior) {
    __shared__ double red[256];
    const int sub = blockIdx.x, tid = threadIdx.x;
    const int I = sub % g.mx, J = sub / g.mx, S = g.bx, n = S * S;
    const int* ss = slotseg + (size_t)sub * R;
    double acc = 0.0;
    for (int c = tid; c < n; c += 256) acc += log(K[(size_t)(J * S + c / S) * g.nx + I * S + c % S]);
    red[tid] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double m = red[0] / n;
    float* x0 = x + (size_t)sub * 2 * n;
    float* x1 = x0 + n;
    for (int c = tid; c < n; c += 256) {
        const int i = c % S, j = c / S;
        x0[c] = (float)(log(K[(size_t)(J * S + j) * g.nx + I * S + i]) - m);
        const int sl[4] = {i == 0 ? j / g.sg : -1, i == S - 1 ? g.nsy + j / g.sg : -1,
                           j == 0 ? 2 * g.nsy + i / g.sg : -1,
                           j == S - 1 ? 2 * g.nsy + g.nsx + i / g.sg : -1};
        double a = 0.0;
        int k = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (sl[s] < 0) continue;
            const int code = ss[sl[s]];
            if (code < 0) continue;
            a += log(beta[code >> 1]) + m;
            ++k;
        }
        x1[c] = k ? (float)(a / k) : 0.f;
    }
    if (tid == 0) {
        int all = 1;
        for (int a = 0; a < R; ++a) all &= ss[a] >= 0;
        interior[sub] = all;
    }
}

// Residual gate of the surrogate's basis: for every column a of an interior
// subdomain, rel_a = |A y_a - e_a|_2 / |e_a|_2 in FP64, with A the local
// Robin matrix and e_a the right-hand side of the basis problem of slot a
// (the Robin conductance on the slot's faces).  The prediction is accepted
// (fb = 2, written to Psi in FP64 as the starting iterate of the FP64-residual
// refinement) when every rel_a <= tau; the largest rel_a goes to resid (the
// gate residual of the subdomain), accepted subdomains are counted.
template <int BX>
__global__ __launch_bounds__(256) void k_gate(Geo g, const double* __restrict__ K,
                                              const int8_t* __restrict__ bct,
                                              const double* __restrict__ beta,
                                              const int* __restrict__ slotseg, int R,
                                              const float* __restrict__ Y,
                                              const int* __restrict__ interior, double tau,
                                              double* __restrict__ Psi, int* __restrict__ fb,
                                              double* __restrict__ resid, int* __restrict__ flags) {
    __shared__ double cf[2 * (32 + 64)];
    __shared__ int rs[2 * (32 + 64)], of[2 * (32 + 64)];
    __shared__ double co[3 * BX * 64];      // per cell: diagonal, coupling right, coupling up
    __shared__ double ys[BX * 64];
    __shared__ double r2[256], e2[256];
    const int sub = blockIdx.x, tid = threadIdx.x;
    const int BY = g.by, n = BX * BY;
    if (!interior[sub]) {
        if (tid == 0) {
            fb[sub] = 0;
            resid[sub] = INFINITY;
        }
        return;
    }
    const int I = sub % g.mx, J = sub / g.mx;
    const int* ss = slotseg + (size_t)sub * R;
    face_prologue<BX>(g, K, bct, beta, ss, I, J, cf, rs, of);
    __syncthreads();
    for (int c = tid; c < n; c += 256) {
        double kv[5], dg, txr, tyu;
        load_kstencil<BX>(g, K, I, J, c % BX, c / BX, kv);
        stencil_coeffs<BX>(g, kv, cf, c % BX, c / BX, &dg, &txr, &tyu);
        co[3 * c] = dg;
        co[3 * c + 1] = txr;
        co[3 * c + 2] = tyu;
    }
    const float* Ys = Y + (size_t)sub * R * n;
    double worst = 0.0;
    for (int a = 0; a < R; ++a) {
        __syncthreads();
        for (int c = tid; c < n; c += 256) ys[c] = (double)Ys[(size_t)a * n + c];
        __syncthreads();
        double rr = 0.0, ee = 0.0;
        for (int c = tid; c < n; c += 256) {
            const int i = c % BX, j = c / BX;
            double v = co[3 * c] * ys[c];
            if (i > 0) v -= co[3 * (c - 1) + 1] * ys[c - 1];
            if (i < BX - 1) v -= co[3 * c + 1] * ys[c + 1];
            if (j > 0) v -= co[3 * (c - BX) + 2] * ys[c - BX];
            if (j < BY - 1) v -= co[3 * c + 2] * ys[c + BX];
            double e = 0.0;
            if (i == 0 && rs[j] == a) e += cf[j];
            if (i == BX - 1 && rs[BY + j] == a) e += cf[BY + j];
            if (j == 0 && rs[2 * BY + i] == a) e += cf[2 * BY + i];
            if (j == BY - 1 && rs[2 * BY + BX + i] == a) e += cf[2 * BY + BX + i];
            rr += (v - e) * (v - e);
            ee += e * e;
        }
        r2[tid] = rr;
        e2[tid] = ee;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) {
                r2[tid] += r2[tid + w];
                e2[tid] += e2[tid + w];
            }
            __syncthreads();
        }
        const double rel = e2[0] > 0.0 ? sqrt(r2[0] / e2[0]) : 0.0;
        worst = fmax(worst, rel);
    }
    const bool acc = worst <= tau;
    if (acc) {
        double* Ps = Psi + (size_t)sub * R * n;
        for (int t = tid; t < R * n; t += 256) Ps[t] = (double)Ys[t];
    }
    if (tid == 0) {
        fb[sub] = acc ? 2 : 0;
        resid[sub] = worst;
        if (acc) atomicAdd(&flags[FLAG_ACCEPTED], 1);
    }
}

template <int BX>
static hipError_t gate_bx(rmrcm_ctx* c, const float* Y, const int* interior, double tau) {
    const Level& L = c->levels[c->D];
    hipLaunchKernelGGL(k_gate<BX>, dim3(c->geo.mx * c->geo.my), dim3(256), 0, c->stream, c->geo, c->K,
                       c->bct, c->beta, L.slotseg, L.nslot, Y, interior, tau, c->Psi, c->fb, c->gres,
                       c->flags);
    return hipGetLastError();
}

hipError_t launch_gate(rmrcm_ctx* c, const float* Y, const int* interior, double tau) {
    if (c->geo.by > 64) return hipErrorInvalidValue;
    switch (c->geo.bx) {
        case 8: return gate_bx<8>(c, Y, interior, tau);
        case 16: return gate_bx<16>(c, Y, interior, tau);
        case 32: return gate_bx<32>(c, Y, interior, tau);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_features(rmrcm_ctx* c, float* x, int* interior) {
    if (c->geo.bx != c->geo.by) return hipErrorInvalidValue;
    const Level& L = c->levels[c->D];
    hipLaunchKernelGGL(k_features, dim3(c->geo.mx * c->geo.my), dim3(256), 0, c->stream, c->geo, c->K,
                       c->beta, L.slotseg, L.nslot, x, interior);
    return hipGetLastError();
}

hipError_t launch_mark_fallback(rmrcm_ctx* c, double tol) {
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL(k_mark_fallback, dim3((nsub + 255) / 256), dim3(256), 0, c->stream, nsub,
                       c->resid, tol, c->fb, c->flags, (const int*)c->irst);
    return hipGetLastError();
}

hipError_t launch_max_resid(rmrcm_ctx* c, int part) {
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL(k_max_resid, dim3(1), dim3(256), 0, c->stream, nsub, c->resid, c->fb, c->prm.ir_tol,
                       c->irst + 2 * part, c->irhist + kIrHist * part, kIrHist);
    return hipGetLastError();
}

hipError_t launch_mark_part_fallback(rmrcm_ctx* c) {
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL(k_mark_part_fallback, dim3((nsub + 255) / 256), dim3(256), 0, c->stream, nsub, c->resid,
                       c->prm.ir_tol, (const int*)c->fb, c->pfb, c->flags, (const int*)(c->irst + 2));
    return hipGetLastError();
}

}  // namespace rmrcm
