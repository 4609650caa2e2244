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

// Row coefficients of block row j: diagonal dg, x-couplings tx (i, i+1) and
// couplings dv to row j+1 (zero for the last row).
__device__ void row_coeffs(const Geo& g, const double* __restrict__ K, const int8_t* __restrict__ bct,
                           const double* __restrict__ beta, const int* __restrict__ ss, int I,
                           int J, int j, int BX, double* dg, double* tx, double* dv) {
    for (int i = threadIdx.x; i < BX; i += blockDim.x) {
        const int gi = I * BX + i, gj = J * g.by + j;
        int sl, of;
        double d = 0.0;
        d += i > 0 ? trans_x(K, g, gi - 1, gj) : bface(g, K, bct, beta, ss, I, J, i, j, 0, &sl, &of);
        const double txr = i < BX - 1 ? trans_x(K, g, gi, gj) : 0.0;
        d += i < BX - 1 ? txr : bface(g, K, bct, beta, ss, I, J, i, j, 1, &sl, &of);
        d += j > 0 ? trans_y(K, g, gi, gj - 1) : bface(g, K, bct, beta, ss, I, J, i, j, 2, &sl, &of);
        const double tyu = j < g.by - 1 ? trans_y(K, g, gi, gj) : 0.0;
        d += j < g.by - 1 ? tyu : bface(g, K, bct, beta, ss, I, J, i, j, 3, &sl, &of);
        dg[i] = d;
        tx[i] = txr;
        dv[i] = tyu;
    }
}

// Cholesky of the SPD block S (bx x bx, in the left half of Aug, bx x 2bx)
// fused with the inversion of its factor: row operations turn [S | I] into
// [L^T | L^{-1}].  Then Pm = L^{-T} L^{-1} = S^{-1}.
template <int BX>
__device__ void chol_inverse(double* Aug, double* mult, double* Pm, int* sing) {
    constexpr int W = 2 * BX;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int k = 0; k < BX; ++k) {
        __syncthreads();
        double piv = Aug[k * W + k];
        if (!(piv > 0.0)) {
            if (tid == 0) *sing = 1;
            piv = 1.0;
        }
        const double r = 1.0 / sqrt(piv);
        for (int t = tid; t < BX; t += nt)
            if (t > k) mult[t] = Aug[t * W + k] * r;
        __syncthreads();
        for (int t = tid; t < W; t += nt) Aug[k * W + t] *= r;
        __syncthreads();
        const int rows = BX - 1 - k;
        for (int idx = tid; idx < rows * W; idx += nt) {
            const int i = k + 1 + idx / W, c = idx % W;
            Aug[i * W + c] -= mult[i] * Aug[k * W + c];
        }
    }
    __syncthreads();
    // Pm[a][b] = sum_{i >= max(a,b)} Li[i][a] Li[i][b], Li = right half
    for (int idx = tid; idx < BX * BX; idx += nt) {
        const int a = idx / BX, b = idx % BX;
        const int i0 = a > b ? a : b;
        double s = 0.0;
        for (int i = i0; i < BX; ++i) s += Aug[i * W + BX + a] * Aug[i * W + BX + b];
        Pm[idx] = s;
    }
    __syncthreads();
}

// Right-hand side block of row j for the basis problems: unit Robin datum
// on one slot per column (column a = slot a).
template <int BX>
__device__ void basis_rhs_row(const Geo& g, const double* __restrict__ K, const int8_t* __restrict__ bct,
                              const double* __restrict__ beta, const int* __restrict__ ss, int I,
                              int J, int j, int R, double* F) {
    for (int t = threadIdx.x; t < BX * R; t += blockDim.x) F[t] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        int sl, of;
        double c = bface(g, K, bct, beta, ss, I, J, 0, j, 0, &sl, &of);
        if (sl >= 0) F[0 * R + sl] += c;
        c = bface(g, K, bct, beta, ss, I, J, BX - 1, j, 1, &sl, &of);
        if (sl >= 0) F[(BX - 1) * R + sl] += c;
    }
    __syncthreads();
    if (j == 0 || j == g.by - 1) {
        const int side = j == 0 ? 2 : 3;
        for (int i = threadIdx.x; i < BX; i += blockDim.x) {
            int sl, of;
            const double c = bface(g, K, bct, beta, ss, I, J, i, j, side, &sl, &of);
            if (sl >= 0) F[i * R + sl] += c;   // distinct (i, sl) per thread
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- K1
// Factor + basis solves.  One workgroup per subdomain.
template <int BX>
__global__ __launch_bounds__(256) void k_local_setup(Geo g, const double* __restrict__ K,
                                                     const int8_t* __restrict__ bct,
                                                     const double* __restrict__ beta,
                                                     const int* __restrict__ slotseg, int R,
                                                     double* __restrict__ Pstore,
                                                     double* __restrict__ Psi,
                                                     double* __restrict__ T, int ld,
                                                     int* __restrict__ flags) {
    extern __shared__ double sm[];
    constexpr int W = 2 * BX;
    double* Aug = sm;               // BX x 2BX
    double* Pm = Aug + BX * W;      // BX x BX
    double* Z = Pm + BX * BX;       // BX x R   (z_j, then x in the back sweep)
    double* Wb = Z + BX * R;        // BX x R   (w_j)
    double* mult = Wb + BX * R;     // BX
    double* dg = mult + BX;
    double* tx = dg + BX;
    double* dv = tx + BX;
    __shared__ int sing;

    const int sub = blockIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int BY = g.by;
    const int n = BX * BY;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int* ss = slotseg + (size_t)sub * R;
    double* Ps = Pstore + (size_t)sub * BY * BX * BX;
    double* Psub = Psi + (size_t)sub * R * n;
    if (tid == 0) sing = 0;

    // S_0 = A_00, z_0 = F_0
    row_coeffs(g, K, bct, beta, ss, I, J, 0, BX, dg, tx, dv);
    __syncthreads();
    for (int t = tid; t < BX * W; t += nt) {
        const int i = t / W, c = t % W;
        double v = 0.0;
        if (c < BX) {
            if (c == i) v = dg[i];
            else if (c == i + 1) v = -tx[i];
            else if (c == i - 1) v = -tx[c];
        } else {
            v = (c - BX == i) ? 1.0 : 0.0;
        }
        Aug[t] = v;
    }
    basis_rhs_row<BX>(g, K, bct, beta, ss, I, J, 0, R, Z);

    for (int j = 0; j < BY; ++j) {
        chol_inverse<BX>(Aug, mult, Pm, &sing);
        for (int t = tid; t < BX * BX; t += nt) Ps[(size_t)j * BX * BX + t] = Pm[t];
        // w_j = P_j z_j
        for (int t = tid; t < BX * R; t += nt) {
            const int i = t / R, a = t % R;
            double s = 0.0;
            for (int k = 0; k < BX; ++k) s += Pm[i * BX + k] * Z[k * R + a];
            Wb[t] = s;
            Psub[(size_t)a * n + j * BX + i] = s;
        }
        __syncthreads();
        if (j + 1 < BY) {
            // D_j: couplings between rows j and j+1 (dv from row j's coefficients)
            for (int t = tid; t < BX; t += nt) mult[t] = dv[t];
            __syncthreads();
            // next row coefficients; keep D_j in mult
            row_coeffs(g, K, bct, beta, ss, I, J, j + 1, BX, dg, tx, dv);
            __syncthreads();
            for (int t = tid; t < BX * W; t += nt) {
                const int i = t / W, c = t % W;
                double v;
                if (c < BX) {
                    v = -mult[i] * Pm[i * BX + c] * mult[c];
                    if (c == i) v += dg[i];
                    else if (c == i + 1) v -= tx[i];
                    else if (c == i - 1) v -= tx[c];
                } else {
                    v = (c - BX == i) ? 1.0 : 0.0;
                }
                Aug[t] = v;
            }
            basis_rhs_row<BX>(g, K, bct, beta, ss, I, J, j + 1, R, Z);
            for (int t = tid; t < BX * R; t += nt) Z[t] += mult[t / R] * Wb[t];
            __syncthreads();
        }
    }
    // back sweep: x_{BY-1} = w_{BY-1} (in Wb); x_j = w_j + P_j D_j x_{j+1}
    for (int t = tid; t < BX * R; t += nt) Z[t] = Wb[t];
    __syncthreads();
    for (int j = BY - 2; j >= 0; --j) {
        // D_j
        for (int i = tid; i < BX; i += nt)
            mult[i] = trans_y(K, g, I * BX + i, J * BY + j);
        for (int t = tid; t < BX * BX; t += nt) Pm[t] = Ps[(size_t)j * BX * BX + t];
        __syncthreads();
        for (int t = tid; t < BX * R; t += nt) Z[t] *= mult[t / R];
        __syncthreads();
        for (int t = tid; t < BX * R; t += nt) {
            const int i = t / R, a = t % R;
            double s = Psub[(size_t)a * n + j * BX + i];
            for (int k = 0; k < BX; ++k) s += Pm[i * BX + k] * Z[k * R + a];
            Wb[t] = s;
        }
        __syncthreads();
        for (int t = tid; t < BX * R; t += nt) {
            const int i = t / R, a = t % R;
            Z[t] = Wb[t];
            Psub[(size_t)a * n + j * BX + i] = Wb[t];
        }
        __syncthreads();
    }
    // traces T[a][b] = sum_{f in slot a} c_f (x_b(cell f) - delta_ab)
    double* Tsub = T + (size_t)sub * R * ld;
    for (int t = tid; t < R * R; t += nt) {
        const int a = t / R, b = t % R;
        double s = 0.0;
        if (ss[a] >= 0 && ss[b] >= 0) {
            int side, base;
            if (a < g.nsy) { side = 0; base = a; }
            else if (a < 2 * g.nsy) { side = 1; base = a - g.nsy; }
            else if (a < 2 * g.nsy + g.nsx) { side = 2; base = a - 2 * g.nsy; }
            else { side = 3; base = a - 2 * g.nsy - g.nsx; }
            for (int f = 0; f < g.sg; ++f) {
                const int pos = base * g.sg + f;
                const int i = side == 0 ? 0 : side == 1 ? BX - 1 : pos;
                const int j = side == 2 ? 0 : side == 3 ? BY - 1 : pos;
                int sl, of;
                const double c = bface(g, K, bct, beta, ss, I, J, i, j, side, &sl, &of);
                s += c * (Psub[(size_t)b * n + j * BX + i] - (a == b ? 1.0 : 0.0));
            }
        }
        Tsub[(size_t)a * ld + b] = s;
    }
    if (tid == 0 && sing) atomicOr(&flags[FLAG_LOCAL_SINGULAR], 1);
}

// ---------------------------------------------------------------- K1p
// Particular solution: the source and the outer boundary data with zero
// Robin data, solved with the stored P_j; writes pbar and the particular
// trace column.
template <int BX>
__global__ __launch_bounds__(64) void k_local_particular(
    Geo g, const double* __restrict__ K, const int8_t* __restrict__ bct,
    const double* __restrict__ beta, const int* __restrict__ slotseg, int R,
    const double* __restrict__ q, const double* __restrict__ bcv,
    const double* __restrict__ Pstore, double* __restrict__ pbar, double* __restrict__ T, int ld) {
    __shared__ double Pm[BX * BX];
    __shared__ double z[BX], w[BX], dprev[BX];
    const int sub = blockIdx.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int BY = g.by, n = BX * BY;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int* ss = slotseg + (size_t)sub * R;
    const double* Ps = Pstore + (size_t)sub * BY * BX * BX;
    double* pb = pbar + (size_t)sub * n;

    for (int i = tid; i < BX; i += nt) w[i] = 0.0, dprev[i] = 0.0;
    for (int j = 0; j < BY; ++j) {
        __syncthreads();
        for (int i = tid; i < BX; i += nt) {
            const int gi = I * BX + i, gj = J * BY + j;
            double f = q ? q[(size_t)gj * g.nx + gi] : 0.0;
            for (int side = 0; side < 4; ++side) {
                const bool on = side == 0 ? i == 0 : side == 1 ? i == BX - 1 : side == 2 ? j == 0 : j == BY - 1;
                if (!on) continue;
                int sl, of;
                const double c = bface(g, K, bct, beta, ss, I, J, i, j, side, &sl, &of);
                if (of >= 0) f += bct[of] == RMRCM_BC_DIRICHLET ? c * bcv[of] : -bcv[of];
            }
            z[i] = f + dprev[i] * w[i];
        }
        for (int t = tid; t < BX * BX; t += nt) Pm[t] = Ps[(size_t)j * BX * BX + t];
        __syncthreads();
        for (int i = tid; i < BX; i += nt) {
            double s = 0.0;
            for (int k = 0; k < BX; ++k) s += Pm[i * BX + k] * z[k];
            w[i] = s;
            pb[j * BX + i] = s;
            dprev[i] = j + 1 < BY ? trans_y(K, g, I * BX + i, J * BY + j) : 0.0;
        }
    }
    __syncthreads();
    for (int i = tid; i < BX; i += nt) z[i] = w[i];   // x_{BY-1}
    for (int j = BY - 2; j >= 0; --j) {
        __syncthreads();
        for (int i = tid; i < BX; i += nt) dprev[i] = trans_y(K, g, I * BX + i, J * BY + j) * z[i];
        for (int t = tid; t < BX * BX; t += nt) Pm[t] = Ps[(size_t)j * BX * BX + t];
        __syncthreads();
        for (int i = tid; i < BX; i += nt) {
            double s = pb[j * BX + i];
            for (int k = 0; k < BX; ++k) s += Pm[i * BX + k] * dprev[k];
            w[i] = s;
        }
        __syncthreads();
        for (int i = tid; i < BX; i += nt) {
            z[i] = w[i];
            pb[j * BX + i] = w[i];
        }
    }
    __syncthreads();
    double* Tsub = T + (size_t)sub * R * ld;
    for (int a = tid; a < R; a += nt) {
        double s = 0.0;
        if (ss[a] >= 0) {
            int side, base;
            if (a < g.nsy) { side = 0; base = a; }
            else if (a < 2 * g.nsy) { side = 1; base = a - g.nsy; }
            else if (a < 2 * g.nsy + g.nsx) { side = 2; base = a - 2 * g.nsy; }
            else { side = 3; base = a - 2 * g.nsy - g.nsx; }
            for (int f = 0; f < g.sg; ++f) {
                const int pos = base * g.sg + f;
                const int i = side == 0 ? 0 : side == 1 ? BX - 1 : pos;
                const int j = side == 2 ? 0 : side == 3 ? BY - 1 : pos;
                int sl, of;
                const double c = bface(g, K, bct, beta, ss, I, J, i, j, side, &sl, &of);
                s += c * pb[j * BX + i];
            }
        }
        Tsub[(size_t)a * ld + (ld - 1)] = s;
    }
}

// ---------------------------------------------------------------- launchers
template <int BX>
static hipError_t setup_bx(rmrcm_ctx* c) {
    const Level& L = c->levels[c->D];
    const int R = L.nslot;
    const size_t lds = sizeof(double) * (size_t)(BX * 2 * BX + BX * BX + 2 * BX * R + 4 * BX);
    hipError_t e = hipFuncSetAttribute((const void*)k_local_setup<BX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL(k_local_setup<BX>, dim3(nsub), dim3(256), lds, c->stream, c->geo, c->K,
                       c->bct, c->beta, L.slotseg, R, c->Pstore, c->Psi, L.T, L.ld, c->flags);
    return hipGetLastError();
}

template <int BX>
static hipError_t part_bx(rmrcm_ctx* c) {
    const Level& L = c->levels[c->D];
    const int nsub = c->geo.mx * c->geo.my;
    hipLaunchKernelGGL(k_local_particular<BX>, dim3(nsub), dim3(64), 0, c->stream, c->geo, c->K,
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
