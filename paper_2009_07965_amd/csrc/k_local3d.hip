// The three-dimensional method (Section 5: a box of nx x ny x nz cells,
// the seven-point two-point-flux scheme, a finest decomposition with no
// division in z and Hbar_z = H_z).  Every subdomain is a column of
// bx x by x nz cells; its skeleton faces are on its four sides, a segment
// covering sg faces along its line by the full height, so the slots, the
// traces and every merge are those of the 2D method.  Only the local
// problems and the reconstruction change.
//
// Local problem of a column (eq. 11.2-12.2 with the lumped velocity mass):
// cells ordered by rows j (the y index), row j being the x-z plane of
// NB = bx * nz cells, element r = k * bx + i.  The matrix is block
// tridiagonal in j: the plane operator A_j (x and z couplings, the y
// couplings' diagonal share, Robin and Dirichlet conductances) and the
// diagonal couplings D_j to row j + 1 (the y transmissibilities).  Block
// elimination with explicit inverses: S_0 = A_0, P_j = S_j^-1,
// S_{j+1} = A_{j+1} - D_j P_j D_j; forward y_0 = b_0,
// y_{j+1} = b_{j+1} + D_j P_j y_j; backward x_last = P_last y_last,
// x_j = P_j (y_j + D_j x_{j+1}).  One workgroup of 256 threads per column;
// S_j is inverted in LDS by Gauss-Jordan without pivoting (S_j is SPD);
// the inverses P_j are the factor store of later particular solves.
// Traces (the outward flux through each slot's faces per unit datum of
// each slot, and of the particular solution) are formed from the solution.

#include <algorithm>

#include "rmrcm_internal.h"

namespace rmrcm {

namespace {

typedef double v4m __attribute__((ext_vector_type(4)));

struct Face3 {
    int kind;      // 0 interior, 1 Robin (slot), 2 outer boundary
    int slot;      // local slot of a Robin face
    int of;        // boundary-face index of an outer face
    double cond;   // transmissibility, Robin |f| / (rho + beta), Dirichlet |f| / rho, 0 (Neumann)
};

__device__ inline double k3(const double* __restrict__ K, const Geo& g, int gi, int gj, int k) {
    return K[((size_t)k * g.ny + gj) * g.nx + gi];
}

// Face `side` (0 W, 1 E, 2 S, 3 N, 4 B, 5 T) of local cell (i, j, k) of
// column (I, J); ss: the column's slot codes.
__device__ inline Face3 face3(const Geo& g, const double* __restrict__ K, const int8_t* __restrict__ bct,
                              const double* __restrict__ beta, const int* __restrict__ ss, int I, int J, int i,
                              int j, int k, int side) {
    const int gi = I * g.bx + i, gj = J * g.by + j;
    int ni = gi, nj = gj, nk = k, of = -1;
    bool skel = false;
    double area, w;
    switch (side) {
        case 0:
            area = g.hy * g.hz, w = g.hx, ni = gi - 1;
            if (gi == 0) of = k * g.ny + gj;
            else skel = i == 0;
            break;
        case 1:
            area = g.hy * g.hz, w = g.hx, ni = gi + 1;
            if (gi == g.nx - 1) of = g.ny * g.nz + k * g.ny + gj;
            else skel = i == g.bx - 1;
            break;
        case 2:
            area = g.hx * g.hz, w = g.hy, nj = gj - 1;
            if (gj == 0) of = 2 * g.ny * g.nz + k * g.nx + gi;
            else skel = j == 0;
            break;
        case 3:
            area = g.hx * g.hz, w = g.hy, nj = gj + 1;
            if (gj == g.ny - 1) of = 2 * g.ny * g.nz + g.nx * g.nz + k * g.nx + gi;
            else skel = j == g.by - 1;
            break;
        case 4:
            area = g.hx * g.hy, w = g.hz, nk = k - 1;
            if (k == 0) of = 2 * g.ny * g.nz + 2 * g.nx * g.nz + gj * g.nx + gi;
            break;
        default:
            area = g.hx * g.hy, w = g.hz, nk = k + 1;
            if (k == g.nz - 1) of = 2 * g.ny * g.nz + 2 * g.nx * g.nz + g.nx * g.ny + gj * g.nx + gi;
            break;
    }
    const double rc = w / (2.0 * k3(K, g, gi, gj, k));
    Face3 f{0, -1, of, 0.0};
    if (of >= 0) {
        f.kind = 2;
        f.cond = bct[of] == RMRCM_BC_DIRICHLET ? area / rc : 0.0;
    } else if (skel) {
        const int a = side == 0 ? j / g.sg
                    : side == 1 ? g.nsy + j / g.sg
                    : side == 2 ? 2 * g.nsy + i / g.sg
                                : 2 * g.nsy + g.nsx + i / g.sg;
        f.kind = 1;
        f.slot = a;
        f.cond = area / (rc + beta[ss[a] >> 1]);
    } else {
        f.cond = area / (rc + w / (2.0 * k3(K, g, ni, nj, nk)));
    }
    return f;
}

__device__ inline size_t cell3(const Geo& g, int i, int j, int k) { return ((size_t)k * g.by + j) * g.bx + i; }

}  // namespace

// Doubles of the Z buffer: the products' output; between a row's products
// the face table of the row (6 NB conductances, 12 NB ints), then during
// the row's factorisation the Gauss-Jordan panels (two buffers of TS pivot
// rows and TS pivot columns of the padded block, NBP = 16 TS, and the
// inverted pivot block).
__host__ __device__ inline size_t local3d_zlen(int nb, int ncol) {
    const size_t ts = (size_t)(nb + 15) / 16, zl = (size_t)nb * (ncol > 12 ? ncol : 12);
    return zl > 66 * ts * ts ? zl : 66 * ts * ts;
}

__host__ __device__ inline size_t local3d_lds(int nb, int ncol) {
    return sizeof(double) *
           ((size_t)nb * (nb + 1) + (size_t)nb * ncol + local3d_zlen(nb, ncol) + 2 * (size_t)nb + 2);
}

// factor = 1: the factorisation (P_j to the factor store), the basis
// (basis = 1: one column per slot) and the particular solution (part = 1),
// with their traces.  factor = 0: the particular solution with the stored
// P_j, and its traces.  The block, padded with the identity to
// NBP = 16 TS rows, is held in registers during its factorisation: thread
// (tr, tc) of the 16 x 16 grid owns the TS x TS tile at rows TS tr.., columns
// TS tc..; each Gauss-Jordan pivot passes its row and column through LDS
// (double-buffered: one barrier per pivot).
template <int TS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_local3d(Geo g, const double* __restrict__ K,
                                                 const int8_t* __restrict__ bct,
                                                 const double* __restrict__ bcv,
                                                 const double* __restrict__ beta,
                                                 const int* __restrict__ slotseg, int R,
                                                 double* __restrict__ Pstore, double* __restrict__ Psi,
                                                 double* __restrict__ pbar, const double* __restrict__ q,
                                                 double* __restrict__ T, int ld, int* __restrict__ flags,
                                                 int factor, int basis, int part) {
    extern __shared__ double sm3[];
    const int sub = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int I = sub % g.mx, J = sub / g.mx;
    const int NB = g.bx * g.nz, BY = g.by, LS = NB + 1;
    const int nbas = basis ? R : 0, ncol = nbas + (part ? 1 : 0);
    const size_t n = (size_t)NB * BY;
    double* S = sm3;                       // NB x LS: S_j, then P_j
    double* Y = S + (size_t)NB * LS;       // NB x ncol
    double* Z = Y + (size_t)NB * ncol;     // NB x ncol
    constexpr int NBP = 16 * TS;
    double* dp = Z + local3d_zlen(NB, ncol);   // couplings D_{j-1}
    double* dn = dp + NB;                  // couplings D_j
    double* piv = dn + NB;                 // [1]: singular
    double* fc = Z;                        // [6][NB] face conductances of the current row (in Z
                                           // between the products)
    int* fk = reinterpret_cast<int*>(fc + 6 * NB);   // [6][NB] kind | slot << 2
    int* fo = fk + 6 * NB;                 // [6][NB] outer-face index
    const int tr = tid / 16, tc = tid % 16;
    double sv[TS][TS];                     // this thread's tile of S_j / P_j
    const int* ss = slotseg + (size_t)sub * R;
    double* Pst = Pstore + (size_t)sub * BY * NB * NB;
    // column c's value at local cell (i, j, k)
    auto col = [&](int c, size_t cell) -> double* {
        return c < nbas ? Psi + ((size_t)sub * R + c) * n + cell : pbar + (size_t)sub * n + cell;
    };
    if (tid == 0) piv[1] = 0.0;
    // Block products Out = Sm In (NB x NB times NB x ncol, row strides LS
    // and ncol): thread (tr, tc) forms rows tr + 16 u (u < TS) of columns
    // tc + 16 w below the last whole group of 16 columns, each In element
    // read once for its TS rows; each column beyond (the particular one of
    // 16 basis columns and it) is shared by all threads: thread (tr, tc)
    // sums the terms x = tc + 16 i of rows tr + 16 u, and the 16 lanes of
    // a thread row (consecutive in their wave) add their sums by shuffles.
    const int nmain = ncol & ~15;
    const int wv = tid >> 6, li = tid & 15, lk = (tid >> 4) & 3;   // matrix-core lane roles
    const int NKS = ((NB + 3) / 4 + 1) & ~1;                         // k-slices, even
    auto product = [&](const double* In, auto&& out) {
        for (int c = nmain; c < ncol; ++c) {
            double acc[TS];
#pragma unroll
            for (int u = 0; u < TS; ++u) acc[u] = 0.0;
            for (int x = tc; x < NB; x += 16) {
                const double y = In[x * ncol + c];
#pragma unroll
                for (int u = 0; u < TS; ++u) {
                    const int r = tr + 16 * u;
                    if (r < NB) acc[u] += S[r * LS + x] * y;
                }
            }
#pragma unroll
            for (int u = 0; u < TS; ++u) {
#pragma unroll
                for (int o = 8; o > 0; o >>= 1) acc[u] += __shfl_xor(acc[u], o, 16);
                const int r = tr + 16 * u;
                if (tc == 0 && r < NB) out(r, c, acc[u]);
            }
        }
        // the groups of 16 columns on the matrix cores (v_mfma_f64_16x16x4):
        // wave w forms row tile w, lane l = x + 16 k holding Sm[16 w + x][4 s + k]
        // (A operand) and In[4 s + k][16 t + x] (B operand) for k-slice s;
        // the result's lane l, register v is row 16 w + l / 16 + 4 v, column
        // 16 t + l % 16.  Two accumulators (even and odd k-slices) halve the
        // dependent chain.
        if (wv < TS) {
            const int r = 16 * wv + li;
            for (int ct = 0; ct < nmain / 16; ++ct) {
                const int cc = 16 * ct + li;
                v4m acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
                for (int ks = 0; ks < NKS; ks += 2) {
                    const int k0 = 4 * ks + lk, k1 = k0 + 4;
                    const double a0 = (r < NB && k0 < NB) ? S[r * LS + k0] : 0.0;
                    const double b0 = k0 < NB ? In[k0 * ncol + cc] : 0.0;
                    const double a1 = (r < NB && k1 < NB) ? S[r * LS + k1] : 0.0;
                    const double b1 = k1 < NB ? In[k1 * ncol + cc] : 0.0;
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ro = 16 * wv + lk + 4 * v;
                    if (ro < NB) out(ro, cc, acc0[v] + acc1[v]);
                }
            }
        }
    };
    // P_j from the factor store into S
    auto load_p = [&](int jr) {
        const double* src = Pst + (size_t)jr * NB * NB;
#pragma unroll
        for (int u = 0; u < TS; ++u)
#pragma unroll
            for (int v = 0; v < TS; ++v) {
                const int r = tr + 16 * u, c = tc + 16 * v;
                if (r < NB && c < NB) S[r * LS + c] = src[r * NB + c];
            }
    };
    // ---- forward: factorisation and y_j
    for (int j = 0; j < BY; ++j) {
        if (j > 0) {
            if (!factor) load_p(j - 1);
            __syncthreads();
            // D_{j-1} P_{j-1} y_{j-1}
            product(Y, [&](int r, int c, double v) { Z[r * ncol + c] = dp[r] * v; });
        }
        __syncthreads();
        // right-hand sides of row j: the coupled term, then each cell's
        // boundary faces (Robin faces of the basis columns, outer data and
        // the source of the particular column) by the cell's own thread;
        // D_j to the next row
        for (int e = tid; e < NB * ncol; e += nt) Y[e] = j > 0 ? Z[e] : 0.0;
        __syncthreads();
        // the faces of row j, one (cell, side) per thread
        for (int w = tid; w < 6 * NB; w += nt) {
            const int side = w / NB, r = w - side * NB, k = r / g.bx, i = r - k * g.bx;
            const Face3 f = face3(g, K, bct, beta, ss, I, J, i, j, k, side);
            fc[w] = f.cond;
            fk[w] = f.kind | (f.slot << 2);
            fo[w] = f.of;
        }
        __syncthreads();
        for (int r = tid; r < NB; r += nt) {
            double* yr = Y + r * ncol;
            if (j < BY - 1) dn[r] = fc[3 * NB + r];
            for (int side = 0; side < 6; ++side) {
                const int kd = fk[side * NB + r];
                if ((kd & 3) == 1) {
                    if ((kd >> 2) < nbas) yr[kd >> 2] += fc[side * NB + r];
                } else if ((kd & 3) == 2 && ncol > nbas) {
                    const int of = fo[side * NB + r];
                    yr[nbas] += bct[of] == RMRCM_BC_DIRICHLET ? fc[side * NB + r] * bcv[of] : -bcv[of];
                }
            }
            if (ncol > nbas && q) {
                const int k = r / g.bx, i = r - k * g.bx;
                yr[nbas] += q[((size_t)k * g.ny + J * BY + j) * g.nx + I * g.bx + i];
            }
        }
        __syncthreads();
        // y_j to the outputs (overwritten by x_j in the backward pass)
        for (int r = tr; r < NB; r += 16) {
            const int k = r / g.bx, i = r - k * g.bx;
            for (int c = tc; c < ncol; c += 16) *col(c, cell3(g, i, j, k)) = Y[r * ncol + c];
        }
        if (factor) {
            // A_j into LDS: zero, then each row's diagonal and x and z
            // couplings by its thread (P_{j-1} in S is no longer needed)
            for (int e = tid; e < NB * LS; e += nt) S[e] = 0.0;
            __syncthreads();
            for (int r = tid; r < NB; r += nt) {
                double d = 0.0;
                for (int side = 0; side < 6; ++side) {
                    const double cv = fc[side * NB + r];
                    d += cv;
                    if ((fk[side * NB + r] & 3) == 0 && side != 2 && side != 3) {
                        const int rc = side == 0 ? r - 1 : side == 1 ? r + 1 : side == 4 ? r - g.bx : r + g.bx;
                        S[r * LS + rc] = -cv;
                    }
                }
                S[r * LS + r] = d;
            }
            __syncthreads();
            // S_j = A_j - D_{j-1} P_{j-1} D_{j-1} on the tiles (P_{j-1} in the registers)
#pragma unroll
            for (int u = 0; u < TS; ++u)
#pragma unroll
                for (int v = 0; v < TS; ++v) {
                    const int r = TS * tr + u, c = TS * tc + v;
                    double a = r == c ? 1.0 : 0.0;
                    if (r < NB && c < NB) {
                        a = S[r * LS + c];
                        if (j > 0) a -= dp[r] * sv[u][v] * dp[c];
                    }
                    sv[u][v] = a;
                }
            // P_j = S_j^-1, block Gauss-Jordan without pivoting on the tiles:
            // step K takes the TS pivots of thread row K at once.  The
            // owners publish the pivot rows (thread row K) and columns
            // (thread column K) to LDS (the face table's buffer, dead by
            // now; two buffers: one barrier per step); the owner of the
            // diagonal tile inverts it in place (Gauss-Jordan, a pivot that
            // is not positive flagged) and publishes the inverse Q; then,
            // with R_J = Q S_KJ,
            //     S_IJ -= S_IK R_J,  S_KJ = R_J,  S_IK = -S_IK Q,  S_KK = Q.
            for (int K = 0; K < 16; ++K) {
                double* rp = Z + (size_t)(K & 1) * (2 * TS * NBP + TS * TS);   // TS x NBP: pivot rows
                double* cp = rp + TS * NBP;                                    // NBP x TS: pivot columns
                double* qb = cp + TS * NBP;                                    // TS x TS: Q
                if (tr == K) {
#pragma unroll
                    for (int u = 0; u < TS; ++u)
#pragma unroll
                        for (int v = 0; v < TS; ++v) rp[u * NBP + TS * tc + v] = sv[u][v];
                }
                if (tc == K) {
#pragma unroll
                    for (int u = 0; u < TS; ++u)
#pragma unroll
                        for (int v = 0; v < TS; ++v) cp[(TS * tr + u) * TS + v] = sv[u][v];
                }
                if (tr == K && tc == K) {
                    bool bad = false;
#pragma unroll
                    for (int k = 0; k < TS; ++k) {
                        double d = sv[k][k];
                        if (!(d > 0.0)) {
                            bad = true;
                            d = 1.0;
                        }
                        const double inv = 1.0 / d;
                        double rk[TS];
#pragma unroll
                        for (int v = 0; v < TS; ++v) rk[v] = sv[k][v] * inv;
#pragma unroll
                        for (int u = 0; u < TS; ++u) {
                            if (u == k) continue;
                            const double m = sv[u][k];
#pragma unroll
                            for (int v = 0; v < TS; ++v) sv[u][v] = fma(-m, rk[v], sv[u][v]);
                            sv[u][k] = -m * inv;
                        }
#pragma unroll
                        for (int v = 0; v < TS; ++v) sv[k][v] = rk[v];
                        sv[k][k] = inv;
                    }
                    if (bad) piv[1] = 1.0;
#pragma unroll
                    for (int u = 0; u < TS; ++u)
#pragma unroll
                        for (int v = 0; v < TS; ++v) qb[u * TS + v] = sv[u][v];
                }
                __syncthreads();
                if (tr == K && tc == K) {
                    // S_KK = Q, already in place
                } else if (tc == K) {
                    // S_IK = -S_IK Q, row by row
#pragma unroll
                    for (int u = 0; u < TS; ++u) {
                        double c[TS];
#pragma unroll
                        for (int w2 = 0; w2 < TS; ++w2) c[w2] = sv[u][w2];
#pragma unroll
                        for (int v = 0; v < TS; ++v) {
                            double acc = 0.0;
#pragma unroll
                            for (int w2 = 0; w2 < TS; ++w2) acc = fma(c[w2], qb[w2 * TS + v], acc);
                            sv[u][v] = -acc;
                        }
                    }
                } else {
                    // R_J = Q S_KJ one row at a time (S_KJ from the panel):
                    // the pivot rows take it, the others S_IJ -= S_IK R_J
#pragma unroll
                    for (int w2 = 0; w2 < TS; ++w2) {
                        double r[TS];
#pragma unroll
                        for (int v = 0; v < TS; ++v) {
                            double acc = 0.0;
#pragma unroll
                            for (int x = 0; x < TS; ++x) acc = fma(qb[w2 * TS + x], rp[x * NBP + TS * tc + v], acc);
                            r[v] = acc;
                        }
                        if (tr == K) {
#pragma unroll
                            for (int v = 0; v < TS; ++v) sv[w2][v] = r[v];
                        } else {
#pragma unroll
                            for (int u = 0; u < TS; ++u) {
                                const double ck = cp[(TS * tr + u) * TS + w2];
#pragma unroll
                                for (int v = 0; v < TS; ++v) sv[u][v] = fma(-ck, r[v], sv[u][v]);
                            }
                        }
                    }
                }
            }
            __syncthreads();
            // P_j to LDS (the products) and to the factor store
#pragma unroll
            for (int u = 0; u < TS; ++u)
#pragma unroll
                for (int v = 0; v < TS; ++v) {
                    const int r = TS * tr + u, c = TS * tc + v;
                    if (r < NB && c < NB) {
                        S[r * LS + c] = sv[u][v];
                        Pst[(size_t)j * NB * NB + r * NB + c] = sv[u][v];
                    }
                }
        }
        __syncthreads();
        for (int r = tid; r < NB; r += nt) dp[r] = dn[r];
        __syncthreads();
    }
    // ---- backward: x_last = P_last y_last; x_j = P_j (y_j + D_j x_{j+1})
    for (int j = BY - 1; j >= 0; --j) {
        if (!factor || j < BY - 1) load_p(j);
        if (j < BY - 1) {
            for (int r = tid; r < NB; r += nt) {
                const int k = r / g.bx, i = r - k * g.bx;
                dn[r] = face3(g, K, bct, beta, ss, I, J, i, j, k, 3).cond;
            }
            __syncthreads();
            for (int r = tr; r < NB; r += 16) {
                const int k = r / g.bx, i = r - k * g.bx;
                for (int c = tc; c < ncol; c += 16)
                    Z[r * ncol + c] = *col(c, cell3(g, i, j, k)) + dn[r] * Y[r * ncol + c];
            }
        } else {
            for (int e = tid; e < NB * ncol; e += nt) Z[e] = Y[e];
        }
        __syncthreads();
        product(Z, [&](int r, int c, double v) {
            Y[r * ncol + c] = v;
            const int k = r / g.bx;
            *col(c, cell3(g, r - k * g.bx, j, k)) = v;
        });
        __syncthreads();
    }
    if (tid == 0 && piv[1] != 0.0) atomicOr(&flags[FLAG_LOCAL_SINGULAR], 1);
    __threadfence_block();
    __syncthreads();
    // ---- traces: T[a][b] = sum over the faces f of slot a of c_f (x_b(f) - delta_ab)
    double* Ts = T + (size_t)sub * R * ld;
    const int nf = g.sg * g.nz;
    for (int e = tid; e < R * ncol; e += nt) {
        const int a = e / ncol, c = e % ncol;
        const int tc = c < nbas ? c : ld - 1;
        double s = 0.0;
        if (ss[a] >= 0 && (c >= nbas || ss[c] >= 0)) {
            const int side = a < g.nsy ? 0 : a < 2 * g.nsy ? 1 : a < 2 * g.nsy + g.nsx ? 2 : 3;
            const int s0 = (side == 0 ? a : side == 1 ? a - g.nsy : side == 2 ? a - 2 * g.nsy
                                                                             : a - 2 * g.nsy - g.nsx) * g.sg;
            for (int t = 0; t < nf; ++t) {
                const int k = t / g.sg, u = s0 + t % g.sg;
                const int i = side == 0 ? 0 : side == 1 ? g.bx - 1 : u;
                const int j = side == 2 ? 0 : side == 3 ? BY - 1 : u;
                const double cf = face3(g, K, bct, beta, ss, I, J, i, j, k, side).cond;
                s += cf * (*col(c, cell3(g, i, j, k)) - (c == a ? 1.0 : 0.0));
            }
        }
        Ts[(size_t)a * ld + tc] = s;
    }
}

// Pressures (pbar + sum_a Psi_a g_a) of every cell, then its six outward
// fluxes: interior faces by the two-point law, Robin faces c (p - g), outer
// faces from the boundary data.
__global__ __launch_bounds__(256) void k_recon3d_p(Geo g, int R, const int* __restrict__ slotseg,
                                                   const double* __restrict__ Psi,
                                                   const double* __restrict__ pbar,
                                                   const double* __restrict__ glo,
                                                   const double* __restrict__ ghi, double* __restrict__ p,
                                                   const int* __restrict__ run) {
    if (run && !*run) return;
    const size_t ncell = geo_ncell(g), n = (size_t)g.bx * g.by * g.nz;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell; t += (size_t)gridDim.x * blockDim.x) {
        const int gi = (int)(t % g.nx), gj = (int)((t / g.nx) % g.ny), k = (int)(t / ((size_t)g.nx * g.ny));
        const int I = gi / g.bx, J = gj / g.by, sub = J * g.mx + I;
        const size_t c = cell3(g, gi - I * g.bx, gj - J * g.by, k);
        const int* ss = slotseg + (size_t)sub * R;
        double v = pbar[(size_t)sub * n + c];
        for (int a = 0; a < R; ++a) {
            const int code = ss[a];
            if (code < 0) continue;
            const double d = (code & 1) ? glo[code >> 1] : ghi[code >> 1];
            v += Psi[((size_t)sub * R + a) * n + c] * d;
        }
        p[t] = v;
    }
}

__global__ __launch_bounds__(256) void k_recon3d_f(Geo g, const double* __restrict__ K,
                                                   const int8_t* __restrict__ bct,
                                                   const double* __restrict__ bcv,
                                                   const double* __restrict__ beta, int R,
                                                   const int* __restrict__ slotseg,
                                                   const double* __restrict__ glo,
                                                   const double* __restrict__ ghi,
                                                   const double* __restrict__ p, double* __restrict__ f,
                                                   const int* __restrict__ run) {
    if (run && !*run) return;
    const size_t ncell = geo_ncell(g);
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell; t += (size_t)gridDim.x * blockDim.x) {
        const int gi = (int)(t % g.nx), gj = (int)((t / g.nx) % g.ny), k = (int)(t / ((size_t)g.nx * g.ny));
        const int I = gi / g.bx, J = gj / g.by, sub = J * g.mx + I;
        const int* ss = slotseg + (size_t)sub * R;
        const double pc = p[t];
        for (int side = 0; side < 6; ++side) {
            const Face3 fc = face3(g, K, bct, beta, ss, I, J, gi - I * g.bx, gj - J * g.by, k, side);
            double v;
            if (fc.kind == 0) {
                const long long d = side == 0 ? -1 : side == 1 ? 1 : side == 2 ? -(long long)g.nx
                                  : side == 3 ? (long long)g.nx : side == 4 ? -(long long)g.nx * g.ny
                                                                          : (long long)g.nx * g.ny;
                v = fc.cond * (pc - p[t + d]);
            } else if (fc.kind == 1) {
                const int code = ss[fc.slot];
                const double gd = (code & 1) ? glo[code >> 1] : ghi[code >> 1];
                v = fc.cond * (pc - gd);
            } else {
                v = bct[fc.of] == RMRCM_BC_DIRICHLET ? fc.cond * (pc - bcv[fc.of]) : bcv[fc.of];
            }
            f[side * ncell + t] = v;
        }
    }
}

template <int TS>
static hipError_t local3d_ts(rmrcm_ctx* c, int factor, int basis, int part) {
    const Level& L = c->levels[c->D];
    const int NB = c->geo.bx * c->geo.nz, ncol = (basis ? L.nslot : 0) + (part ? 1 : 0);
    const size_t lds = local3d_lds(NB, ncol);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e =
        hipFuncSetAttribute((const void*)k_local3d<TS>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_local3d<TS>, dim3(c->geo.mx * c->geo.my), dim3(256), lds, c->stream, c->geo, c->K,
                       c->bct, c->bcv, c->beta, L.slotseg, L.nslot, c->Pstore, c->Psi, c->pbar, c->q, L.T, L.ld,
                       c->flags, factor, basis, part);
    return hipGetLastError();
}

hipError_t launch_local3d(rmrcm_ctx* c, int factor, int basis, int part) {
    switch ((c->geo.bx * c->geo.nz + 15) / 16) {
        case 1: return local3d_ts<1>(c, factor, basis, part);
        case 2: return local3d_ts<2>(c, factor, basis, part);
        case 3: return local3d_ts<3>(c, factor, basis, part);
        case 4: return local3d_ts<4>(c, factor, basis, part);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_reconstruct3d(rmrcm_ctx* c) {
    const Level& L = c->levels[c->D];
    const size_t ncell = geo_ncell(c->geo);
    const unsigned nb = (unsigned)std::min<size_t>((ncell + 255) / 256, 8192);
    hipLaunchKernelGGL(k_recon3d_p, dim3(nb), dim3(256), 0, c->stream, c->geo, L.nslot, L.slotseg, c->Psi, c->pbar,
                       c->glo, c->ghi, c->pout, c->run_ptr);
    hipLaunchKernelGGL(k_recon3d_f, dim3(nb), dim3(256), 0, c->stream, c->geo, c->K, c->bct, c->bcv, c->beta,
                       L.nslot, L.slotseg, c->glo, c->ghi, c->pout, c->fout, c->run_ptr);
    return hipGetLastError();
}

}  // namespace rmrcm
