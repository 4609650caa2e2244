"""O-4: brute-force monolithic MRCM on tiny grids (oracle).

One dense linear system holds every fine cell pressure and every interface
unknown (U_e, P_e).  It is assembled face by face with plain loops from the
discrete variational formulation eq. 11.2-14.2 (Section 2) with the lumped
RT0 face laws, and shares no basis, trace or segment-table code with O-2,
O-3 or O-5: the segment of a skeleton face, the Robin parameter and the
sign n_i.n are all recomputed here from the grid.

Unknown order: p (cell j*nx+i), then U (documented segment order), then P.
Rows: one cell balance per cell, then eq. 14.2 and eq. 13.2 per segment.
General interface spaces: U on U-segments of seg_u faces and P on
P-segments of seg_p faces (each recomputed here from the face position),
eq. 14.2 one row per U-segment, eq. 13.2 one per P-segment, beta per
U-segment.

The system is held sparse (entries summed per (row, column)) and solved by
SuperLU.  With ``ext_iters > 0`` the solution is refined that many times
with residuals computed in extended precision (numpy's long double), and
the fluxes formed in it: the exact solution of the same discrete system to
well below FP64 accuracy, which bounds what any FP64 solver of it reaches
when the system is ill conditioned (large alpha).

Pinned by its role: it is the arbiter for every sign and convention of
O-3; on homogeneous vertical strips it reproduces the linear pressure.
"""

from __future__ import annotations

from collections import defaultdict

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def monolithic_solve(prob, ext_iters=0):
    nx, ny = prob.nx, prob.ny
    bx, by = prob.sub_nx, prob.sub_ny
    su = getattr(prob, "seg_u", 0) or prob.seg
    sp_ = getattr(prob, "seg_p", 0) or prob.seg
    mx, my = nx // bx, ny // by
    hx, hy = prob.lx / nx, prob.ly / ny
    K = prob.K

    def counts(sg):
        nv = (mx - 1) * (ny // sg)
        return nv, nv + (my - 1) * (nx // sg)

    nvu, nsu = counts(su)
    nvp, nsp = counts(sp_)
    N = nx * ny

    def seg_id(i, j, d, sg, nv):
        """Segment (of length sg) of the face of cell (i,j) in direction d
        (0W,1E,2S,3N) if that face lies on the skeleton, else -1; and the
        cell's sign."""
        if d == 1 and i + 1 < nx and (i + 1) % bx == 0:
            return ((i + 1) // bx - 1) * (ny // sg) + j // sg, +1
        if d == 0 and i > 0 and i % bx == 0:
            return (i // bx - 1) * (ny // sg) + j // sg, -1
        if d == 3 and j + 1 < ny and (j + 1) % by == 0:
            return nv + ((j + 1) // by - 1) * (nx // sg) + i // sg, +1
        if d == 2 and j > 0 and j % by == 0:
            return nv + (j // by - 1) * (nx // sg) + i // sg, -1
        return -1, 0

    def seg_of_face(i, j, d):
        """(U-segment, P-segment, sign) of a skeleton face, (-1, -1, 0)
        elsewhere."""
        u, s = seg_id(i, j, d, su, nvu)
        q, _ = seg_id(i, j, d, sp_, nvp)
        return u, q, s

    def neighbour(i, j, d):
        di, dj = ((-1, 0), (1, 0), (0, -1), (0, 1))[d]
        return i + di, j + dj

    # Robin parameter per U-segment from the harmonic means of its faces.
    hsum = np.zeros(nsu)
    hcnt = np.zeros(nsu)
    length = np.zeros(nsu)
    for j in range(ny):
        for i in range(nx):
            for d in (1, 3):
                e, _q, s = seg_of_face(i, j, d)
                if e < 0:
                    continue
                a, b = neighbour(i, j, d)
                k1, k2 = K[j, i], K[b, a]
                hsum[e] += 2 * k1 * k2 / (k1 + k2)
                hcnt[e] += 1
                length[e] += hy if d == 1 else hx
    beta = prob.alpha * length / (hsum / np.maximum(hcnt, 1))

    nt = N + nsu + nsp
    M = defaultdict(float)
    rhs = np.zeros(nt)
    iU = lambda e: N + e          # noqa: E731
    iP = lambda q: N + nsu + q    # noqa: E731
    for j in range(ny):
        for i in range(nx):
            c = j * nx + i
            rhs[c] += prob.q[j, i]
            for d in range(4):
                area = hy if d < 2 else hx
                rho_c = (hx if d < 2 else hy) / (2 * K[j, i])
                a, b = neighbour(i, j, d)
                e, q, s = seg_of_face(i, j, d)
                if 0 <= a < nx and 0 <= b < ny and e < 0:
                    rho_n = (hx if d < 2 else hy) / (2 * K[b, a])
                    t = area / (rho_c + rho_n)
                    M[c, c] += t
                    M[c, b * nx + a] -= t
                elif e >= 0:
                    # Robin face: F = cR (p_c - (P_q - beta_e s U_e))
                    cR = area / (rho_c + beta[e])
                    M[c, c] += cR
                    M[c, iP(q)] -= cR
                    M[c, iU(e)] += cR * beta[e] * s
                    # its share of the segment's trace F^i_e
                    # eq. 14.2 row e: beta_e (s F^i_e) ...
                    M[iU(e), c] += beta[e] * s * cR
                    M[iU(e), iP(q)] -= beta[e] * s * cR
                    M[iU(e), iU(e)] += beta[e] * s * cR * beta[e] * s
                    # eq. 13.2 row q: F^i_e
                    M[iP(q), c] += cR
                    M[iP(q), iP(q)] -= cR
                    M[iP(q), iU(e)] += cR * beta[e] * s
                else:
                    f = (j if d == 0 else ny + j if d == 1 else
                         2 * ny + i if d == 2 else 2 * ny + nx + i)
                    if prob.bc_type[f] == 1:
                        cd = area / rho_c
                        M[c, c] += cd
                        rhs[c] += cd * prob.bc_value[f]
                    else:
                        rhs[c] -= prob.bc_value[f]
    for e in range(nsu):
        M[iU(e), iU(e)] -= 2 * beta[e] * length[e]
    n = nt
    if not np.any(prob.bc_type == 1):
        # zero-mean gauge, bordered with the constant null vector
        for c in range(N):
            M[c, nt] = 1.0
            M[nt, c] = 1.0
        rhs = np.concatenate([rhs, [0.0]])
        n = nt + 1
    keys = list(M.keys())
    A = sp.csc_matrix(([M[k] for k in keys], ([k[0] for k in keys], [k[1] for k in keys])), shape=(n, n))
    lu = spla.splu(A)
    sol = lu.solve(rhs)
    if ext_iters:
        Al = A.astype(np.longdouble)
        bl = rhs.astype(np.longdouble)
        sol = sol.astype(np.longdouble)
        for _ in range(ext_iters):
            r = bl - Al @ sol
            sol = sol + lu.solve(np.asarray(r, dtype=np.float64)).astype(np.longdouble)
        K = K.astype(np.longdouble)
        hx, hy = np.longdouble(prob.lx) / nx, np.longdouble(prob.ly) / ny
        beta = beta.astype(np.longdouble)
    sol = sol[:nt]
    p = sol[:N].reshape(ny, nx)
    U = sol[N:N + nsu]
    P = sol[N + nsu:]
    # one-sided outward fluxes
    F = np.zeros((4, ny, nx), dtype=sol.dtype)
    for j in range(ny):
        for i in range(nx):
            for d in range(4):
                area = hy if d < 2 else hx
                rho_c = (hx if d < 2 else hy) / (2 * K[j, i])
                a, b = neighbour(i, j, d)
                e, q, s = seg_of_face(i, j, d)
                if 0 <= a < nx and 0 <= b < ny and e < 0:
                    rho_n = (hx if d < 2 else hy) / (2 * K[b, a])
                    F[d, j, i] = area / (rho_c + rho_n) * (p[j, i] - p[b, a])
                elif e >= 0:
                    g = P[q] - beta[e] * s * U[e]
                    F[d, j, i] = area / (rho_c + beta[e]) * (p[j, i] - g)
                else:
                    f = (j if d == 0 else ny + j if d == 1 else
                         2 * ny + i if d == 2 else 2 * ny + nx + i)
                    if prob.bc_type[f] == 1:
                        F[d, j, i] = area / rho_c * (p[j, i] - prob.bc_value[f])
                    else:
                        F[d, j, i] = prob.bc_value[f]
    f64 = lambda a: np.asarray(a, dtype=np.float64)   # noqa: E731
    return f64(p), f64(F), f64(U), f64(P)
