"""O-4: brute-force monolithic MRCM on tiny grids (oracle).

One dense linear system holds every fine cell pressure and every interface
unknown (U_e, P_e).  It is assembled face by face with plain loops from the
discrete variational formulation eq. 11.2-14.2 (Section 2) with the lumped
RT0 face laws, and shares no basis, trace or segment-table code with O-2,
O-3 or O-5: the segment of a skeleton face, the Robin parameter and the
sign n_i.n are all recomputed here from the grid.

Unknown order: p (cell j*nx+i), then U (documented segment order), then P.
Rows: one cell balance per cell, then eq. 14.2 and eq. 13.2 per segment.

Pinned by its role: it is the arbiter for every sign and convention of
O-3; on homogeneous vertical strips it reproduces the linear pressure.
"""

from __future__ import annotations

import numpy as np


def monolithic_solve(prob):
    nx, ny = prob.nx, prob.ny
    bx, by, sg = prob.sub_nx, prob.sub_ny, prob.seg
    mx, my = nx // bx, ny // by
    hx, hy = prob.lx / nx, prob.ly / ny
    K = prob.K
    nv = (mx - 1) * (ny // sg)
    nh = (my - 1) * (nx // sg)
    ns = nv + nh
    N = nx * ny

    def seg_of_face(i, j, d):
        """Segment id of the face of cell (i,j) in direction d (0W,1E,2S,3N)
        if that face lies on the skeleton, else -1; and the cell's sign."""
        if d == 1 and i + 1 < nx and (i + 1) % bx == 0:
            return ((i + 1) // bx - 1) * (ny // sg) + j // sg, +1
        if d == 0 and i > 0 and i % bx == 0:
            return (i // bx - 1) * (ny // sg) + j // sg, -1
        if d == 3 and j + 1 < ny and (j + 1) % by == 0:
            return nv + ((j + 1) // by - 1) * (nx // sg) + i // sg, +1
        if d == 2 and j > 0 and j % by == 0:
            return nv + (j // by - 1) * (nx // sg) + i // sg, -1
        return -1, 0

    def neighbour(i, j, d):
        di, dj = ((-1, 0), (1, 0), (0, -1), (0, 1))[d]
        return i + di, j + dj

    # Robin parameter per segment from the harmonic means of its faces.
    hsum = np.zeros(ns)
    hcnt = np.zeros(ns)
    length = np.zeros(ns)
    for j in range(ny):
        for i in range(nx):
            for d in (1, 3):
                e, s = seg_of_face(i, j, d)
                if e < 0:
                    continue
                a, b = neighbour(i, j, d)
                k1, k2 = K[j, i], K[b, a]
                hsum[e] += 2 * k1 * k2 / (k1 + k2)
                hcnt[e] += 1
                length[e] += hy if d == 1 else hx
    beta = prob.alpha * length / (hsum / np.maximum(hcnt, 1))

    M = np.zeros((N + 2 * ns, N + 2 * ns))
    rhs = np.zeros(N + 2 * ns)
    iU = lambda e: N + e          # noqa: E731
    iP = lambda e: N + ns + e     # noqa: E731
    for j in range(ny):
        for i in range(nx):
            c = j * nx + i
            rhs[c] += prob.q[j, i]
            for d in range(4):
                area = hy if d < 2 else hx
                rho_c = (hx if d < 2 else hy) / (2 * K[j, i])
                a, b = neighbour(i, j, d)
                e, s = seg_of_face(i, j, d)
                if 0 <= a < nx and 0 <= b < ny and e < 0:
                    rho_n = (hx if d < 2 else hy) / (2 * K[b, a])
                    t = area / (rho_c + rho_n)
                    M[c, c] += t
                    M[c, b * nx + a] -= t
                elif e >= 0:
                    # Robin face: F = cR (p_c - (P_e - beta_e s U_e))
                    cR = area / (rho_c + beta[e])
                    M[c, c] += cR
                    M[c, iP(e)] -= cR
                    M[c, iU(e)] += cR * beta[e] * s
                    # its share of the segment's trace F^i_e
                    # eq. 14.2 row e: beta_e (s F^i_e) ...
                    M[iU(e), c] += beta[e] * s * cR
                    M[iU(e), iP(e)] -= beta[e] * s * cR
                    M[iU(e), iU(e)] += beta[e] * s * cR * beta[e] * s
                    # eq. 13.2 row: F^i_e
                    M[iP(e), c] += cR
                    M[iP(e), iP(e)] -= cR
                    M[iP(e), iU(e)] += cR * beta[e] * s
                else:
                    f = (j if d == 0 else ny + j if d == 1 else
                         2 * ny + i if d == 2 else 2 * ny + nx + i)
                    if prob.bc_type[f] == 1:
                        cd = area / rho_c
                        M[c, c] += cd
                        rhs[c] += cd * prob.bc_value[f]
                    else:
                        rhs[c] -= prob.bc_value[f]
    for e in range(ns):
        M[iU(e), iU(e)] -= 2 * beta[e] * length[e]
    if not np.any(prob.bc_type == 1):
        # zero-mean gauge, bordered with the constant null vector
        Mb = np.zeros((N + 2 * ns + 1, N + 2 * ns + 1))
        Mb[:-1, :-1] = M
        Mb[:N, -1] = 1.0
        Mb[N + ns:N + 2 * ns, -1] = 0.0
        Mb[-1, :N] = 1.0
        sol = np.linalg.solve(Mb, np.concatenate([rhs, [0.0]]))[:-1]
    else:
        sol = np.linalg.solve(M, rhs)
    p = sol[:N].reshape(ny, nx)
    U = sol[N:N + ns]
    P = sol[N + ns:]
    # one-sided outward fluxes
    F = np.zeros((4, ny, nx))
    for j in range(ny):
        for i in range(nx):
            for d in range(4):
                area = hy if d < 2 else hx
                rho_c = (hx if d < 2 else hy) / (2 * K[j, i])
                a, b = neighbour(i, j, d)
                e, s = seg_of_face(i, j, d)
                if 0 <= a < nx and 0 <= b < ny and e < 0:
                    rho_n = (hx if d < 2 else hy) / (2 * K[b, a])
                    F[d, j, i] = area / (rho_c + rho_n) * (p[j, i] - p[b, a])
                elif e >= 0:
                    g = P[e] - beta[e] * s * U[e]
                    F[d, j, i] = area / (rho_c + beta[e]) * (p[j, i] - g)
                else:
                    f = (j if d == 0 else ny + j if d == 1 else
                         2 * ny + i if d == 2 else 2 * ny + nx + i)
                    if prob.bc_type[f] == 1:
                        F[d, j, i] = area / rho_c * (p[j, i] - prob.bc_value[f])
                    else:
                        F[d, j, i] = prob.bc_value[f]
    return p, F, U, P
