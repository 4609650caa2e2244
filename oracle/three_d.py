"""O-6: the three-dimensional method (oracle; test infrastructure, imported
only by the tests, the smoke check and the benchmark's CPU baseline).

The paper's experiments are three-dimensional (Section 5): a box
[0, lx] x [0, ly] x [0, lz], the seven-point two-point-flux scheme (RT0 with
a lumped velocity mass on hexahedra), and a finest decomposition with no
division in z (Section 5.1), with Hbar_z = H_z: a skeleton segment is seg
fine faces along its interface line by the full height, and the
decomposition, its segments, slots and hierarchy are those of the 2D
method applied to the columns.  The Robin parameter of a segment is
alpha Hbar / Keff with Hbar its length along the interface (the z extent
being fixed) and Keff the mean over all of its fine faces of the harmonic
mean of the two adjacent permeabilities (the Robin-beta and
effective-permeability equations); the measure |e| in eq. 14.2 is the
segment's area.

Contents: ``fine_solve3d`` (the global fine solve), ``Decomposition3D``,
``local_solve3d`` (the local Robin problems eq. 11.2-12.2 with one basis per
segment side and the particular solution, their traces),
``mrcm_solve3d`` (the plain non-recursive method: the interface system of
oracle.mrcm on these traces, then the local solutions), and
``monolithic_solve3d`` (brute force on tiny grids: every cell pressure and
every (U, P) in one system assembled face by face from eq. 11.2-14.2 with
its own segment arithmetic).

Faces of a cell: 0 W (-x), 1 E (+x), 2 S (-y), 3 N (+y), 4 B (-z),
5 T (+z); fluxes are (6, nz, ny, nx) one-sided outward integrated fluxes.
Boundary data in the order of workloads.Problem3D.

Pinned by (tests/test_oracle_3d.py): the exactly linear pressure of a
homogeneous box with W/E Dirichlet data (fine and MRCM); with K, sources
and boundary data independent of z every layer carries the 2D solution
of the same columns (fine and MRCM, against the 2D oracle); nz = 1
reduces to the 2D oracle; O-6 MRCM = O-6 brute force on tiny grids
(Dirichlet, mixed, all-Neumann data, alpha over six decades); per-cell
conservation and eq. 13.2 / 14.2 on every segment.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mrcm import assemble_interface_system, robin_data, _gauge_row
from .tpfa import solve_refined


def spacing3d(prob):
    return prob.lx / prob.nx, prob.ly / prob.ny, prob.lz / prob.nz


def face_area(side, hx, hy, hz):
    return (hy * hz, hy * hz, hx * hz, hx * hz, hx * hy, hx * hy)[side]


def face_width(side, hx, hy, hz):
    """Cell width normal to the face (rho = width / (2 K))."""
    return (hx, hx, hy, hy, hz, hz)[side]


NEIGHBOUR = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))   # (di, dj, dk)


def outer_face_index(side, i, j, k, nx, ny, nz):
    """Index of an outer boundary face in the Problem3D layout."""
    if side == 0:
        return k * ny + j
    if side == 1:
        return ny * nz + k * ny + j
    if side == 2:
        return 2 * ny * nz + k * nx + i
    if side == 3:
        return 2 * ny * nz + nx * nz + k * nx + i
    if side == 4:
        return 2 * ny * nz + 2 * nx * nz + j * nx + i
    return 2 * ny * nz + 2 * nx * nz + nx * ny + j * nx + i


def box_matrix(K, hx, hy, hz, diag_extra):
    """Seven-point TPFA matrix of a (nz, ny, nx) box of cells, cell index
    (k * ny + j) * nx + i; diag_extra adds the boundary-face conductances."""
    nz, ny, nx = K.shape
    idx = np.arange(nz * ny * nx).reshape(nz, ny, nx)
    diag = diag_extra.astype(np.float64).copy()
    rows, cols, vals = [], [], []
    for axis, w, area in ((2, hx, hy * hz), (1, hy, hx * hz), (0, hz, hx * hy)):
        if K.shape[axis] < 2:
            continue
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        t = area / (w / (2.0 * K[lo]) + w / (2.0 * K[hi]))
        a, b = idx[lo].ravel(), idx[hi].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-t.ravel(), -t.ravel()]
        diag[lo] += t
        diag[hi] += t
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    n = nz * ny * nx
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def box_fluxes(K, p, hx, hy, hz):
    """Outward fluxes of the interior faces of a box (boundary faces 0)."""
    F = np.zeros((6,) + p.shape)
    for axis, w, area, s_lo, s_hi in ((2, hx, hy * hz, 1, 0), (1, hy, hx * hz, 3, 2), (0, hz, hx * hy, 5, 4)):
        if p.shape[axis] < 2:
            continue
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        t = area / (w / (2.0 * K[lo]) + w / (2.0 * K[hi]))
        f = t * (p[lo] - p[hi])
        F[s_lo][lo] = f
        F[s_hi][hi] = -f
    return F


def _outer_faces(nx, ny, nz, i0, i1, j0, j1):
    """(side, i, j, k) of the outer boundary faces of the cells of the
    column [i0, i1) x [j0, j1) (global indices)."""
    out = []
    for k in range(nz):
        for j in range(j0, j1):
            if i0 == 0:
                out.append((0, 0, j, k))
            if i1 == nx:
                out.append((1, nx - 1, j, k))
        for i in range(i0, i1):
            if j0 == 0:
                out.append((2, i, 0, k))
            if j1 == ny:
                out.append((3, i, ny - 1, k))
    for j in range(j0, j1):
        for i in range(i0, i1):
            out.append((4, i, j, 0))
            out.append((5, i, j, nz - 1))
    return out


def fine_solve3d(prob):
    """O-1 in 3D: the global fine solve.  Returns (p (nz, ny, nx), F)."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    hx, hy, hz = spacing3d(prob)
    K = prob.K
    diag = np.zeros((nz, ny, nx))
    rhs = prob.q.astype(np.float64).copy()
    faces = _outer_faces(nx, ny, nz, 0, nx, 0, ny)
    for (side, i, j, k) in faces:
        f = outer_face_index(side, i, j, k, nx, ny, nz)
        if prob.bc_type[f] == 1:
            c = face_area(side, hx, hy, hz) / (face_width(side, hx, hy, hz) / (2.0 * K[k, j, i]))
            diag[k, j, i] += c
            rhs[k, j, i] += c * prob.bc_value[f]
        else:
            rhs[k, j, i] -= prob.bc_value[f]
    A = box_matrix(K, hx, hy, hz, diag)
    n = nx * ny * nz
    if np.any(prob.bc_type == 1):
        p = solve_refined(A, rhs.ravel())
    else:
        ones = sp.csr_matrix(np.ones((n, 1)))
        Ab = sp.bmat([[A, ones], [ones.T, None]]).tocsr()
        p = solve_refined(Ab, np.concatenate([rhs.ravel(), [0.0]]))[:n]
    p = p.reshape(nz, ny, nx)
    F = box_fluxes(K, p, hx, hy, hz)
    for (side, i, j, k) in faces:
        f = outer_face_index(side, i, j, k, nx, ny, nz)
        if prob.bc_type[f] == 1:
            c = face_area(side, hx, hy, hz) / (face_width(side, hx, hy, hz) / (2.0 * K[k, j, i]))
            F[side, k, j, i] = c * (p[k, j, i] - prob.bc_value[f])
        else:
            F[side, k, j, i] = prob.bc_value[f]
    return p, F


class Decomposition3D:
    """Columns of sub_nx x sub_ny x nz cells; segments, slots, signs and
    their documented order as in the 2D decomposition (oracle.decomp), a
    segment covering seg faces along its line and every layer."""

    def __init__(self, prob):
        nx, ny, nz = prob.nx, prob.ny, prob.nz
        bx, by, sg = prob.sub_nx, prob.sub_ny, prob.seg
        if min(nx, ny, nz, bx, by, sg) <= 0 or nx % bx or ny % by or bx % sg or by % sg:
            raise ValueError("invalid geometry")
        self.nx, self.ny, self.nz, self.bx, self.by, self.sg = nx, ny, nz, bx, by, sg
        self.mx, self.my = nx // bx, ny // by
        if (self.mx & (self.mx - 1)) or (self.my & (self.my - 1)):
            raise ValueError("subdomain counts per direction must be powers of two")
        self.hx, self.hy, self.hz = spacing3d(prob)
        self.nsx, self.nsy = bx // sg, by // sg
        self.lines_v, self.lines_h = ny // sg, nx // sg
        self.nv = (self.mx - 1) * self.lines_v
        self.nseg = self.nv + (self.my - 1) * self.lines_h
        K = prob.K
        beta = np.zeros(self.nseg)
        area = np.zeros(self.nseg)
        for e in range(self.nseg):
            if e < self.nv:
                I, s = e // self.lines_v + 1, e % self.lines_v
                js = np.arange(s * sg, (s + 1) * sg)
                kl = K[:, js, I * bx - 1]
                kh = K[:, js, I * bx]
                hbar = sg * self.hy
                area[e] = sg * nz * self.hy * self.hz
            else:
                r = e - self.nv
                J, s = r // self.lines_h + 1, r % self.lines_h
                is_ = np.arange(s * sg, (s + 1) * sg)
                kl = K[:, J * by - 1, is_]
                kh = K[:, J * by, is_]
                hbar = sg * self.hx
                area[e] = sg * nz * self.hx * self.hz
            keff = np.mean(2.0 * kl * kh / (kl + kh))
            beta[e] = prob.alpha * hbar / keff
        self.seg_beta = beta
        self.seg_length = area
        # MuMM spaces: one U and one P per segment (the interface system of
        # oracle.mrcm reads these)
        self.nU = self.nP = self.nseg
        self.seg_useg = self.seg_pseg = np.arange(self.nseg)
        self.useg_beta = beta
        self.useg_length = area

    def vseg(self, I, k):
        return (I - 1) * self.lines_v + k

    def hseg(self, J, k):
        return self.nv + (J - 1) * self.lines_h + k

    def subdomain_slots(self, I, J):
        """(segment or -1, sign, side, s) for the W, E, S, N slots."""
        out = []
        for s in range(self.nsy):
            out.append((self.vseg(I, J * self.nsy + s) if I > 0 else -1, -1, 0, s))
        for s in range(self.nsy):
            out.append((self.vseg(I + 1, J * self.nsy + s) if I < self.mx - 1 else -1, +1, 1, s))
        for s in range(self.nsx):
            out.append((self.hseg(J, I * self.nsx + s) if J > 0 else -1, -1, 2, s))
        for s in range(self.nsx):
            out.append((self.hseg(J + 1, I * self.nsx + s) if J < self.my - 1 else -1, +1, 3, s))
        return out

    def slot_faces(self, side, s):
        """Local (i, j, k) of the cells behind the faces of slot (side, s)."""
        t = range(s * self.sg, (s + 1) * self.sg)
        if side == 0:
            return [(0, j, k) for k in range(self.nz) for j in t]
        if side == 1:
            return [(self.bx - 1, j, k) for k in range(self.nz) for j in t]
        if side == 2:
            return [(i, 0, k) for k in range(self.nz) for i in t]
        return [(i, self.by - 1, k) for k in range(self.nz) for i in t]


class Local3D:
    pass


def local_solve3d(prob, dec, I, J):
    """Local Robin problems of column (I, J): basis Psi (n x slots; cell
    index (k * by + j) * bx + i), particular pbar, traces T and tbar (as in
    oracle.local)."""
    bx, by, nz = dec.bx, dec.by, dec.nz
    hx, hy, hz = dec.hx, dec.hy, dec.hz
    K = prob.K[:, J * by:(J + 1) * by, I * bx:(I + 1) * bx]
    slots = dec.subdomain_slots(I, J)
    robin = np.zeros((6, nz, by, bx))
    extc = np.zeros((6, nz, by, bx))
    rhs_part = prob.q[:, J * by:(J + 1) * by, I * bx:(I + 1) * bx].astype(np.float64).copy()
    for (e, _sgn, side, s) in slots:
        if e < 0:
            continue
        for (i, j, k) in dec.slot_faces(side, s):
            rho = face_width(side, hx, hy, hz) / (2.0 * K[k, j, i])
            robin[side, k, j, i] = face_area(side, hx, hy, hz) / (rho + dec.seg_beta[e])
    for (side, gi, gj, k) in _outer_faces(prob.nx, prob.ny, nz, I * bx, (I + 1) * bx, J * by, (J + 1) * by):
        i, j = gi - I * bx, gj - J * by
        f = outer_face_index(side, gi, gj, k, prob.nx, prob.ny, nz)
        if prob.bc_type[f] == 1:
            c = face_area(side, hx, hy, hz) / (face_width(side, hx, hy, hz) / (2.0 * K[k, j, i]))
            extc[side, k, j, i] = c
            rhs_part[k, j, i] += c * prob.bc_value[f]
        else:
            rhs_part[k, j, i] -= prob.bc_value[f]
    A = box_matrix(K, hx, hy, hz, robin.sum(axis=0) + extc.sum(axis=0))
    n = nz * by * bx
    ns = len(slots)
    Psi = np.zeros((n, ns))
    for a, (e, _sgn, side, s) in enumerate(slots):
        if e < 0:
            continue
        b = np.zeros((nz, by, bx))
        for (i, j, k) in dec.slot_faces(side, s):
            b[k, j, i] += robin[side, k, j, i]
        Psi[:, a] = solve_refined(A, b.ravel())
    pbar = solve_refined(A, rhs_part.ravel())
    T = np.zeros((ns, ns))
    tbar = np.zeros(ns)
    for a, (e, _sgn, side, s) in enumerate(slots):
        if e < 0:
            continue
        for (i, j, k) in dec.slot_faces(side, s):
            c = robin[side, k, j, i]
            cell = (k * by + j) * bx + i
            for bb in range(ns):
                if slots[bb][0] >= 0:
                    T[a, bb] += c * (Psi[cell, bb] - (1.0 if bb == a else 0.0))
            tbar[a] += c * pbar[cell]
    r = Local3D()
    r.I, r.J, r.slots, r.Psi, r.pbar, r.T, r.tbar = I, J, slots, Psi, pbar, T, tbar
    r.robin, r.extc, r.K = robin, extc, K
    return r


def mrcm_solve3d(prob):
    """O-3 in 3D: returns (p, F, U, P, dec)."""
    dec = Decomposition3D(prob)
    loc = {(I, J): local_solve3d(prob, dec, I, J) for J in range(dec.my) for I in range(dec.mx)}
    ns = dec.nseg
    if ns == 0:
        U = P = np.zeros(0)
    else:
        A, b = assemble_interface_system(dec, loc)
        if np.any(prob.bc_type == 1):
            X = solve_refined(A, b)
        else:
            w, c0 = _gauge_row(prob, dec, loc)
            nullv = np.concatenate([np.zeros(ns), np.ones(ns)])
            Ab = sp.bmat([[A, sp.csr_matrix(nullv[:, None])], [sp.csr_matrix(w[None, :]), None]]).tocsr()
            X = solve_refined(Ab, np.concatenate([b, [-c0]]))[:2 * ns]
        U, P = X[:ns], X[ns:]
    bx, by, nz = dec.bx, dec.by, dec.nz
    p = np.zeros((nz, prob.ny, prob.nx))
    F = np.zeros((6, nz, prob.ny, prob.nx))
    for (I, J), r in loc.items():
        g = robin_data(r, U, P, dec)
        pl = (r.pbar + r.Psi @ g).reshape(nz, by, bx)
        Fl = box_fluxes(r.K, pl, dec.hx, dec.hy, dec.hz)
        for a, (e, _sgn, side, s) in enumerate(r.slots):
            if e < 0:
                continue
            for (i, j, k) in dec.slot_faces(side, s):
                Fl[side, k, j, i] = r.robin[side, k, j, i] * (pl[k, j, i] - g[a])
        for (side, gi, gj, k) in _outer_faces(prob.nx, prob.ny, nz, I * bx, (I + 1) * bx, J * by, (J + 1) * by):
            i, j = gi - I * bx, gj - J * by
            f = outer_face_index(side, gi, gj, k, prob.nx, prob.ny, nz)
            if prob.bc_type[f] == 1:
                Fl[side, k, j, i] = r.extc[side, k, j, i] * (pl[k, j, i] - prob.bc_value[f])
            else:
                Fl[side, k, j, i] = prob.bc_value[f]
        p[:, J * by:(J + 1) * by, I * bx:(I + 1) * bx] = pl
        F[:, :, J * by:(J + 1) * by, I * bx:(I + 1) * bx] = Fl
    return p, F, U, P, dec


def monolithic_solve3d(prob):
    """O-4 in 3D: cell pressures, U and P of every segment in one system,
    face by face (tiny grids).  Returns (p, F, U, P)."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    bx, by, sg = prob.sub_nx, prob.sub_ny, prob.seg
    mx, my = nx // bx, ny // by
    hx, hy, hz = spacing3d(prob)
    K = prob.K
    nv = (mx - 1) * (ny // sg)
    ns = nv + (my - 1) * (nx // sg)
    N = nx * ny * nz

    def seg_of_face(i, j, d):
        if d == 1 and i + 1 < nx and (i + 1) % bx == 0:
            return ((i + 1) // bx - 1) * (ny // sg) + j // sg, +1
        if d == 0 and i > 0 and i % bx == 0:
            return (i // bx - 1) * (ny // sg) + j // sg, -1
        if d == 3 and j + 1 < ny and (j + 1) % by == 0:
            return nv + ((j + 1) // by - 1) * (nx // sg) + i // sg, +1
        if d == 2 and j > 0 and j % by == 0:
            return nv + (j // by - 1) * (nx // sg) + i // sg, -1
        return -1, 0

    hsum = np.zeros(ns)
    cnt = np.zeros(ns)
    area = np.zeros(ns)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for d in (1, 3):
                    e, _s = seg_of_face(i, j, d)
                    if e < 0:
                        continue
                    di, dj, _dk = NEIGHBOUR[d]
                    k1, k2 = K[k, j, i], K[k, j + dj, i + di]
                    hsum[e] += 2 * k1 * k2 / (k1 + k2)
                    cnt[e] += 1
                    area[e] += face_area(d, hx, hy, hz)
    hbar = np.array([sg * (hy if e < nv else hx) for e in range(ns)])
    beta = prob.alpha * hbar / (hsum / np.maximum(cnt, 1))
    rows, cols, vals = [], [], []
    rhs = np.zeros(N + 2 * ns)

    def add(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    iU = lambda e: N + e         # noqa: E731
    iP = lambda e: N + ns + e    # noqa: E731
    cell = lambda i, j, k: (k * ny + j) * nx + i   # noqa: E731
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = cell(i, j, k)
                rhs[c] += prob.q[k, j, i]
                for d in range(6):
                    ar = face_area(d, hx, hy, hz)
                    rho = face_width(d, hx, hy, hz) / (2 * K[k, j, i])
                    di, dj, dk = NEIGHBOUR[d]
                    a, b, kk = i + di, j + dj, k + dk
                    inside = 0 <= a < nx and 0 <= b < ny and 0 <= kk < nz
                    e, s = seg_of_face(i, j, d) if d < 4 else (-1, 0)
                    if inside and e < 0:
                        t = ar / (rho + face_width(d, hx, hy, hz) / (2 * K[kk, b, a]))
                        add(c, c, t)
                        add(c, cell(a, b, kk), -t)
                    elif e >= 0:
                        cR = ar / (rho + beta[e])
                        add(c, c, cR)
                        add(c, iP(e), -cR)
                        add(c, iU(e), cR * beta[e] * s)
                        add(iU(e), c, beta[e] * s * cR)
                        add(iU(e), iP(e), -beta[e] * s * cR)
                        add(iU(e), iU(e), beta[e] * beta[e] * cR)
                        add(iP(e), c, cR)
                        add(iP(e), iP(e), -cR)
                        add(iP(e), iU(e), cR * beta[e] * s)
                    else:
                        f = outer_face_index(d, i, j, k, nx, ny, nz)
                        if prob.bc_type[f] == 1:
                            add(c, c, ar / rho)
                            rhs[c] += ar / rho * prob.bc_value[f]
                        else:
                            rhs[c] -= prob.bc_value[f]
    for e in range(ns):
        add(iU(e), iU(e), -2 * beta[e] * area[e])
    n = N + 2 * ns
    if not np.any(prob.bc_type == 1):
        for c in range(N):
            add(c, n, 1.0)
            add(n, c, 1.0)
        rhs = np.concatenate([rhs, [0.0]])
        n += 1
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsc()
    sol = solve_refined(A, rhs)[:N + 2 * ns]
    p = sol[:N].reshape(nz, ny, nx)
    U, P = sol[N:N + ns], sol[N + ns:]
    F = np.zeros((6, nz, ny, nx))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for d in range(6):
                    ar = face_area(d, hx, hy, hz)
                    rho = face_width(d, hx, hy, hz) / (2 * K[k, j, i])
                    di, dj, dk = NEIGHBOUR[d]
                    a, b, kk = i + di, j + dj, k + dk
                    inside = 0 <= a < nx and 0 <= b < ny and 0 <= kk < nz
                    e, s = seg_of_face(i, j, d) if d < 4 else (-1, 0)
                    if inside and e < 0:
                        t = ar / (rho + face_width(d, hx, hy, hz) / (2 * K[kk, b, a]))
                        F[d, k, j, i] = t * (p[k, j, i] - p[kk, b, a])
                    elif e >= 0:
                        F[d, k, j, i] = ar / (rho + beta[e]) * (p[k, j, i] - (P[e] - beta[e] * s * U[e]))
                    else:
                        f = outer_face_index(d, i, j, k, nx, ny, nz)
                        if prob.bc_type[f] == 1:
                            F[d, k, j, i] = ar / rho * (p[k, j, i] - prob.bc_value[f])
                        else:
                            F[d, k, j, i] = prob.bc_value[f]
    return p, F, U, P
