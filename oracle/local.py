"""O-2: local Robin problems on one subdomain (oracle).

The local problem is eq. 11.2-12.2 of Section 2 on subdomain i: the
lowest-order mixed system with, on every skeleton face, the Robin term
``(P_H - beta U_H n_i.n + beta u.n_i, v.n_i)``.  With the lumped mass a
Robin face of cell c in segment e carries the outward flux
``F = |f| (p_c - g_e) / (rho_c + beta_e)`` where
``g_e = P_e - beta_e (n_i.n) U_e`` is the Robin datum (the interface
unknowns enter the local problem only through it).

Additive split (Section 2.1, eq. addu/addp):
* basis column for slot a: unit Robin datum on that slot's segment, zero
  on the other slots, zero source and zero outer-boundary data (the P-type
  basis problem eq. 11Hhatbasisb with psi = 1 on the segment; the U-type
  problem eq. 11Hhatbasisa is the same with datum -beta (n_i.n));
* particular column: zero Robin data, the actual source and outer data.

Traces: ``T[a, b]`` is the outward integrated flux through the segment of
slot a when slot b carries the unit datum; ``tbar[a]`` the same for the
particular solution.  Inactive (outer-boundary) slots give zero rows and
columns.

Pinned by: a loop-by-loop dense assembly on tiny blocks, partition of
unity (all-ones Robin data reproduce p = 1 without source or Dirichlet
faces), the discrete maximum principle and the K -> cK invariance.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .tpfa import half_resistances, transmissibilities, block_matrix, solve_refined


@dataclass
class LocalResult:
    I: int
    J: int
    slots: list          # (segment id or -1, sign, side, s)
    Psi: np.ndarray      # (n, nslots) basis pressures, cell index j*bx + i
    pbar: np.ndarray     # (n,) particular pressure
    T: np.ndarray        # (nslots, nslots) traces of the basis
    tbar: np.ndarray     # (nslots,) traces of the particular solution
    robin_c: np.ndarray  # (by, bx, 4) Robin face conductances (0 where not Robin)
    ext_c: np.ndarray    # (by, bx, 4) Dirichlet conductance on outer faces
    tx: np.ndarray
    ty: np.ndarray


def _face_cells(side, s, sg, bx, by):
    """Local cells (i, j) of the faces of slot (side, s)."""
    t = np.arange(s * sg, (s + 1) * sg)
    if side == 0:
        return [(0, j) for j in t]
    if side == 1:
        return [(bx - 1, j) for j in t]
    if side == 2:
        return [(i, 0) for i in t]
    return [(i, by - 1) for i in t]


def local_solve(prob, dec, I, J, with_particular=True) -> LocalResult:
    bx, by, sg = dec.bx, dec.by, dec.sg
    hx, hy = dec.hx, dec.hy
    cs = dec.subdomain_cells(I, J)
    K = prob.K[cs]
    rx, ry = half_resistances(K, hx, hy)
    tx, ty = transmissibilities(K, hx, hy)
    slots = dec.subdomain_slots(I, J)
    ns = len(slots)
    n = bx * by
    diag = np.zeros((by, bx))
    robin_c = np.zeros((by, bx, 4))
    ext_c = np.zeros((by, bx, 4))
    B = np.zeros((n, ns))
    f = np.zeros(n)
    if with_particular:
        f += prob.q[cs].ravel()
    area = (hy, hy, hx, hx)
    rho = lambda side, i, j: rx[j, i] if side < 2 else ry[j, i]  # noqa: E731
    # skeleton (Robin) faces, slot by slot
    for a, (e, sign, side, s) in enumerate(slots):
        if e < 0:
            continue
        beta = dec.seg_beta[e]
        for (i, j) in _face_cells(side, s, sg, bx, by):
            c = area[side] / (rho(side, i, j) + beta)
            robin_c[j, i, side] = c
            diag[j, i] += c
            B[j * bx + i, a] += c
    # outer-boundary faces of this subdomain
    nx, ny = prob.nx, prob.ny
    gi0, gj0 = I * bx, J * by
    for side in range(4):
        if side == 0 and I != 0:
            continue
        if side == 1 and I != dec.mx - 1:
            continue
        if side == 2 and J != 0:
            continue
        if side == 3 and J != dec.my - 1:
            continue
        cells = ([(0, j) for j in range(by)] if side == 0 else
                 [(bx - 1, j) for j in range(by)] if side == 1 else
                 [(i, 0) for i in range(bx)] if side == 2 else
                 [(i, by - 1) for i in range(bx)])
        for (i, j) in cells:
            gi, gj = gi0 + i, gj0 + j
            fidx = (gj if side == 0 else ny + gj if side == 1 else
                    2 * ny + gi if side == 2 else 2 * ny + nx + gi)
            if prob.bc_type[fidx] == 1:
                c = area[side] / rho(side, i, j)
                ext_c[j, i, side] = c
                diag[j, i] += c
                if with_particular:
                    f[j * bx + i] += c * prob.bc_value[fidx]
            elif with_particular:
                f[j * bx + i] -= prob.bc_value[fidx]
    A = block_matrix(tx, ty, diag)
    X = solve_refined(A, np.column_stack([B, f]))
    Psi, pbar = X[:, :ns], X[:, ns]
    T = np.zeros((ns, ns))
    tbar = np.zeros(ns)
    for a, (e, sign, side, s) in enumerate(slots):
        if e < 0:
            continue
        for (i, j) in _face_cells(side, s, sg, bx, by):
            c = robin_c[j, i, side]
            idx = j * bx + i
            T[a, :] += c * Psi[idx, :]
            T[a, a] -= c
            tbar[a] += c * pbar[idx]
    for b, (e, *_r) in enumerate(slots):
        if e < 0:
            T[:, b] = 0.0
    return LocalResult(I, J, slots, Psi, pbar, T, tbar, robin_c, ext_c, tx, ty)


def local_fluxes(res: LocalResult, p, g_slots, prob, dec, homogeneous=False):
    """Outward integrated fluxes (4, by, bx) of a subdomain given its cell
    pressures and the Robin datum of every slot.  ``homogeneous`` takes the
    outer-boundary data as zero (basis functions)."""
    bx, by, sg = dec.bx, dec.by, dec.sg
    F = np.zeros((4, by, bx))
    tx, ty = res.tx, res.ty
    F[0][:, 1:] = tx * (p[:, 1:] - p[:, :-1])
    F[1][:, :-1] = tx * (p[:, :-1] - p[:, 1:])
    F[2][1:, :] = ty * (p[1:, :] - p[:-1, :])
    F[3][:-1, :] = ty * (p[:-1, :] - p[1:, :])
    for a, (e, sign, side, s) in enumerate(res.slots):
        if e < 0:
            continue
        for (i, j) in _face_cells(side, s, sg, bx, by):
            F[side, j, i] = res.robin_c[j, i, side] * (p[j, i] - g_slots[a])
    nx, ny = prob.nx, prob.ny
    gi0, gj0 = res.I * bx, res.J * by
    for side in range(4):
        if side == 0 and res.I != 0:
            continue
        if side == 1 and res.I != dec.mx - 1:
            continue
        if side == 2 and res.J != 0:
            continue
        if side == 3 and res.J != dec.my - 1:
            continue
        cells = ([(0, j) for j in range(by)] if side == 0 else
                 [(bx - 1, j) for j in range(by)] if side == 1 else
                 [(i, 0) for i in range(bx)] if side == 2 else
                 [(i, by - 1) for i in range(bx)])
        for (i, j) in cells:
            gi, gj = gi0 + i, gj0 + j
            fidx = (gj if side == 0 else ny + gj if side == 1 else
                    2 * ny + gi if side == 2 else 2 * ny + nx + gi)
            gval = 0.0 if homogeneous else prob.bc_value[fidx]
            if prob.bc_type[fidx] == 1:
                F[side, j, i] = res.ext_c[j, i, side] * (p[j, i] - gval)
            else:
                F[side, j, i] = gval
    return F
