"""Downscaling of the MRCM fluxes across the skeleton (oracle; test
infrastructure, imported only by the tests, smoke() and the benchmark's CPU
baseline).

The coarse interface conditions (eq. 13.2 and 14.2) hold on segments of
length Hbar, so the two one-sided fine fluxes through a skeleton face
differ and the velocity is conservative only at the Hbar scale; Section 4
leaves the recovery of fine-scale conservation to downscaling or smoothing
methods from the literature without fixing one.  The reading taken here is
a local Neumann post-processing:

1. each fine skeleton face between cell a (subdomain i) and cell b
   (subdomain k) gets the single flux ``Fbar_ab = (F_a - F_b) / 2``, the
   mean of a's outward flux and minus b's (so ``Fbar_ba = -Fbar_ab``); by
   eq. 13.2 its sum over a segment equals either side's segment flux;
2. on every subdomain the fine two-point problem is solved with the actual
   source and outer boundary data and the averaged fluxes prescribed on its
   skeleton faces (Neumann data);
3. a subdomain with no Dirichlet face has its pressure fixed up to a
   constant; the constant makes its mean cell pressure that of the input
   pressure (a bordered system with one multiplier, which also absorbs the
   round-off defect of the data's compatibility);
4. the result: the new cell pressures, interior fluxes from them, the
   averaged fluxes on skeleton faces, outer fluxes from the boundary data.

The output flux is single-valued on every face and conservative in every
cell.  Pinned by: a single-valued conservative input (the fine solution)
comes back unchanged; with one fine face per segment the MRCM solution
is the fine one, so its downscaling is too; idempotence; cell
conservation, single-valuedness, the segment flux sums and the subdomain
means of pure-Neumann subdomains (tests/test_oracle.py).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .decomp import Decomposition
from .tpfa import half_resistances, transmissibilities, block_matrix, solve_refined


def _outer_faces(prob, dec, I, J):
    """(side, i, j, face index) of the outer-boundary faces of a subdomain."""
    bx, by = dec.bx, dec.by
    nx, ny = prob.nx, prob.ny
    gi0, gj0 = I * bx, J * by
    out = []
    for side in range(4):
        if (side == 0 and I != 0) or (side == 1 and I != dec.mx - 1):
            continue
        if (side == 2 and J != 0) or (side == 3 and J != dec.my - 1):
            continue
        cells = ([(0, j) for j in range(by)] if side == 0 else
                 [(bx - 1, j) for j in range(by)] if side == 1 else
                 [(i, 0) for i in range(bx)] if side == 2 else
                 [(i, by - 1) for i in range(bx)])
        for (i, j) in cells:
            gi, gj = gi0 + i, gj0 + j
            fidx = (gj if side == 0 else ny + gj if side == 1 else
                    2 * ny + gi if side == 2 else 2 * ny + nx + gi)
            out.append((side, i, j, fidx))
    return out


def averaged_skeleton_flux(prob, dec, F):
    """(4, ny, nx): on every skeleton face the averaged outward flux of its
    cell (step 1); zero elsewhere."""
    bx, by = dec.bx, dec.by
    Fb = np.zeros_like(F)
    W, E, S, N = F
    # vertical subdomain lines: cells on the E side of one subdomain and on
    # the W side of the next
    for I in range(1, dec.mx):
        gi = I * bx                       # W-side cells of subdomain column I
        fab = 0.5 * (E[:, gi - 1] - W[:, gi])
        Fb[1][:, gi - 1] = fab
        Fb[0][:, gi] = -fab
    for J in range(1, dec.my):
        gj = J * by
        fab = 0.5 * (N[gj - 1, :] - S[gj, :])
        Fb[3][gj - 1, :] = fab
        Fb[2][gj, :] = -fab
    return Fb


def downscale(prob, p, F):
    """Steps 1-4 above for the pressure p (ny, nx) and one-sided outward
    fluxes F (4, ny, nx) of an MRCM solution on prob's decomposition.
    Returns the downscaled (p, F)."""
    dec = Decomposition(prob)
    bx, by = dec.bx, dec.by
    hx, hy = dec.hx, dec.hy
    area = (hy, hy, hx, hx)
    Fb = averaged_skeleton_flux(prob, dec, F)
    pd = np.zeros_like(p)
    Fd = np.zeros_like(F)
    for J in range(dec.my):
        for I in range(dec.mx):
            cs = dec.subdomain_cells(I, J)
            K = prob.K[cs]
            rx, ry = half_resistances(K, hx, hy)
            tx, ty = transmissibilities(K, hx, hy)
            diag = np.zeros((by, bx))
            f = prob.q[cs].ravel().astype(np.float64).copy()
            outer = _outer_faces(prob, dec, I, J)
            dirichlet = False
            for (side, i, j, fidx) in outer:
                if prob.bc_type[fidx] == 1:
                    c = area[side] / (rx[j, i] if side < 2 else ry[j, i])
                    diag[j, i] += c
                    f[j * bx + i] += c * prob.bc_value[fidx]
                    dirichlet = True
                else:
                    f[j * bx + i] -= prob.bc_value[fidx]
            # prescribed outward fluxes on the skeleton faces move to the
            # right-hand side
            fsk = Fb[(slice(None),) + cs]
            f -= fsk.sum(axis=0).ravel()
            A = block_matrix(tx, ty, diag)
            n = bx * by
            if dirichlet:
                pl = solve_refined(A, f)
            else:
                ones = np.ones((n, 1))
                Ab = sp.bmat([[A, sp.csr_matrix(ones)], [sp.csr_matrix(ones.T), None]]).tocsr()
                sol = solve_refined(Ab, np.concatenate([f, [p[cs].sum()]]))
                pl = sol[:n]
            pl = pl.reshape(by, bx)
            pd[cs] = pl
            Fl = np.zeros((4, by, bx))
            Fl[0][:, 1:] = tx * (pl[:, 1:] - pl[:, :-1])
            Fl[1][:, :-1] = tx * (pl[:, :-1] - pl[:, 1:])
            Fl[2][1:, :] = ty * (pl[1:, :] - pl[:-1, :])
            Fl[3][:-1, :] = ty * (pl[:-1, :] - pl[1:, :])
            # skeleton faces: the averaged fluxes (the subdomain's boundary
            # cells on sides that are not on the outer boundary)
            if I > 0:
                Fl[0][:, 0] = fsk[0][:, 0]
            if I < dec.mx - 1:
                Fl[1][:, bx - 1] = fsk[1][:, bx - 1]
            if J > 0:
                Fl[2][0, :] = fsk[2][0, :]
            if J < dec.my - 1:
                Fl[3][by - 1, :] = fsk[3][by - 1, :]
            for (side, i, j, fidx) in outer:
                if prob.bc_type[fidx] == 1:
                    c = area[side] / (rx[j, i] if side < 2 else ry[j, i])
                    Fl[side, j, i] = c * (pl[j, i] - prob.bc_value[fidx])
                else:
                    Fl[side, j, i] = prob.bc_value[fidx]
            Fd[(slice(None),) + cs] = Fl
    return pd, Fd
