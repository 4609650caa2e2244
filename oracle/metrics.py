"""Norms and residual checks used to pin results (oracle).

* ``rel_l2``             — ||a - b||_2 / ||b||_2 over all entries.
* ``cell_balance``       — per-cell mass conservation: the four outward
                           fluxes of a cell sum to its source (eq. 12.2 with
                           the lumped scheme), returned relative to the
                           largest flux.
* ``interface_residual`` — eq. 13.2 and eq. 14.2 evaluated on every segment
                           from one-sided fluxes and the interface values.
"""

from __future__ import annotations

import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    d = np.linalg.norm((a - b).ravel())
    return d / nb if nb > 0 else d


def cell_balance(F, q):
    s = F.sum(axis=0) - q
    scale = max(np.abs(F).max(), np.abs(q).max(), 1e-300)
    return np.abs(s).max() / scale


def cell_backward_error(prob, p, F):
    """Per-cell conservation residual |sum_f F_f - q_c| divided by the scale
    of the terms that cancel in it: (sum over the cell's faces of the full
    two-point conductance) * max|p| + |q_c|.  This is the cell-wise
    backward error of the balance; it stays near machine precision at any
    permeability contrast, while the residual relative to max|F| grows with
    the contrast."""
    K = prob.K
    hx, hy = prob.lx / prob.nx, prob.ly / prob.ny
    cx = hy / (hx / (2 * K))          # half-cell conductance of an x-face
    cy = hx / (hy / (2 * K))
    scale = (2 * cx + 2 * cy) * np.abs(p).max() + np.abs(prob.q)
    r = np.abs(F.sum(axis=0) - prob.q)
    return float((r / scale).max())


def interface_residual(dec, F, U):
    """Max relative residual of eq. 13.2 (tested with the indicator of
    every P-segment) and eq. 14.2 (divided by beta, with that of every
    U-segment; U holds one value per U-segment)."""
    r13 = np.zeros(dec.nP)
    r14 = np.zeros(dec.nU)
    for e in range(dec.nseg):
        vert = dec.seg_orient[e] == 0
        flo = sum(F[1 if vert else 3, j, i] for (i, j) in dec.seg_lo_cells[e])
        fhi = sum(F[0 if vert else 2, j, i] for (i, j) in dec.seg_hi_cells[e])
        r13[dec.seg_pseg[e]] += flo + fhi
        r14[dec.seg_useg[e]] += flo - fhi
    r14 -= 2.0 * dec.useg_length * U
    scale = max(np.abs(F).max(), 1e-300)
    return np.abs(r13).max() / scale, np.abs(r14).max() / scale
