"""O-1: the global fine-grid solve (oracle).

The reference solution the paper compares against is a single-domain mixed
solve on the fine grid (Section 5.4).  Here it is the lowest-order RT0 /
lumped-mass system of ``oracle.tpfa`` on the whole grid with the external
boundary data, solved directly (SuperLU) with one refinement step.  With
no Dirichlet face the pressure is fixed by a zero-mean gauge through a
bordered system (one Lagrange multiplier).

Pinned by: the exactly linear pressure for homogeneous and y-layered
permeability, and the 1D series-harmonic flux for x-layered permeability.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .tpfa import spacing, half_resistances, transmissibilities, block_matrix, solve_refined


def _boundary_terms(prob, rx, ry, hx, hy):
    """Diagonal additions and right-hand side from the outer boundary."""
    nx, ny = prob.nx, prob.ny
    diag = np.zeros((ny, nx))
    rhs = prob.q.astype(np.float64).copy()
    cond = np.zeros(2 * ny + 2 * nx)    # Dirichlet conductance per boundary face
    t, v = prob.bc_type, prob.bc_value
    for f in range(2 * ny + 2 * nx):
        if f < ny:
            i, j, area, rho = 0, f, hy, rx[f, 0]
        elif f < 2 * ny:
            i, j, area, rho = nx - 1, f - ny, hy, rx[f - ny, nx - 1]
        elif f < 2 * ny + nx:
            i, j, area, rho = f - 2 * ny, 0, hx, ry[0, f - 2 * ny]
        else:
            i, j, area, rho = f - 2 * ny - nx, ny - 1, hx, ry[ny - 1, f - 2 * ny - nx]
        if t[f] == 1:
            c = area / rho
            cond[f] = c
            diag[j, i] += c
            rhs[j, i] += c * v[f]
        else:
            rhs[j, i] -= v[f]
    return diag, rhs, cond


def fine_fluxes(prob, p, tx, ty, cond):
    """Outward integrated flux of every cell through its W, E, S, N faces."""
    nx, ny = prob.nx, prob.ny
    F = np.zeros((4, ny, nx))
    F[0][:, 1:] = tx * (p[:, 1:] - p[:, :-1])
    F[1][:, :-1] = tx * (p[:, :-1] - p[:, 1:])
    F[2][1:, :] = ty * (p[1:, :] - p[:-1, :])
    F[3][:-1, :] = ty * (p[:-1, :] - p[1:, :])
    t, v = prob.bc_type, prob.bc_value
    for f in range(2 * ny + 2 * nx):
        if f < ny:
            side, i, j = 0, 0, f
        elif f < 2 * ny:
            side, i, j = 1, nx - 1, f - ny
        elif f < 2 * ny + nx:
            side, i, j = 2, f - 2 * ny, 0
        else:
            side, i, j = 3, f - 2 * ny - nx, ny - 1
        F[side, j, i] = cond[f] * (p[j, i] - v[f]) if t[f] == 1 else v[f]
    return F


def fine_solve(prob):
    """Returns (p (ny, nx), F (4, ny, nx))."""
    hx, hy = spacing(prob.nx, prob.ny, prob.lx, prob.ly)
    rx, ry = half_resistances(prob.K, hx, hy)
    tx, ty = transmissibilities(prob.K, hx, hy)
    diag, rhs, cond = _boundary_terms(prob, rx, ry, hx, hy)
    A = block_matrix(tx, ty, diag)
    n = prob.nx * prob.ny
    if np.any(prob.bc_type == 1):
        p = solve_refined(A, rhs.ravel())
    else:
        ones = sp.csr_matrix(np.ones((n, 1)))
        Ab = sp.bmat([[A, ones], [ones.T, None]]).tocsr()
        sol = solve_refined(Ab, np.concatenate([rhs.ravel(), [0.0]]))
        p = sol[:n]
    p = p.reshape(prob.ny, prob.nx)
    return p, fine_fluxes(prob, p, tx, ty, cond)
