"""Two-point flux discretisation on a uniform Cartesian grid (oracle).

Lowest-order Raviart-Thomas on rectangles with the trapezoidal (lumped)
velocity mass reduces to a pressure-only system (Section 2.1 says RT0 is
equivalent to a conservative cell-centred finite volume scheme; Section 4
says the local solver builds a linear system for the pressure variable).
With lumping, each face ``f`` of cell ``c`` carries a half-cell resistance
``rho = h_perp / (2 K_c)`` and the integrated outward flux through an
interior face between cells ``a`` and ``b`` is
``F = |f| (p_a - p_b) / (rho_a + rho_b)``.  A Dirichlet face adds
``F = |f| (p_c - g_D) / rho_c`` and a Robin face with data ``g`` and
parameter ``beta`` adds ``F = |f| (p_c - g) / (rho_c + beta)`` (from the
Robin term of eq. 11.2 tested with the face's velocity basis function).

Cell ``(i, j)`` of a ``w x h`` block has linear index ``j * w + i``.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def spacing(nx, ny, lx, ly):
    return lx / nx, ly / ny


def half_resistances(K, hx, hy):
    """rho for x-faces (normal width hx) and y-faces (normal width hy)."""
    return hx / (2.0 * K), hy / (2.0 * K)


def transmissibilities(K, hx, hy):
    """Interior face transmissibilities.

    tx[j, i] couples cells (i, j) and (i+1, j)  (area hy);
    ty[j, i] couples cells (i, j) and (i, j+1)  (area hx).
    """
    rx, ry = half_resistances(K, hx, hy)
    tx = hy / (rx[:, :-1] + rx[:, 1:])
    ty = hx / (ry[:-1, :] + ry[1:, :])
    return tx, ty


def block_matrix(tx, ty, diag_extra):
    """Assemble the SPD TPFA matrix of an h x w block of cells.

    ``tx`` (h, w-1) and ``ty`` (h-1, w) are the interior transmissibilities,
    ``diag_extra`` (h, w) the sum of boundary-face conductances of each cell.
    Returns a CSR matrix A with (A p)_c = sum over faces of outward flux
    (boundary data moved to the right-hand side).
    """
    h, w = diag_extra.shape
    n = h * w
    idx = np.arange(n).reshape(h, w)
    rows, cols, vals = [], [], []
    diag = diag_extra.astype(np.float64).copy()
    if w > 1:
        a = idx[:, :-1].ravel()
        b = idx[:, 1:].ravel()
        t = tx.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-t, -t]
        diag[:, :-1] += tx
        diag[:, 1:] += tx
    if h > 1:
        a = idx[:-1, :].ravel()
        b = idx[1:, :].ravel()
        t = ty.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-t, -t]
        diag[:-1, :] += ty
        diag[1:, :] += ty
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    return A


def solve_refined(A, B):
    """Sparse LU solve (SuperLU) of A X = B plus one step of iterative
    refinement in float64."""
    import scipy.sparse.linalg as spla
    lu = spla.splu(A.tocsc())
    X = lu.solve(B)
    R = B - A @ X
    X = X + lu.solve(R)
    return X


def boundary_faces(nx, ny):
    """Boundary faces in the documented order W(ny) E(ny) S(nx) N(nx).

    Returns arrays (i, j, side) with side 0=W, 1=E, 2=S, 3=N."""
    jj = np.arange(ny)
    ii = np.arange(nx)
    i = np.concatenate([np.zeros(ny, int), np.full(ny, nx - 1), ii, ii])
    j = np.concatenate([jj, jj, np.zeros(nx, int), np.full(nx, ny - 1)])
    side = np.concatenate([np.zeros(ny, int), np.ones(ny, int),
                           np.full(nx, 2), np.full(nx, 3)])
    return i, j, side
