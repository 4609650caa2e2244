"""Domain decomposition, skeleton segments and Robin parameter (oracle).

* Subdomains: a uniform ``mx x my`` array of ``sub_nx x sub_ny``-cell
  rectangles (the finest decomposition of Section 3.1; Section 4 requires
  each direction to be split into a power of two).
* Skeleton segments: each interface between two subdomains is cut into
  pieces of ``seg`` fine faces, the intermediate scale Hbar of Section 4.
  Interface spaces are piecewise constant on those pieces (the MuMM choice
  of Section 4 and Section 5.1).
* Global normal: the paper points it to the subdomain with the larger
  index (Section 2); here it points to +x on vertical segments and to +y on
  horizontal ones (a relabelling of the subdomains; the cell pressures and
  face fluxes do not depend on it, only the sign of U does).
* Robin parameter per segment: ``beta = alpha * Hbar / Keff`` with
  ``Keff`` the mean over the segment's fine faces of the harmonic mean of
  the two adjacent cell permeabilities (Section 5.1, the Robin-beta and
  effective-permeability equations; N read as the number of fine faces of
  the segment and Hbar as its physical length).

Documented global segment order: vertical segments first, by interface
line x = I*sub_nx*hx (I = 1..mx-1) and then bottom to top; then horizontal
segments by line y = J*sub_ny*hy (J = 1..my-1) and then left to right.

Subdomain slots: the boundary segments of a subdomain listed W (bottom to
top), E, S (left to right), N; a slot on the outer boundary is inactive
(segment id -1).  The slot's sign ``s = n_i . n`` is -1 on W and S (the
subdomain is on the high side of the segment) and +1 on E and N.
"""

from __future__ import annotations

import numpy as np

from .tpfa import spacing


def _is_pow2(v):
    return v > 0 and (v & (v - 1)) == 0


class Decomposition:
    def __init__(self, prob):
        nx, ny = prob.nx, prob.ny
        bx, by, sg = prob.sub_nx, prob.sub_ny, prob.seg
        if nx <= 0 or ny <= 0 or bx <= 0 or by <= 0 or sg <= 0:
            raise ValueError("sizes must be positive")
        if nx % bx or ny % by:
            raise ValueError("subdomain size must divide the grid")
        if bx % sg or by % sg:
            raise ValueError("segment length must divide the subdomain size")
        self.mx, self.my = nx // bx, ny // by
        if not (_is_pow2(self.mx) and _is_pow2(self.my)):
            raise ValueError("subdomain counts per direction must be powers of two")
        self.nx, self.ny, self.bx, self.by, self.sg = nx, ny, bx, by, sg
        self.hx, self.hy = spacing(nx, ny, prob.lx, prob.ly)
        self.nsx, self.nsy = bx // sg, by // sg          # segments per S/N side, W/E side
        self.lines_v = ny // sg                           # segments along one vertical line
        self.lines_h = nx // sg
        self.nv = (self.mx - 1) * self.lines_v
        self.nh = (self.my - 1) * self.lines_h
        self.nseg = self.nv + self.nh
        K = prob.K
        # per-segment geometry: low/high cells of each fine face
        lo_cells, hi_cells, length, beta = [], [], np.zeros(self.nseg), np.zeros(self.nseg)
        orient = np.zeros(self.nseg, dtype=int)
        for e in range(self.nseg):
            if e < self.nv:
                I = e // self.lines_v + 1
                k = e % self.lines_v
                i_lo, i_hi = I * bx - 1, I * bx
                js = np.arange(k * sg, (k + 1) * sg)
                lo = [(i_lo, j) for j in js]
                hi = [(i_hi, j) for j in js]
                length[e] = sg * self.hy
                orient[e] = 0
            else:
                r = e - self.nv
                J = r // self.lines_h + 1
                k = r % self.lines_h
                j_lo, j_hi = J * by - 1, J * by
                is_ = np.arange(k * sg, (k + 1) * sg)
                lo = [(i, j_lo) for i in is_]
                hi = [(i, j_hi) for i in is_]
                length[e] = sg * self.hx
                orient[e] = 1
            kl = np.array([K[j, i] for (i, j) in lo])
            kh = np.array([K[j, i] for (i, j) in hi])
            keff = np.mean(2.0 * kl * kh / (kl + kh))
            beta[e] = prob.alpha * length[e] / keff
            lo_cells.append(lo)
            hi_cells.append(hi)
        self.seg_lo_cells = lo_cells
        self.seg_hi_cells = hi_cells
        self.seg_length = length
        self.seg_beta = beta
        self.seg_orient = orient

    # ------------------------------------------------------------------
    def vseg(self, I, k):
        """Vertical segment on line I (1..mx-1), k-th from the bottom."""
        return (I - 1) * self.lines_v + k

    def hseg(self, J, k):
        return self.nv + (J - 1) * self.lines_h + k

    def subdomain_slots(self, I, J):
        """List of (segment id or -1, sign, side, s) for W, E, S, N slots."""
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

    def subdomain_cells(self, I, J):
        return (slice(J * self.by, (J + 1) * self.by), slice(I * self.bx, (I + 1) * self.bx))

    def count_local_solves(self):
        """Local solves at the finest level: one per (segment, side) plus one
        particular per subdomain (Section 4: one basis per Hbar piece when
        the U and P bases coincide; Table 3 counts)."""
        return 2 * self.nseg + self.mx * self.my
