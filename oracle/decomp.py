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
* General interface spaces (Section 2 leaves U_H and P_H free; Section 4
  takes them equal): U_H piecewise constant on U-segments of ``seg_u``
  faces, P_H on P-segments of ``seg_p`` faces, the longer a multiple of the
  shorter.  The pieces of length ``min(seg_u, seg_p)`` are the segments
  above (slots, local solves, traces); every piece lies in one U-segment
  and one P-segment.  beta is that of the piece's U-segment (Hbar = the
  U-segment's length, Keff over its faces): it multiplies U_H in the Robin
  condition and weights eq. 14.2, both on U-segments.  With a constant
  beta on every piece, the datum of a subdomain's face is constant on each
  piece, so the U-type (eq. 11Hhatbasisa) and P-type (eq. 11Hhatbasisb)
  bases of a segment are sums of piece bases (the U-type one times
  ``-beta s``): one local solve per piece and side gives all of them.

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
        bx, by = prob.sub_nx, prob.sub_ny
        su = getattr(prob, "seg_u", 0) or prob.seg
        sp = getattr(prob, "seg_p", 0) or prob.seg
        sg = min(su, sp)
        if nx <= 0 or ny <= 0 or bx <= 0 or by <= 0 or sg <= 0:
            raise ValueError("sizes must be positive")
        if nx % bx or ny % by:
            raise ValueError("subdomain size must divide the grid")
        if bx % su or by % su or bx % sp or by % sp:
            raise ValueError("segment length must divide the subdomain size")
        if max(su, sp) % sg:
            raise ValueError("the longer interface segment must be a multiple of the shorter")
        self.seg_u_cells, self.seg_p_cells = su, sp
        self.mu, self.mp = su // sg, sp // sg      # pieces per U-segment, per P-segment
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
        # U- and P-segments: the same order as the pieces (vertical lines,
        # then horizontal ones), n_u / n_p per line
        self.nUv = (self.mx - 1) * (ny // su)
        self.nU = self.nUv + (self.my - 1) * (nx // su)
        self.nPv = (self.mx - 1) * (ny // sp)
        self.nP = self.nPv + (self.my - 1) * (nx // sp)
        # per-piece geometry: low/high cells of each fine face
        lo_cells, hi_cells, length = [], [], np.zeros(self.nseg)
        orient = np.zeros(self.nseg, dtype=int)
        useg = np.zeros(self.nseg, dtype=int)
        pseg = np.zeros(self.nseg, dtype=int)
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
                useg[e] = (I - 1) * (ny // su) + k // self.mu
                pseg[e] = (I - 1) * (ny // sp) + k // self.mp
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
                useg[e] = self.nUv + (J - 1) * (nx // su) + k // self.mu
                pseg[e] = self.nPv + (J - 1) * (nx // sp) + k // self.mp
            lo_cells.append(lo)
            hi_cells.append(hi)
        # beta per U-segment from all of its faces, then per piece
        hsum = np.zeros(self.nU)
        nfac = np.zeros(self.nU)
        ulen = np.zeros(self.nU)
        for e in range(self.nseg):
            kl = np.array([K[j, i] for (i, j) in lo_cells[e]])
            kh = np.array([K[j, i] for (i, j) in hi_cells[e]])
            hsum[useg[e]] += np.sum(2.0 * kl * kh / (kl + kh))
            nfac[useg[e]] += len(kl)
            ulen[useg[e]] += length[e]
        self.useg_beta = prob.alpha * ulen / (hsum / np.maximum(nfac, 1)) if self.nU else np.zeros(0)
        self.useg_length = ulen
        plen = np.zeros(self.nP)
        np.add.at(plen, pseg, length)
        self.pseg_length = plen
        self.seg_lo_cells = lo_cells
        self.seg_hi_cells = hi_cells
        self.seg_length = length
        self.seg_beta = self.useg_beta[useg] if self.nseg else np.zeros(0)
        self.seg_orient = orient
        self.seg_useg = useg
        self.seg_pseg = pseg

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
