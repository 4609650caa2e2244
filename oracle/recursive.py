"""O-5: Algorithm 1, the recursive MRCM (oracle).

Section 3: a nested binary hierarchy of decompositions (eq. dd.l, dd.2),
each subdomain of level l the union of two subdomains of level l+1 sharing
the interface gamma (eq. interface.1).  Algorithm 1 (RecMRCM) recurses to
the finest level, computes the multiscale basis functions (MMBFs) and the
particular solution there by the local mixed solver, and on the way back
solves, for every pair, the interface system eq. linsys restricted to
gamma, then forms the parent's MMBFs and particular solution as
combinations of the children's (eq. new_bfs, eq. particular).

Literal representation: every MMBF and particular solution is carried as a
full field (cell pressures and four one-sided outward face fluxes) over its
subdomain.  Interface degrees of freedom are the paper's: one U and one P
per segment (piecewise-constant MuMM spaces), with U-type basis problems
eq. 11Hhatbasisa (Robin datum -beta n_i.n) and P-type eq. 11Hhatbasisb
(Robin datum 1).

Reading of the garbled eq. new_bfs (the printed formula adds particular
solutions inside a basis function and attaches the boundary term to the
second child only): the parent MMBF for boundary DOF s is the MMBF for s
of the child whose boundary carries s, plus the sum over gamma DOFs k of
X_{k,s} times the children's MMBFs for k, each on its own child.  The
particular solution follows eq. particular as printed.  At level 0 the
particular solution of the whole domain is the answer.

The interface values of the final solution are recovered top-down from the
stored coefficients (the Remark of Section 3.2: track the combinations back
to the finest level).

Split rule: the side with more subdomains is cut first, x on ties (the
paper fixes only binary splits; the result does not depend on the order).
"""

from __future__ import annotations

import numpy as np

from .decomp import Decomposition
from .local import local_solve, local_fluxes


class _Node:
    def __init__(self, I0, I1, J0, J1):
        self.I0, self.I1, self.J0, self.J1 = I0, I1, J0, J1
        self.children = None
        self.cut = None


def _build_tree(I0, I1, J0, J1, order):
    node = _Node(I0, I1, J0, J1)
    nxs, nys = I1 - I0, J1 - J0
    if nxs * nys == 1:
        return node
    if order == "x-first":
        cut_x = nxs >= nys
    else:
        cut_x = nxs > nys or nys == 1
    if cut_x:
        Im = (I0 + I1) // 2
        node.cut = "x"
        node.children = (_build_tree(I0, Im, J0, J1, order), _build_tree(Im, I1, J0, J1, order))
    else:
        Jm = (J0 + J1) // 2
        node.cut = "y"
        node.children = (_build_tree(I0, I1, J0, Jm, order), _build_tree(I0, I1, Jm, J1, order))
    return node


def _node_segments(dec, node):
    """Active boundary segments of a node with the node's sign n_i.n."""
    segs = []
    for J in range(node.J0, node.J1):
        for s in range(dec.nsy):
            if node.I0 > 0:
                segs.append((dec.vseg(node.I0, J * dec.nsy + s), -1))
            if node.I1 < dec.mx:
                segs.append((dec.vseg(node.I1, J * dec.nsy + s), +1))
    for I in range(node.I0, node.I1):
        for s in range(dec.nsx):
            if node.J0 > 0:
                segs.append((dec.hseg(node.J0, I * dec.nsx + s), -1))
            if node.J1 < dec.my:
                segs.append((dec.hseg(node.J1, I * dec.nsx + s), +1))
    return segs


def _gamma_segments(dec, node):
    c1 = node.children[0]
    if node.cut == "x":
        return [dec.vseg(c1.I1, J * dec.nsy + s) for J in range(node.J0, node.J1)
                for s in range(dec.nsy)]
    return [dec.hseg(c1.J1, I * dec.nsx + s) for I in range(node.I0, node.I1)
            for s in range(dec.nsx)]


def _trace(dec, node, field_F, e, sign):
    """Integral over segment e of the node-outward normal flux of a field."""
    tot = 0.0
    cells = dec.seg_lo_cells[e] if sign > 0 else dec.seg_hi_cells[e]
    side = (1 if dec.seg_orient[e] == 0 else 3) if sign > 0 else (0 if dec.seg_orient[e] == 0 else 2)
    for (i, j) in cells:
        tot += field_F[side, j - node.J0 * dec.by, i - node.I0 * dec.bx]
    return tot


class RecursiveMRCM:
    def __init__(self, prob, order="x-first"):
        self.prob = prob
        self.dec = Decomposition(prob)
        self.root = _build_tree(0, self.dec.mx, 0, self.dec.my, order)

    # fields are (p (h, w), F (4, h, w)) over the node's cells
    def _leaf(self, node):
        dec, prob = self.dec, self.prob
        r = local_solve(prob, dec, node.I0, node.J0)
        ns = len(r.slots)
        dofs, fields = [], []
        for a, (e, sign, _side, _s) in enumerate(r.slots):
            if e < 0:
                continue
            for kind in ("U", "P"):
                datum = -dec.seg_beta[e] * sign if kind == "U" else 1.0
                g = np.zeros(ns)
                g[a] = datum
                p = (r.Psi[:, a] * datum).reshape(dec.by, dec.bx)
                F = local_fluxes(r, p, g, prob, dec, homogeneous=True)
                dofs.append((kind, e))
                fields.append((p, F))
        pbar = r.pbar.reshape(dec.by, dec.bx)
        Fbar = local_fluxes(r, pbar, np.zeros(ns), prob, dec)
        return dofs, fields, (pbar, Fbar)

    def _rec(self, node):
        """RecMRCM(node): returns (dofs, MMBF fields, particular field)."""
        if node.children is None:
            return self._leaf(node)
        dec = self.dec
        c1, c2 = node.children
        d1, f1, pb1 = self._rec(c1)
        d2, f2, pb2 = self._rec(c2)
        gam = _gamma_segments(dec, node)
        kdofs = [(k, e) for k in ("U", "P") for e in gam]          # xi DOFs
        kidx = {kd: n for n, kd in enumerate(kdofs)}
        xi = len(kdofs)
        kids = ((c1, d1, f1, pb1, +1), (c2, d2, f2, pb2, -1))      # gamma sign per child
        # traces on gamma of the children's gamma MMBFs
        A = np.zeros((xi, xi))
        for (c, dd, ff, pb, sg) in kids:
            didx = {kd: n for n, kd in enumerate(dd)}
            for kd in kdofs:
                p, F = ff[didx[kd]]
                col = kidx[kd]
                for r_i, e in enumerate(gam):
                    tr = _trace(dec, c, F, e, sg)
                    b = dec.seg_beta[e]
                    A[r_i, col] += b * sg * tr               # eq. 14.2 tested with phi^r
                    A[len(gam) + r_i, col] += tr             # eq. 13.2 tested with psi^r
        for r_i, e in enumerate(gam):
            A[r_i, kidx[("U", e)]] -= 2.0 * dec.seg_beta[e] * dec.seg_length[e]
        # parent DOFs: the children's boundary DOFs not on gamma
        gset = set(gam)
        pdofs = []
        for (c, dd, ff, pb, sg) in kids:
            for kd in dd:
                if kd[1] not in gset and kd not in pdofs:
                    pdofs.append(kd)
        ncol = len(pdofs) + 1
        rhs = np.zeros((xi, ncol))
        for (c, dd, ff, pb, sg) in kids:
            didx = {kd: n for n, kd in enumerate(dd)}
            for col in range(ncol):
                if col < len(pdofs):
                    if pdofs[col] not in didx:
                        continue
                    p, F = ff[didx[pdofs[col]]]
                else:
                    p, F = pb
                for r_i, e in enumerate(gam):
                    tr = _trace(dec, c, F, e, sg)
                    rhs[r_i, col] -= dec.seg_beta[e] * sg * tr
                    rhs[len(gam) + r_i, col] -= tr
        X = np.linalg.solve(A, rhs)
        node.X, node.kdofs, node.pdofs = X, kdofs, pdofs
        # combine: parent MMBFs (eq. new_bfs, reading above) and particular
        h = (node.J1 - node.J0) * dec.by
        w = (node.I1 - node.I0) * dec.bx
        out = []
        for col in range(ncol):
            P = np.zeros((h, w))
            Fp = np.zeros((4, h, w))
            for (c, dd, ff, pb, sg) in kids:
                didx = {kd: n for n, kd in enumerate(dd)}
                ys = slice((c.J0 - node.J0) * dec.by, (c.J1 - node.J0) * dec.by)
                xs = slice((c.I0 - node.I0) * dec.bx, (c.I1 - node.I0) * dec.bx)
                if col < len(pdofs):
                    if pdofs[col] in didx:
                        p0, F0 = ff[didx[pdofs[col]]]
                    else:
                        p0 = np.zeros(((c.J1 - c.J0) * dec.by, (c.I1 - c.I0) * dec.bx))
                        F0 = np.zeros((4,) + p0.shape)
                else:
                    p0, F0 = pb
                pc = p0.copy()
                Fc = F0.copy()
                for kd in kdofs:
                    x = X[kidx[kd], col]
                    pk, Fk = ff[didx[kd]]
                    pc += x * pk
                    Fc += x * Fk
                P[ys, xs] = pc
                Fp[:, ys, xs] = Fc
            out.append((P, Fp))
        return pdofs, out[:-1], out[-1]

    def solve(self):
        _dofs, _f, (p, F) = self._rec(self.root)
        U = np.zeros(self.dec.nseg)
        P = np.zeros(self.dec.nseg)
        self._down(self.root, {}, U, P)
        return p, F, U, P

    def _down(self, node, known, U, P):
        """Top-down recovery of the interface values from the coefficients."""
        if node.children is None:
            return
        vec = np.array([known[kd] for kd in node.pdofs] + [1.0])
        x = node.X @ vec
        vals = dict(known)
        for n, (k, e) in enumerate(node.kdofs):
            vals[(k, e)] = x[n]
            (U if k == "U" else P)[e] = x[n]
        for c in node.children:
            self._down(c, vals, U, P)


def recursive_solve(prob, order="x-first"):
    """Returns (p, F, U, P) of Algorithm 1."""
    return RecursiveMRCM(prob, order).solve()
