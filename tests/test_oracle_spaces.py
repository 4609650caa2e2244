"""Pins of the oracle's general MRCM interface spaces (Section 2: U_H and
P_H chosen apart; Section 4 takes them equal, the MuMM).

U_H is piecewise constant on U-segments of seg_u faces and P_H on
P-segments of seg_p faces, the longer a multiple of the shorter.  The
non-recursive oracle (oracle.mrcm) assembles the interface system from the
local bases of the pieces; the brute-force monolithic system
(oracle.monolithic) is assembled face by face from eq. 11.2-14.2 with its
own segment arithmetic.  Checked:

* the two agree for U coarser than P, P coarser than U, U on single faces,
  for Dirichlet, mixed and all-Neumann boundary data and alpha over six
  decades;
* the linear pressure on vertical strips (K constant on each longer
  segment) is reproduced exactly with distinct spaces;
* per-cell conservation, eq. 13.2 on every P-segment and eq. 14.2 on every
  U-segment; on a heterogeneous field the flux is NOT continuous on the
  finer pieces when P_H is coarser (the spaces are really distinct);
* the U-type basis problem eq. 11Hhatbasisa on a U-segment, solved
  directly, equals -beta s times the sum of the piece bases (the reading
  that one local solve per piece and side gives every basis function);
* the number of interface unknowns n_U + n_P.
"""

import numpy as np
import pytest

from helpers import make_problem
from oracle.decomp import Decomposition
from oracle.local import local_solve
from oracle.metrics import rel_l2, cell_balance, interface_residual
from oracle.monolithic import monolithic_solve
from oracle.mrcm import mrcm_solve
from oracle.tpfa import block_matrix, solve_refined
from workloads import Problem, dirichlet_we

SPACES = [(4, 2), (2, 4), (8, 2), (2, 8), (1, 4), (4, 1)]


@pytest.mark.parametrize("su,sp", SPACES)
@pytest.mark.parametrize("bc", ["we", "mixed", "fivespot"])
@pytest.mark.parametrize("alpha", [1e-3, 1.0, 1e3])
def test_general_spaces_match_brute_force(su, sp, bc, alpha):
    prob = make_problem(16, b=8, seg=2, log_var=2.0, alpha=alpha, bc=bc,
                        source=(bc != "fivespot"), seed=5).with_(seg_u=su, seg_p=sp)
    r = mrcm_solve(prob)
    p, F, U, P = monolithic_solve(prob)
    assert rel_l2(r.p, p) < 1e-11 and rel_l2(r.F, F) < 1e-11
    assert r.U.shape == U.shape and r.P.shape == P.shape
    assert rel_l2(r.U, U) < 1e-9
    # P is fixed to within the gauge's conditioning (large alpha, all-Neumann)
    assert rel_l2(r.P, P) < (1e-8 if alpha > 1 else 1e-11)


@pytest.mark.parametrize("su,sp", [(8, 2), (2, 8), (4, 4)])
@pytest.mark.parametrize("alpha", [0.1, 1.0, 100.0])
def test_general_spaces_vertical_strips_exactly_linear(su, sp, alpha):
    """K = K(y) constant on every longer segment: p = 1 - x has a constant
    face pressure and a flux constant on each U-segment, so it is in the
    discrete spaces and the method reproduces it."""
    nx, ny, L = 32, 16, max(su, sp)
    t, v = dirichlet_we(nx, ny)
    rng = np.random.default_rng(9)
    kseg = np.exp(rng.standard_normal(ny // L))
    K = np.repeat(np.repeat(kseg, L)[:, None], nx, axis=1)
    prob = Problem(nx=nx, ny=ny, K=K, q=np.zeros((ny, nx)), bc_type=t, bc_value=v,
                   sub_nx=8, sub_ny=16, seg=min(su, sp), alpha=alpha, seg_u=su, seg_p=sp)
    r = mrcm_solve(prob)
    xc = (np.arange(nx) + 0.5) / nx
    assert np.abs(r.p - (1 - xc)[None, :]).max() < 1e-12


def test_general_spaces_conservation_and_interface_equations():
    prob = make_problem(32, b=8, seg=2, log_var=3.0, source=True, bc="mixed").with_(seg_u=2, seg_p=8)
    r = mrcm_solve(prob)
    dec = r.dec
    assert cell_balance(r.F, prob.q) < 1e-12
    r13, r14 = interface_residual(dec, r.F, r.U)
    assert r13 < 1e-12 and r14 < 1e-12
    # continuity on the 2-face pieces fails: only P-segment sums vanish
    worst = 0.0
    for e in range(dec.nseg):
        vert = dec.seg_orient[e] == 0
        flo = sum(r.F[1 if vert else 3, j, i] for (i, j) in dec.seg_lo_cells[e])
        fhi = sum(r.F[0 if vert else 2, j, i] for (i, j) in dec.seg_hi_cells[e])
        worst = max(worst, abs(flo + fhi))
    assert worst > 1e-6 * np.abs(r.F).max()


def test_unknown_counts():
    prob = make_problem(32, b=8, seg=2).with_(seg_u=8, seg_p=2)
    dec = Decomposition(prob)
    # 3 vertical and 3 horizontal interface lines of 32 faces each
    assert dec.nseg == 6 * 16 and dec.nU == 6 * 4 and dec.nP == 6 * 16
    r = mrcm_solve(prob)
    assert r.U.size == dec.nU and r.P.size == dec.nP


@pytest.mark.parametrize("su,sp", [(8, 2), (2, 8)])
def test_u_basis_is_a_sum_of_piece_bases(su, sp):
    """Eq. 11Hhatbasisa with U_H = indicator of one U-segment and P_H = 0,
    solved directly on an interior subdomain: its Robin datum is -beta s on
    the U-segment's faces; its pressure equals -beta s times the sum of the
    basis columns of the segment's pieces.  The same for eq. 11Hhatbasisb
    on a P-segment (datum 1, the plain sum)."""
    prob = make_problem(32, b=8, seg=2, log_var=3.0, seed=13).with_(seg_u=su, seg_p=sp)
    dec = Decomposition(prob)
    I, J = 1, 2
    r = local_solve(prob, dec, I, J, with_particular=False)
    A = block_matrix(r.tx, r.ty, r.robin_c.sum(axis=2) + r.ext_c.sum(axis=2))
    n = dec.bx * dec.by
    for kind in ("U", "P"):
        target = dec.seg_useg if kind == "U" else dec.seg_pseg
        # the segment of the first E-side slot
        e0 = next(e for (e, sg, side, s) in r.slots if side == 1 and e >= 0)
        idx = target[e0]
        rhs = np.zeros(n)
        comb = np.zeros(n)
        for a, (e, sgn, side, s) in enumerate(r.slots):
            if e < 0 or target[e] != idx:
                continue
            datum = -dec.seg_beta[e] * sgn if kind == "U" else 1.0
            for t in range(s * dec.sg, (s + 1) * dec.sg):
                i, j = (0, t) if side == 0 else (dec.bx - 1, t) if side == 1 else (t, 0) if side == 2 else (t, dec.by - 1)
                rhs[j * dec.bx + i] += r.robin_c[j, i, side] * datum
            comb += datum * r.Psi[:, a]
        direct = solve_refined(A, rhs)
        assert np.abs(direct - comb).max() <= 1e-12 * np.abs(direct).max()
        npieces = dec.mu if kind == "U" else dec.mp
        assert sum(1 for (e, *_r) in r.slots if e >= 0 and target[e] == idx) == npieces
