"""Pins of the downscaling oracle (oracle/downscale.py): local Neumann
solves with the averaged skeleton fluxes, recovering a single-valued,
cell-conservative flux from the MRCM solution (Section 4 leaves the method
open; the reading is stated in the oracle's header)."""

import numpy as np
import pytest

from helpers import make_problem
from oracle.decomp import Decomposition
from oracle.downscale import downscale, averaged_skeleton_flux
from oracle.fine import fine_solve
from oracle.metrics import rel_l2, cell_backward_error
from oracle.mrcm import mrcm_solve


def opposite_flux_defect(F):
    """max over interior faces of |F_out(a) + F_out(b)| / max|F|: zero for a
    single-valued flux."""
    W, E, S, N = F
    d = max(np.abs(E[:, :-1] + W[:, 1:]).max(), np.abs(N[:-1, :] + S[1:, :]).max())
    return d / np.abs(F).max()


CASES = {
    "grf_b4_seg2": dict(nx=32, b=8, seg=2, log_var=3.0, lam=0.1, seed=5),
    "grf_source_rect": dict(nx=32, ny=64, b=8, by=16, seg=4, log_var=2.0, source=True, seed=8),
    "mixed_bc": dict(nx=32, b=8, seg=4, bc="mixed", log_var=2.0, seed=9),
    "fivespot": dict(nx=32, b=8, seg=4, bc="fivespot", log_var=2.0, seed=10),
    "high_contrast_alpha": dict(nx=32, b=8, seg=8, log_var=6.0, lam=0.05, alpha=1e3, seed=12),
}


def problem(name):
    kw = dict(CASES[name])
    nx = kw.pop("nx")
    return make_problem(nx, **kw)


def test_fine_solution_is_a_fixed_point():
    """A single-valued, conservative input (the fine solution) satisfies
    every local Neumann problem with its own fluxes and has the right
    subdomain means: it comes back unchanged (a dropped source, boundary or
    skeleton term, a sign of the average or a wrong gauge breaks this)."""
    for name in CASES:
        prob = problem(name)
        pf, Ff = fine_solve(prob)
        pd, Fd = downscale(prob, pf, Ff)
        assert rel_l2(pd, pf) < 1e-11, name
        assert rel_l2(Fd, Ff) < 1e-11, name


@pytest.mark.parametrize("alpha", [1e-2, 1.0, 1e3])
def test_one_face_segments_give_the_fine_solution(alpha):
    """With one fine face per segment the MRCM solution is the fine one
    (pinned separately), so its downscaling is too."""
    prob = make_problem(32, b=8, seg=1, log_var=3.0, lam=0.1, alpha=alpha, seed=21, source=True)
    m = mrcm_solve(prob)
    pf, Ff = fine_solve(prob)
    pd, Fd = downscale(prob, m.p, m.F)
    assert rel_l2(pd, pf) < 1e-10 and rel_l2(Fd, Ff) < 1e-10


@pytest.mark.parametrize("name", sorted(CASES))
def test_conservative_single_valued_idempotent(name):
    prob = problem(name)
    m = mrcm_solve(prob)
    assert opposite_flux_defect(m.F) > 1e-6          # the MRCM flux is two-valued
    pd, Fd = downscale(prob, m.p, m.F)
    assert opposite_flux_defect(Fd) < 1e-13
    assert cell_backward_error(prob, pd, Fd) < 1e-12
    # the downscaled solution is a fixed point
    p2, F2 = downscale(prob, pd, Fd)
    assert rel_l2(p2, pd) < 1e-12 and rel_l2(F2, Fd) < 1e-12
    # the change is of the size of the MRCM two-valuedness, not more
    assert rel_l2(Fd, m.F) < 50 * opposite_flux_defect(m.F) + 1e-12


@pytest.mark.parametrize("name", sorted(CASES))
def test_segment_sums_and_pure_neumann_means(name):
    """Each segment's total flux is that of the MRCM solution (eq. 13.2
    makes both sides' sums equal); subdomains with no Dirichlet face keep
    the MRCM mean pressure."""
    prob = problem(name)
    dec = Decomposition(prob)
    m = mrcm_solve(prob)
    pd, Fd = downscale(prob, m.p, m.F)
    bx, by, sg = dec.bx, dec.by, dec.sg
    scale = np.abs(m.F).max() * sg
    for I in range(1, dec.mx):
        gi = I * bx
        a = m.F[1][:, gi - 1].reshape(-1, sg).sum(1)
        b = -m.F[0][:, gi].reshape(-1, sg).sum(1)
        d = Fd[1][:, gi - 1].reshape(-1, sg).sum(1)
        assert np.abs(a - b).max() < 1e-10 * scale
        assert np.abs(d - a).max() < 1e-10 * scale
    for J in range(1, dec.my):
        gj = J * by
        a = m.F[3][gj - 1, :].reshape(-1, sg).sum(1)
        d = Fd[3][gj - 1, :].reshape(-1, sg).sum(1)
        assert np.abs(d - a).max() < 1e-10 * scale
    dirichlet = prob.bc_type == 1
    nx, ny = prob.nx, prob.ny
    for J in range(dec.my):
        for I in range(dec.mx):
            faces = []
            if I == 0:
                faces += list(range(J * by, (J + 1) * by))
            if I == dec.mx - 1:
                faces += list(range(ny + J * by, ny + (J + 1) * by))
            if J == 0:
                faces += list(range(2 * ny + I * bx, 2 * ny + (I + 1) * bx))
            if J == dec.my - 1:
                faces += list(range(2 * ny + nx + I * bx, 2 * ny + nx + (I + 1) * bx))
            if not dirichlet[faces].any():
                cs = dec.subdomain_cells(I, J)
                assert abs(pd[cs].mean() - m.p[cs].mean()) < 1e-12 * (np.abs(m.p).max() + 1)


def test_averaged_flux_is_antisymmetric():
    prob = problem("grf_b4_seg2")
    dec = Decomposition(prob)
    m = mrcm_solve(prob)
    Fb = averaged_skeleton_flux(prob, dec, m.F)
    W, E, S, N = Fb
    assert np.array_equal(E[:, 7], -W[:, 8]) and np.array_equal(N[7, :], -S[8, :])
    assert np.all(E[:, 8] == 0) and np.all(W[:, 0] == 0)
