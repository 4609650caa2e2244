"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the fact it checks.  A plausible slip anywhere in the
oracle (a dropped Robin term, a wrong sign of n_i.n, a transposed trace, a
wrong harmonic mean) fails at least one of them: the brute-force monolithic
system fixes every convention, seg = 1 fixes the Robin algebra for any
alpha, and the closed forms fix the discretisation itself.
"""

import os

import numpy as np
import pytest

from helpers import make_problem
from oracle.decomp import Decomposition
from oracle.fine import fine_solve
from oracle.local import local_solve
from oracle.metrics import rel_l2, cell_balance, cell_backward_error, interface_residual
from oracle.monolithic import monolithic_solve
from oracle.mrcm import mrcm_solve
from oracle.recursive import recursive_solve
from workloads import Problem, dirichlet_we, config_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- O-1 ---
@pytest.mark.parametrize("kval", [1.0, 3.7])
def test_fine_linear_pressure_homogeneous(kval):
    """Homogeneous K, p = 1 on W, 0 on E, no flow elsewhere: the exact
    solution p = 1 - x is reproduced exactly by the two-point scheme."""
    nx, ny = 24, 10
    t, v = dirichlet_we(nx, ny)
    P = Problem(nx=nx, ny=ny, K=np.full((ny, nx), kval), q=np.zeros((ny, nx)),
                bc_type=t, bc_value=v, sub_nx=nx, sub_ny=ny, seg=1)
    p, F = fine_solve(P)
    xc = (np.arange(nx) + 0.5) / nx
    assert np.abs(p - (1 - xc)[None, :]).max() < 1e-13
    # outward flux through the E face is K * |f| * 1 (unit gradient)
    assert np.abs(F[1] - kval / ny).max() < 1e-13
    assert np.abs(F[2]).max() < 1e-13


def test_fine_linear_pressure_y_layers():
    """K = K(y): each row is an independent 1D problem, p stays linear."""
    nx, ny = 16, 12
    rng = np.random.default_rng(1)
    K = np.repeat(np.exp(rng.standard_normal(ny))[:, None], nx, axis=1)
    t, v = dirichlet_we(nx, ny)
    P = Problem(nx=nx, ny=ny, K=K, q=np.zeros((ny, nx)), bc_type=t, bc_value=v,
                sub_nx=nx, sub_ny=ny, seg=1)
    p, F = fine_solve(P)
    xc = (np.arange(nx) + 0.5) / nx
    assert np.abs(p - (1 - xc)[None, :]).max() < 1e-13


def test_fine_series_harmonic_flux():
    """K = K(x): the flux through every row is 1 / sum_i hx / (K_i hy),
    the series (harmonic) resistance of the row."""
    nx, ny = 20, 6
    rng = np.random.default_rng(2)
    kx = np.exp(2 * rng.standard_normal(nx))
    K = np.repeat(kx[None, :], ny, axis=0)
    t, v = dirichlet_we(nx, ny)
    P = Problem(nx=nx, ny=ny, K=K, q=np.zeros((ny, nx)), bc_type=t, bc_value=v,
                sub_nx=nx, sub_ny=ny, seg=1)
    p, F = fine_solve(P)
    hx, hy = 1.0 / nx, 1.0 / ny
    flux = 1.0 / np.sum(hx / (kx * hy))
    assert np.abs(F[1][:, -1] - flux).max() < 1e-13 * flux
    assert np.abs(F[1][:, :-1] + F[0][:, 1:]).max() < 1e-14


def test_fine_all_neumann_gauge():
    """Quarter five-spot with no flow everywhere: zero-mean gauge and
    per-cell conservation."""
    P = make_problem(16, bc="fivespot")
    p, F = fine_solve(P)
    assert abs(p.mean()) < 1e-12
    assert cell_balance(F, P.q) < 1e-12


# ---------------------------------------------------------------- O-2 ---
def _dense_local_matrix(P, dec, I, J):
    """Loop-by-loop assembly of the local Robin matrix and unit-datum RHS,
    written independently of oracle.local."""
    bx, by = dec.bx, dec.by
    hx, hy = dec.hx, dec.hy
    n = bx * by
    A = np.zeros((n, n))
    slots = dec.subdomain_slots(I, J)
    B = np.zeros((n, len(slots)))
    for j in range(by):
        for i in range(bx):
            c = j * bx + i
            gi, gj = I * bx + i, J * by + j
            for d, (di, dj) in enumerate(((-1, 0), (1, 0), (0, -1), (0, 1))):
                area = hy if d < 2 else hx
                h = hx if d < 2 else hy
                ni, nj = i + di, j + dj
                rc = h / (2 * P.K[gj, gi])
                if 0 <= ni < bx and 0 <= nj < by:
                    rn = h / (2 * P.K[gj + dj, gi + di])
                    A[c, c] += area / (rc + rn)
                    A[c, nj * bx + ni] -= area / (rc + rn)
                    continue
                on_outer = not (0 <= gi + di < P.nx and 0 <= gj + dj < P.ny)
                if on_outer:
                    f = (gj if d == 0 else P.ny + gj if d == 1 else
                         2 * P.ny + gi if d == 2 else 2 * P.ny + P.nx + gi)
                    if P.bc_type[f] == 1:
                        A[c, c] += area / rc
                    continue
                # skeleton face: find its slot
                s_along = (j if d < 2 else i) // dec.sg
                nsy, nsx = dec.nsy, dec.nsx
                a = (s_along if d == 0 else nsy + s_along if d == 1 else
                     2 * nsy + s_along if d == 2 else 2 * nsy + nsx + s_along)
                e = slots[a][0]
                beta = dec.seg_beta[e]
                A[c, c] += area / (rc + beta)
                B[c, a] += area / (rc + beta)
    return A, B


@pytest.mark.parametrize("IJ", [(0, 0), (1, 1), (2, 1)])
def test_local_basis_matches_dense_assembly(IJ):
    P = make_problem(16, ny=8, b=4, seg=2, log_var=2.0)
    dec = Decomposition(P)
    r = local_solve(P, dec, *IJ)
    A, B = _dense_local_matrix(P, dec, *IJ)
    Psi = np.linalg.solve(A, B)
    assert rel_l2(r.Psi, Psi) < 1e-13


def test_local_partition_of_unity_and_max_principle():
    """With no Dirichlet face and no source, Robin datum 1 on every active
    slot gives p = 1 (sum of the basis is 1 cell by cell); each basis
    function lies in [0, 1]; the summed traces vanish (no net outflow)."""
    P = make_problem(32, b=8, seg=4, log_var=3.0)
    dec = Decomposition(P)
    for IJ in [(1, 1), (2, 1), (1, 3)]:
        r = local_solve(P, dec, *IJ)
        act = [a for a, s in enumerate(r.slots) if s[0] >= 0]
        s = r.Psi[:, act].sum(axis=1)
        assert np.abs(s - 1).max() < 1e-13
        assert r.Psi.min() > -1e-14 and r.Psi.max() < 1 + 1e-14
        assert np.abs(r.T[:, act].sum(axis=0)).max() < 1e-12 * np.abs(r.T).max()
        assert np.abs(r.T - r.T.T).max() < 1e-13 * np.abs(r.T).max()


def test_local_scale_invariance():
    """K -> cK leaves the basis pressures unchanged and scales traces by c
    (beta scales as 1/c through the effective permeability)."""
    P = make_problem(16, b=8, seg=4, log_var=2.0)
    P2 = P.with_(K=P.K * 7.5)
    d1, d2 = Decomposition(P), Decomposition(P2)
    r1, r2 = local_solve(P, d1, 1, 0), local_solve(P2, d2, 1, 0)
    assert rel_l2(r2.Psi, r1.Psi) < 1e-13
    assert rel_l2(r2.T, 7.5 * r1.T) < 1e-13


def test_robin_beta_special_cases():
    """beta = alpha Hbar / Keff: homogeneous K gives alpha Hbar / K; a
    two-material interface (K=1 | K=3) gives the harmonic mean 1.5."""
    nx = ny = 8
    K = np.ones((ny, nx))
    K[:, 4:] = 3.0
    t, v = dirichlet_we(nx, ny)
    P = Problem(nx=nx, ny=ny, K=K, q=np.zeros((ny, nx)), bc_type=t, bc_value=v,
                sub_nx=4, sub_ny=4, seg=2, alpha=2.5)
    dec = Decomposition(P)
    hbar = 2 / 8
    for e in range(dec.nseg):
        if dec.seg_orient[e] == 0:
            assert abs(dec.seg_beta[e] - 2.5 * hbar / 1.5) < 1e-15
        else:
            k = 1.0 if dec.seg_lo_cells[e][0][0] < 4 else 3.0
            assert abs(dec.seg_beta[e] - 2.5 * hbar / k) < 1e-15


# ---------------------------------------------------------------- O-3 ---
CASES = [
    dict(nx=8, b=4, seg=2),
    dict(nx=8, b=4, seg=1, alpha=0.3),
    dict(nx=8, b=4, seg=4, alpha=10.0),
    dict(nx=16, ny=8, b=4, seg=2, bc="mixed"),
    dict(nx=8, ny=16, b=4, by=2, seg=2, source=True),
    dict(nx=8, b=2, seg=1, bc="fivespot"),
    dict(nx=16, ny=8, b=2, by=4, seg=1, log_var=3.0),
]


@pytest.mark.parametrize("case", CASES)
def test_mrcm_equals_monolithic(case):
    """O-3's basis decomposition and all signs agree with the brute-force
    monolithic system (eq. 11.2-14.2 assembled cell by cell)."""
    P = make_problem(**case)
    r = mrcm_solve(P)
    p4, F4, U4, P4 = monolithic_solve(P)
    assert rel_l2(r.p, p4) < 1e-11
    assert rel_l2(r.F, F4) < 1e-11
    assert rel_l2(r.U, U4) < 1e-10
    assert rel_l2(r.P, P4) < 1e-11


@pytest.mark.parametrize("alpha", [1e-3, 1.0, 1e3, 1e6])
def test_mrcm_seg1_equals_fine(alpha):
    """When every segment is a single fine face, the interface spaces are
    the full set of fine faces and the method reproduces the fine solution
    for any alpha > 0."""
    P = make_problem(32, b=8, seg=1, alpha=alpha, log_var=2.0, source=True)
    r = mrcm_solve(P)
    pf, Ff = fine_solve(P)
    tol = 1e-10 if alpha < 1e5 else 1e-8
    assert rel_l2(r.p, pf) < tol
    assert rel_l2(r.F, Ff) < tol


@pytest.mark.parametrize("alpha", [0.1, 1.0, 100.0])
def test_mrcm_vertical_strips_exactly_linear(alpha):
    """Vertical strips only (one subdomain in y) with K constant on every
    segment: the linear pressure satisfies every local Robin problem with
    piecewise-constant data, so the method is exact."""
    nx, ny = 32, 8
    t, v = dirichlet_we(nx, ny)
    rng = np.random.default_rng(4)
    kseg = np.exp(rng.standard_normal(ny // 4))        # K(y), constant per segment
    K = np.repeat(np.repeat(kseg, 4)[:, None], nx, axis=1)
    P = Problem(nx=nx, ny=ny, K=K, q=np.zeros((ny, nx)), bc_type=t, bc_value=v,
                sub_nx=8, sub_ny=8, seg=4, alpha=alpha)
    r = mrcm_solve(P)
    xc = (np.arange(nx) + 0.5) / nx
    assert np.abs(r.p - (1 - xc)[None, :]).max() < 1e-12
    pf, Ff = fine_solve(P)
    assert rel_l2(r.F, Ff) < 1e-12


def test_mrcm_conservation_and_interface_equations():
    """Per-cell mass conservation of the one-sided fluxes and the interface
    equations eq. 13.2 / 14.2 on every segment."""
    P = make_problem(32, b=8, seg=4, log_var=3.0, source=True, bc="mixed")
    r = mrcm_solve(P)
    assert cell_balance(r.F, P.q) < 1e-12
    r13, r14 = interface_residual(r.dec, r.F, r.U)
    assert r13 < 1e-12 and r14 < 1e-12


def test_conservation_backward_error_high_contrast():
    """At high contrast the balance residual relative to max|F| grows with
    the contrast, but the per-cell backward error stays at round-off; a
    wrong face law (here: one flux perturbed by 1e-9 of its size) is seen."""
    P = make_problem(64, b=16, seg=4, log_var=9.0, lam=0.05)
    r = mrcm_solve(P)
    assert cell_backward_error(P, r.p, r.F) < 1e-13
    F2 = r.F.copy()
    F2[1, 10, 10] *= 1 + 1e-6
    assert cell_backward_error(P, r.p, F2) > 1e-12


def test_mrcm_superposition():
    """The solution is affine in the data: u(q1+q2, g) = u(q1, g) + u(q2, 0)."""
    P = make_problem(16, b=4, seg=2, source=True)
    rng = np.random.default_rng(9)
    q2 = rng.standard_normal(P.q.shape)
    a = mrcm_solve(P.with_(q=P.q + q2))
    b = mrcm_solve(P)
    c = mrcm_solve(P.with_(q=q2, bc_value=np.zeros_like(P.bc_value)))
    assert rel_l2(a.p, b.p + c.p) < 1e-12
    assert rel_l2(a.F, b.F + c.F) < 1e-12


def test_mrcm_all_neumann_gauge():
    P = make_problem(16, b=4, seg=2, bc="fivespot", log_var=2.0)
    r = mrcm_solve(P)
    assert abs(r.p.mean()) < 1e-12
    assert cell_balance(r.F, P.q) < 1e-12
    p4, F4, _u, _p = monolithic_solve(P)
    assert rel_l2(r.p, p4) < 1e-11 and rel_l2(r.F, F4) < 1e-11


def test_decomposition_rejects_bad_geometry():
    for kw in (dict(nx=12, b=4), dict(nx=16, b=4, seg=3), dict(nx=10, b=4)):
        with pytest.raises(ValueError):
            Decomposition(make_problem(log_var=0, **kw))


def test_table3_local_solve_counts():
    """Table 3: local problems at the finest level for Hbar = H and H/4."""
    rows = np.loadtxt(os.path.join(GOLDEN, "table3_mmbf_counts.txt"), dtype=int)
    for mx, my, c1, c4 in rows:
        for div, want in ((1, c1), (4, c4)):
            b = 8
            t, v = dirichlet_we(mx * b, my * b)
            P = Problem(nx=mx * b, ny=my * b, K=np.ones((my * b, mx * b)),
                        q=np.zeros((my * b, mx * b)), bc_type=t, bc_value=v,
                        sub_nx=b, sub_ny=b, seg=b // div)
            assert Decomposition(P).count_local_solves() == want


def test_finest_interface_system_size():
    """With Hbar = H the finest interface system is 2x2 (one U and one P),
    and each coarser level of the same orientation doubles it."""
    from oracle.recursive import RecursiveMRCM, _gamma_segments
    P = make_problem(32, b=8, seg=8)
    R = RecursiveMRCM(P)
    sizes = {}

    def walk(node, depth):
        if node.children is None:
            return
        sizes.setdefault(depth, set()).add(2 * len(_gamma_segments(R.dec, node)))
        for c in node.children:
            walk(c, depth + 1)
    walk(R.root, 0)
    assert sizes[max(sizes)] == {2}
    assert sizes[0] == {8}


# ---------------------------------------------------------------- O-5 ---
@pytest.mark.parametrize("order", ["x-first", "y-first"])
def test_recursive_equals_nonrecursive(order):
    """Algorithm 1 (nested pairwise interface solves) equals the single
    global interface system: the recursion is an exact nested
    elimination, whatever the split order."""
    P = config_problem(1)
    r = mrcm_solve(P)
    p5, F5, U5, P5 = recursive_solve(P, order=order)
    assert rel_l2(p5, r.p) < 1e-10
    assert rel_l2(F5, r.F) < 1e-10
    assert rel_l2(U5, r.U) < 1e-10
    assert rel_l2(P5, r.P) < 1e-10


def test_recursive_rectangular_and_sources():
    P = make_problem(32, ny=16, b=4, seg=2, source=True, bc="mixed", log_var=2.0)
    r = mrcm_solve(P)
    p5, F5, U5, P5 = recursive_solve(P)
    assert rel_l2(p5, r.p) < 1e-10 and rel_l2(F5, r.F) < 1e-10


def test_alpha_trend_homogeneous():
    """Section 2 and Section 5.1: large alpha drives the method towards the
    flux-continuous limit; on the homogeneous problem of Section 5.4 the
    velocity error against the fine solution falls as alpha grows, and the
    finer interface space (Hbar = H/4) is more accurate than Hbar = H.
    (The absolute values of the paper's accuracy tables are not
    reproduced: parity unpinned beyond this trend.)"""
    n, b = 64, 16
    t, v = dirichlet_we(n, n)
    errs = {}
    for alpha in (1.0, 1e3, 1e6):
        for div in (1, 4):
            P = Problem(nx=n, ny=n, K=np.ones((n, n)), q=np.zeros((n, n)),
                        bc_type=t, bc_value=v, sub_nx=b, sub_ny=b, seg=b // div,
                        alpha=alpha)
            r = mrcm_solve(P)
            _p, Ff = fine_solve(P)
            errs[alpha, div] = rel_l2(r.F, Ff)
    assert errs[1.0, 1] > errs[1e3, 1] > errs[1e6, 1]
    for alpha in (1.0, 1e3, 1e6):
        assert errs[alpha, 4] < errs[alpha, 1]
    assert errs[1e6, 4] < 1e-5


# ------------------------------------------------- O-4, extended precision
def test_extended_precision_monolithic_agrees_at_alpha_1():
    """The extended-precision refinement of O-4 changes nothing where the
    system is well conditioned; there it equals O-3."""
    P = make_problem(32, b=8, seg=2, log_var=3.0, source=True, bc="mixed")
    p0, F0, U0, P0 = monolithic_solve(P)
    p1, F1, U1, P1 = monolithic_solve(P, ext_iters=3)
    assert rel_l2(p1, p0) < 1e-13 and rel_l2(F1, F0) < 1e-12
    r = mrcm_solve(P)
    assert rel_l2(r.p, p1) < 1e-12 and rel_l2(r.F, F1) < 1e-12


def test_alpha_1e6_accuracy_floor():
    """At alpha = 1e6 the discrete system is ill conditioned: its exact
    solution (O-4 refined in extended precision) moves by well under 1e-10
    when every permeability changes by one unit in the last place (the
    reference is well defined at that level), while the FP64 oracle O-3 is
    within 2e-9 of it but not within 1e-10 (the floor of FP64 solvers,
    against which the GPU path at this alpha is tested)."""
    P = make_problem(64, b=16, seg=4, alpha=1e6, log_var=3.0, lam=0.1, seed=40, source=True)
    p, F, _U, _P = monolithic_solve(P, ext_iters=4)
    rng = np.random.default_rng(1)
    K2 = P.K * (1 + np.finfo(float).eps * rng.choice([-1.0, 1.0], size=P.K.shape))
    p2, F2, _U2, _P2 = monolithic_solve(P.with_(K=K2), ext_iters=4)
    assert rel_l2(p2, p) < 1e-10 and rel_l2(F2, F) < 1e-10
    r = mrcm_solve(P)
    assert rel_l2(r.p, p) < 2e-9 and rel_l2(r.F, F) < 2e-9
    assert max(rel_l2(r.p, p), rel_l2(r.F, F)) > 1e-11
