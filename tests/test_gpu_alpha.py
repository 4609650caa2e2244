"""The Robin parameter alpha over its range (Section 5.1: beta_e =
alpha Hbar_e / Keff_e; small alpha approaches the MMMFEM coupling, large
alpha the MHM coupling; the paper's accuracy runs use alpha = 1e6): the
FP64 GPU path against the oracle at the FP64 bar and the mixed path at the
mixed bar, on heterogeneous fields with 16- and 32-cell subdomains.

At alpha = 1e6 the local Robin systems are nearly singular (the Robin
conductance |f| / (rho + beta) is about 1e-6 of the interior couplings)
and no FP64 solver reaches the 1e-10 bar: against the solution of the
monolithic system refined in extended precision (oracle.monolithic with
ext_iters) the oracle itself is 3e-10 (p) and 6e-10 to 1e-9 (F) away.
There the GPU path (with its interface refinement, which takes the
interface residual from ~1e-11 to ~1e-15) is held to 2e-9 (p) and 1e-8
(F) against that solution and to ten times the oracle's own distance."""

import sys

import numpy as np
import pytest

from helpers import make_problem
from oracle.metrics import rel_l2, cell_backward_error
from oracle.monolithic import monolithic_solve
from oracle.mrcm import mrcm_solve

pytestmark = pytest.mark.gpu
ALPHAS = [1e-6, 1e-3, 1e3, 1e6]


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2009_07965_amd as lib
    return lib


def run(L, prob, **kw):
    S = L.Solver.from_problem(prob, **kw)
    try:
        return S.solve(prob.q, prob.bc_value)
    finally:
        S.close()


@pytest.mark.parametrize("alpha", ALPHAS[:3])
@pytest.mark.parametrize("shape", [(128, 16, 4), (256, 32, 8)])
def test_fp64_alpha_matches_oracle(L, alpha, shape):
    n, b, seg = shape
    prob = make_problem(n, b=b, seg=seg, alpha=alpha, log_var=3.0, lam=0.1, seed=40, source=True)
    print("[gpu] alpha %g, %d^2, b %d" % (alpha, n, b), flush=True)
    p, F = run(L, prob)
    ref = mrcm_solve(prob)
    ep, ef = rel_l2(p, ref.p), rel_l2(F, ref.F)
    print("    p %.2e F %.2e" % (ep, ef), flush=True)
    assert ep <= 1e-10 and ef <= 1e-10
    assert cell_backward_error(prob, p, F) < 1e-12


@pytest.mark.parametrize("shape", [(128, 16, 4), (256, 32, 8)])
def test_fp64_alpha_1e6_against_extended_precision(L, shape):
    n, b, seg = shape
    prob = make_problem(n, b=b, seg=seg, alpha=1e6, log_var=3.0, lam=0.1, seed=40, source=True)
    print("[gpu] alpha 1e6, %d^2, b %d" % (n, b), flush=True)
    S = L.Solver.from_problem(prob)
    try:
        p, F = S.solve(prob.q, prob.bc_value)
        st = S.stats()
    finally:
        S.close()
    pe, Fe, _U, _P = monolithic_solve(prob, ext_iters=4)
    ref = mrcm_solve(prob)
    ep, ef = rel_l2(p, pe), rel_l2(F, Fe)
    op, of = rel_l2(ref.p, pe), rel_l2(ref.F, Fe)
    print("    vs extended: GPU p %.2e F %.2e, oracle p %.2e F %.2e; interface residual %.2e -> %.2e"
          % (ep, ef, op, of, st["interface_residual"], st["interface_residual_refined"]), flush=True)
    assert st["interface_refined"] == 1 and 0 < st["interface_residual_refined"] < 1e-13
    assert ep <= 2e-9 and ef <= 1e-8
    assert ep <= 10 * op and ef <= 10 * of
    # the balance's backward error: its scale (conductances x max|p|)
    # leaves out the Robin data |g| ~ beta |U| >> |p| at this alpha; the
    # oracle's own is 2.2e-12 and 2.7e-12 on these two problems
    ob = cell_backward_error(prob, ref.p, ref.F)
    assert cell_backward_error(prob, p, F) < max(1e-11, 5 * ob)


@pytest.mark.parametrize("alpha", [1e-6, 1e6])
def test_mixed_alpha_extremes(L, alpha):
    prob = make_problem(128, b=16, seg=4, alpha=alpha, log_var=3.0, lam=0.1, seed=41)
    print("[gpu] mixed, alpha %g" % alpha, flush=True)
    p, F = run(L, prob, precision=1)
    ref = mrcm_solve(prob)
    assert rel_l2(p, ref.p) <= 1e-9 and rel_l2(F, ref.F) <= 1e-9


def test_alpha_limits_on_the_gpu(L):
    """Small alpha weights pressure continuity (the face pressures seen from
    the two sides of a skeleton face agree: the MMMFEM limit), large alpha
    flux continuity (the two one-sided fluxes agree: the MHM limit)."""
    dp, df = [], []
    for alpha in ALPHAS:
        prob = make_problem(128, b=16, seg=4, alpha=alpha, log_var=2.0, lam=0.1, seed=42)
        p, F = run(L, prob)
        bx = prob.sub_nx
        hx, hy = 1.0 / prob.nx, 1.0 / prob.ny
        a, b = slice(bx - 1, -1, bx), slice(bx, None, bx)          # cells left / right of the lines
        Fa, Fb = F[1][:, a], F[0][:, b]
        df.append(np.abs(Fa + Fb).max() / np.abs(F).max())
        la = p[:, a] - hx / (2 * prob.K[:, a]) * Fa / hy             # face pressure from the left
        lb = p[:, b] - hx / (2 * prob.K[:, b]) * Fb / hy             # and from the right
        dp.append(np.abs(la - lb).max() / np.abs(p).max())
    print("    flux defects %s, face-pressure defects %s" % (df, dp), flush=True)
    assert df[-1] < 1e-3 * df[0]
    assert dp[0] < 1e-3 * dp[-1]
