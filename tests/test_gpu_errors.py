"""Error paths on the GPU that the host can force without a faulty kernel:
the memory plan against what a context really allocates, a memory cap one
byte short, a refinement that cannot reach its tolerance, and a legal
permeability whose local system is singular in floating point (the device
flag of the local factorisation, ESINGULAR at the sync)."""

import numpy as np
import pytest

from helpers import make_problem
from oracle.metrics import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2009_07965_amd as lib
    return lib


@pytest.mark.parametrize("precision", [0, 1])
def test_plan_equals_allocation(L, precision):
    prob = make_problem(128, b=16, seg=4, log_var=2.0)
    print("[gpu-errors] plan vs allocation, precision %d" % precision, flush=True)
    S = L.Solver.from_problem(prob, precision=precision)
    try:
        got = S.stats()["device_bytes"]
        plan = L.rmrcm_plan_bytes(S.params)
    finally:
        S.close()
    assert got == plan


def test_cap_one_byte_short_is_enomem(L):
    prob = make_problem(128, b=16, seg=4, log_var=2.0)
    print("[gpu-errors] memory cap", flush=True)
    S = L.Solver.from_problem(prob)
    try:
        plan = L.rmrcm_plan_bytes(S.params)
    finally:
        S.close()
    with pytest.raises(L.RMRCMError) as ei:
        L.Solver.from_problem(prob, mem_cap=plan - 1)
    assert ei.value.status == -2
    S = L.Solver.from_problem(prob, mem_cap=plan)     # exactly the plan: fits
    S.close()


def test_unreachable_tolerance_at_solve_falls_back_to_fp64(L):
    """Setup with the default refinement (converges), then a tolerance no
    refinement reaches with one pass: the particular solution of every
    subdomain is solved again in FP64 (its subdomain factored in FP64 for
    that solve), the solve succeeds and counts them, and its result is that
    of the FP64 particular solutions; restoring the defaults gives the
    first solve's result again, bit for bit."""
    prob = make_problem(128, b=16, seg=4, log_var=2.0, source=True)
    print("[gpu-errors] particular fallback at solve", flush=True)
    S = L.Solver.from_problem(prob, precision=1)
    try:
        p0, F0 = S.solve(prob.q, prob.bc_value)
        assert S.stats()["fp64_particular_fallback_subdomains"] == 0
        L.rmrcm_set_refinement(S.ctx, 1e-300, 1)
        p1, F1 = S.solve(prob.q, prob.bc_value)
        assert S.stats()["fp64_particular_fallback_subdomains"] == 64
        assert rel_l2(p1, p0) < 1e-9 and rel_l2(F1, F0) < 1e-9
        L.rmrcm_set_refinement(S.ctx, 1e-11, 6)
        p2, F2 = S.solve(prob.q, prob.bc_value)
        assert np.array_equal(p0, p2) and np.array_equal(F0, F2)
    finally:
        S.close()
    S = L.Solver.from_problem(prob)
    try:
        pr, Fr = S.solve(prob.q, prob.bc_value)
    finally:
        S.close()
    assert rel_l2(p1, pr) < 1e-9 and rel_l2(F1, Fr) < 1e-9


def test_set_refinement_rejects(L):
    prob = make_problem(64, b=16, seg=4)
    S = L.Solver.from_problem(prob)
    try:
        with pytest.raises(L.RMRCMError) as ei:
            L.rmrcm_set_refinement(S.ctx, 1e-12, 3)
        assert ei.value.status == -7           # FP64 context
    finally:
        S.close()
    S = L.Solver.from_problem(prob, precision=1)
    try:
        for tol, it in ((0.0, 3), (1e-12, 0)):
            with pytest.raises(L.RMRCMError) as ei:
                L.rmrcm_set_refinement(S.ctx, tol, it)
            assert ei.value.status == -1
    finally:
        S.close()


def test_subnormal_permeability_is_esingular(L):
    """A subdomain whose permeability is the smallest positive subnormal
    passes the permeability check (finite and positive), but every half-cell
    resistance h / (2 K) overflows, so every face conductance of its local
    system is 0 and its first pivot is 0: the FP64 factorisation flags it
    and setup returns ESINGULAR (-4).  Every kernel after the flagged one is
    bounded and indexes through the level tables only, so the NaN data it
    leaves change no access.  A context on the same grid with a regular
    permeability afterwards solves to the oracle's bar."""
    from oracle.mrcm import mrcm_solve
    prob = make_problem(64, b=16, seg=4, log_var=1.0, seed=7)
    prob.K[16:32, 16:32] = 5e-324
    assert prob.K[20, 20] > 0.0
    print("[gpu-errors] subnormal permeability", flush=True)
    with pytest.raises(L.RMRCMError) as ei:
        L.Solver.from_problem(prob)
    assert ei.value.status == -4
    good = make_problem(64, b=16, seg=4, log_var=1.0, seed=7)
    S = L.Solver.from_problem(good)
    try:
        p, _F = S.solve(good.q, good.bc_value)
    finally:
        S.close()
    assert rel_l2(p, mrcm_solve(good).p) <= 1e-10
