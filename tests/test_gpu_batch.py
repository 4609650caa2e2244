"""Ensemble batches (rmrcm_batch_*) on the GPU.

Members of the five-spot ensemble (all no-flow boundaries, +1/-1 wells,
subdomains of 8, 16 and 32 cells) at 128^2, plus W/E Dirichlet problems,
solved together: against the oracle element by element (FP64 bar 1e-10),
bit for bit against the same problems solved one context at a time (the
batch replays captured graphs of the same kernels), over repeated graph
replays with new data, and with a member whose data are incompatible.
"""

import sys

import numpy as np
import pytest

from helpers import make_problem
from oracle.metrics import rel_l2
from oracle.mrcm import mrcm_solve
from workloads import ensemble_member

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2009_07965_amd as L
    return L


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def members():
    # b = 16, 32, 8, 8 (ensemble members at 128^2) and two W/E problems
    ms = [ensemble_member(m, n_override=128) for m in (0, 1, 2, 6)]
    ms.append(make_problem(64, b=16, seg=4, log_var=2.0, source=True))
    ms.append(make_problem(128, ny=64, b=8, seg=2, log_var=3.0, bc="mixed"))
    return ms


def single(L, prob):
    S = L.Solver.from_problem(prob)
    try:
        return S.solve(prob.q, prob.bc_value)
    finally:
        S.close()


def test_batch_matches_oracle_and_single_contexts(lib):
    probs = members()
    say("[gpu] batch of %d: %s" % (len(probs), [(p.nx, p.sub_nx) for p in probs]))
    B = lib.Batch(probs)
    try:
        st = B.stats()
        assert st["members"] == len(probs) and st["graph_members"] == len(probs)
        P, F = B.solve([p.q for p in probs], [p.bc_value for p in probs])
    finally:
        B.close()
    for k, pr in enumerate(probs):
        ref = mrcm_solve(pr)
        if pr.bc_type.max() == 0:          # all Neumann: compare after the zero-mean gauge
            rp = ref.p - ref.p.mean()
        else:
            rp = ref.p
        assert rel_l2(P[k], rp) <= TOL, (k, rel_l2(P[k], rp))
        assert rel_l2(F[k], ref.F) <= TOL, (k, rel_l2(F[k], ref.F))
        p1, f1 = single(lib, pr)
        assert np.array_equal(p1, P[k]) and np.array_equal(f1, F[k]), k


def test_batch_graph_replays_with_new_data(lib):
    """Three solves with different sources and boundary data, eager host
    work in between; every replay equals a fresh single-context solve."""
    probs = members()[4:]                 # the two W/E problems
    B = lib.Batch(probs, autotune=False)
    rng = np.random.default_rng(5)
    try:
        for rep in range(3):
            qs = [rng.standard_normal(p.q.shape) / p.ncells for p in probs]
            bvs = []
            for p in probs:
                bv = p.bc_value.copy()
                bv[:p.ny] = 1.0 + rep
                bvs.append(bv)
            say("[gpu] batch replay %d" % rep)
            P, F = B.solve(qs, bvs)
            for k, p in enumerate(probs):
                pr = p.with_(q=qs[k], bc_value=bvs[k])
                p1, f1 = single(lib, pr)
                assert np.array_equal(p1, P[k]) and np.array_equal(f1, F[k]), (rep, k)
    finally:
        B.close()


def test_batch_refactor(lib):
    probs = members()[:3]
    new = [p.with_(K=np.exp(0.5 * np.log(p.K))) for p in probs]
    B = lib.Batch(probs, autotune=False)
    try:
        say("[gpu] batch refactor")
        B.refactor([p.K for p in new])
        P, F = B.solve([p.q for p in new], [p.bc_value for p in new])
    finally:
        B.close()
    for k, pr in enumerate(new):
        ref = mrcm_solve(pr)
        e = rel_l2(P[k], ref.p - ref.p.mean())
        if e > TOL:             # tell a stale factorisation from other errors
            old = mrcm_solve(probs[k])
            pytest.fail("member %d: rel err %.3e vs the new field, %.3e vs the old one"
                        % (k, e, rel_l2(P[k], old.p - old.p.mean())))
        assert rel_l2(F[k], ref.F) <= TOL


def test_batch_reports_incompatible_member(lib):
    """All-Neumann data whose net source is not zero: that member's status
    is EINVAL at sync, the others are OK."""
    probs = members()[:3]
    B = lib.Batch(probs, autotune=False)
    try:
        qs = [p.q.copy() for p in probs]
        qs[1][3, 3] += 1.0
        say("[gpu] incompatible member")
        B.solve(qs, [p.bc_value for p in probs], wait=False)
        with pytest.raises(lib.RMRCMError) as ei:
            B.sync()
        assert "[0, -1, 0]" in str(ei.value)
        P, F = B.solve([p.q for p in probs], [p.bc_value for p in probs])
        assert B.sync() == [0, 0, 0]
    finally:
        B.close()


def test_autotune_does_not_change_results(lib):
    prob = make_problem(256, b=8, seg=2, log_var=2.0)
    S = lib.Solver.from_problem(prob)
    try:
        say("[gpu] autotune")
        p0, f0 = S.solve(prob.q, prob.bc_value)
        S.autotune()
        S.refactor(prob.K)
        p1, f1 = S.solve(prob.q, prob.bc_value)
    finally:
        S.close()
    assert np.array_equal(p0, p1) and np.array_equal(f0, f1)
