"""rmrcm_step (refactor + solve as one unit, a replayed HIP graph for FP64
contexts with device arrays) on the GPU.

The graph carries the particular problem as one more column of the local
sweeps and of the merges below the top, where rmrcm_refactor followed by
rmrcm_solve runs it as a chain of its own: the two differ only in the order
of the particular sweeps' sums, so they are compared at STEP_TOL (rounding
of the sweeps, 1e-16, times the growth through the hierarchy), and both
with the oracle at the FP64 bar.  Replays with new permeability and sources
at the same pointers, new output arrays (a new capture, bit for bit), the
same chain without a graph (bit for bit), host arrays (the eager path, bit
for bit), subdomains 8, 16 and 32 cells wide
(8: the particular solve follows the local setup in the same chain) and an
incompatible all-Neumann source (EINVAL at sync).
"""

import sys

import numpy as np
import pytest

from helpers import make_problem
from oracle.metrics import rel_l2
from oracle.mrcm import mrcm_solve

pytestmark = pytest.mark.gpu

TOL = 1e-10
STEP_TOL = 1e-12


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2009_07965_amd as L
    return L, torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev_arrays(torch, prob):
    d = torch.device("cuda:0")
    return (torch.from_numpy(prob.K).to(d), torch.from_numpy(prob.q).to(d),
            torch.from_numpy(prob.bc_value).to(d),
            torch.zeros((prob.ny, prob.nx), dtype=torch.float64, device=d),
            torch.zeros((4, prob.ny, prob.nx), dtype=torch.float64, device=d))


def eager(L, prob):
    S = L.Solver.from_problem(prob)
    try:
        return S.solve(prob.q, prob.bc_value)
    finally:
        S.close()


@pytest.mark.parametrize("n,b,seg", [(256, 32, 8), (128, 16, 4), (64, 8, 2)])
def test_step_equals_refactor_and_solve(env, n, b, seg):
    L, torch = env
    base = make_problem(n, b=b, seg=seg, log_var=2.0, seed=31)
    probs = [make_problem(n, b=b, seg=seg, log_var=lv, lam=0.08, seed=40 + k, source=True)
             for k, lv in enumerate((1.0, 3.0, 4.5))]
    S = L.Solver.from_problem(base)
    stream = torch.cuda.Stream()
    try:
        S.set_stream(stream.cuda_stream)
        K, q, bv, pd, fd = dev_arrays(torch, probs[0])
        for k, pr in enumerate(probs):
            say("[gpu] step %d, n %d, b %d" % (k, n, b))
            K.copy_(torch.from_numpy(pr.K))
            q.copy_(torch.from_numpy(pr.q))
            bv.copy_(torch.from_numpy(pr.bc_value))
            torch.cuda.synchronize()
            S.step(K, q, bv, pd, fd)
            S.sync()
            p, F = pd.cpu().numpy(), fd.cpu().numpy()
            pe, Fe = eager(L, pr)
            assert rel_l2(p, pe) <= STEP_TOL and rel_l2(F, Fe) <= STEP_TOL, k
            ref = mrcm_solve(pr)
            assert rel_l2(p, ref.p) <= TOL and rel_l2(F, ref.F) <= TOL
        st = S.stats()              # timers of the last run outside the graph
        assert st["setup_ms"]["local"] > 0      # from the setup at creation
        # new output arrays: a new capture, same numbers
        pd2 = torch.zeros_like(pd)
        fd2 = torch.zeros_like(fd)
        S.step(K, q, bv, pd2, fd2)
        S.sync()
        assert torch.equal(pd2, pd) and torch.equal(fd2, fd)
        # an ordinary solve after steps (eager path, same context)
        p3, F3 = S.solve(probs[-1].q, probs[-1].bc_value)
        assert rel_l2(p3, pd.cpu().numpy()) <= STEP_TOL and rel_l2(F3, fd.cpu().numpy()) <= STEP_TOL
    finally:
        S.close()


@pytest.mark.parametrize("n,b,seg", [(256, 32, 8), (64, 8, 2), (256, 8, 1)])
def test_step_without_graph_equals_graph(env, n, b, seg):
    """rmrcm_set_step_graph(0): the same chain launch by launch, bit for bit
    the graph's results, with the phase timers recording it."""
    L, torch = env
    pr = make_problem(n, b=b, seg=seg, log_var=3.0, lam=0.08, seed=61, source=True)
    S = L.Solver.from_problem(pr)
    stream = torch.cuda.Stream()
    try:
        S.set_stream(stream.cuda_stream)
        K, q, bv, pd, fd = dev_arrays(torch, pr)
        say("[gpu] step graph vs launch by launch, n %d, b %d" % (n, b))
        S.step(K, q, bv, pd, fd)
        S.sync()
        pg, Fg = pd.clone(), fd.clone()
        S.set_step_graph(False)
        pd.zero_()
        fd.zero_()
        S.step(K, q, bv, pd, fd)
        S.sync()
        assert torch.equal(pd, pg) and torch.equal(fd, Fg)
        st = S.stats()
        assert st["setup_ms"]["local"] > 0 and st["setup_ms"]["merge"] > 0
        assert st["solve_ms"]["down"] > 0 and st["solve_ms"]["reconstruct"] > 0
        S.set_step_graph(True)
        S.step(K, q, bv, pd, fd)
        S.sync()
        assert torch.equal(pd, pg) and torch.equal(fd, Fg)
    finally:
        S.close()


def test_step_host_arrays_take_the_eager_path(env):
    L, _torch = env
    pr = make_problem(128, b=16, seg=4, log_var=2.0, seed=51, source=True)
    S = L.Solver.from_problem(make_problem(128, b=16, seg=4, log_var=1.0, seed=50))
    try:
        say("[gpu] step, host arrays")
        p, F = S.step(pr.K, pr.q, pr.bc_value)
    finally:
        S.close()
    pe, Fe = eager(L, pr)
    assert np.array_equal(p, pe) and np.array_equal(F, Fe)


def test_step_incompatible_neumann_data_at_sync(env):
    """All-Neumann problem with a net source: the device check marks the
    data and the sync after the step returns EINVAL; a compatible step
    afterwards succeeds."""
    L, torch = env
    from paper_2009_07965_amd import RMRCMError
    from workloads import ensemble_member
    pr = ensemble_member(0, n_override=128)
    S = L.Solver.from_problem(pr)
    stream = torch.cuda.Stream()
    try:
        S.set_stream(stream.cuda_stream)
        K, q, bv, pd, fd = dev_arrays(torch, pr)
        q[3, 3] += 1.0
        say("[gpu] step, incompatible data")
        S.step(K, q, bv, pd, fd)
        with pytest.raises(RMRCMError):
            S.sync()
        q[3, 3] -= 1.0
        S.step(K, q, bv, pd, fd)
        S.sync()
        ref = mrcm_solve(pr)
        p = pd.cpu().numpy()
        assert rel_l2(p, ref.p - ref.p.mean()) <= TOL
    finally:
        S.close()


def test_step_single_subdomain(env):
    """One subdomain with Dirichlet faces (no interface, no merge level):
    the step is the local problem alone; against the eager solve and the
    oracle, and a second step with new data at the same pointers."""
    L, torch = env
    pr = make_problem(32, b=32, seg=8, source=True, seed=61)
    S = L.Solver.from_problem(pr)
    stream = torch.cuda.Stream()
    try:
        S.set_stream(stream.cuda_stream)
        K, q, bv, pd, fd = dev_arrays(torch, pr)
        say("[gpu] step, one subdomain")
        S.step(K, q, bv, pd, fd)
        S.sync()
        p1, F1 = pd.cpu().numpy(), fd.cpu().numpy()
        pr2 = make_problem(32, b=32, seg=8, source=True, seed=62, log_var=2.0)
        K.copy_(torch.from_numpy(pr2.K))
        q.copy_(torch.from_numpy(pr2.q))
        bv.copy_(torch.from_numpy(pr2.bc_value))
        torch.cuda.synchronize()
        S.step(K, q, bv, pd, fd)
        S.sync()
        p2, F2 = pd.cpu().numpy(), fd.cpu().numpy()
    finally:
        S.close()
    for prob, p, F in ((pr, p1, F1), (pr2, p2, F2)):
        pe, Fe = eager(L, prob)
        assert rel_l2(p, pe) <= STEP_TOL and rel_l2(F, Fe) <= STEP_TOL
        ref = mrcm_solve(prob)
        assert rel_l2(p, ref.p) <= TOL and rel_l2(F, ref.F) <= TOL
