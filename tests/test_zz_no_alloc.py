"""rmrcm_step_noalloc, the allocation-free FP64 step, through the C ABI.

Compared with the context-based entry points it varies (rmrcm_setup +
rmrcm_step on device arrays, the same kernels in the same order): bit for
bit, on two calls in a row, the second with a smaller problem (the scratch
keeps the first call's contents, which the second must not see), plus the
oracle at the FP64 bar.  Also: a problem larger than the scratch is
rejected before any device work (ETOOBIG), host pointers are rejected
(EINVAL), and a non-positive permeability found on the device is returned
as EINVAL with the next call unaffected.
"""

import sys

import numpy as np
import pytest

from helpers import make_problem
from oracle.metrics import rel_l2
from oracle.mrcm import mrcm_solve

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def params(L, prob):
    p = L.rmrcm_default_params()
    p.nx, p.ny, p.lx, p.ly = prob.nx, prob.ny, prob.lx, prob.ly
    p.sub_nx, p.sub_ny, p.seg, p.alpha = prob.sub_nx, prob.sub_ny, prob.seg, prob.alpha
    return p


def dev(torch, prob):
    d = torch.device("cuda:0")
    return (torch.from_numpy(prob.K).to(d), torch.from_numpy(prob.bc_type).to(d),
            torch.from_numpy(prob.q).to(d), torch.from_numpy(prob.bc_value).to(d),
            torch.zeros((prob.ny, prob.nx), dtype=torch.float64, device=d),
            torch.zeros((4, prob.ny, prob.nx), dtype=torch.float64, device=d))


def with_context(L, torch, prob):
    """rmrcm_setup + rmrcm_step on device arrays (the existing entry points)."""
    K, bt, q, bv, pd, fd = dev(torch, prob)
    S = L.Solver(prob.nx, prob.ny, K, bt, prob.sub_nx, prob.sub_ny, prob.seg, alpha=prob.alpha)
    try:
        S.step(K, q, bv, pd, fd)
        S.sync()
    finally:
        S.close()
    return pd.cpu().numpy(), fd.cpu().numpy()


def noalloc(L, torch, prob, stream=None, source=True):
    K, bt, q, bv, pd, fd = dev(torch, prob)
    torch.cuda.synchronize()
    L.rmrcm_step_noalloc(params(L, prob), K, prob.bc_type, q if source else None, bv, pd, fd,
                         stream.cuda_stream if stream is not None else None)
    return pd.cpu().numpy(), fd.cpu().numpy()


def test_two_calls_second_smaller(env):
    L, torch = env
    big = make_problem(512, b=32, seg=8, log_var=3.0, lam=0.08, seed=91, source=True)
    small = make_problem(128, b=16, seg=4, log_var=2.0, seed=92, source=True, bc="mixed")
    stream = torch.cuda.Stream()
    for k, prob in enumerate((big, small)):
        say("[gpu] noalloc call %d: %dx%d b %d" % (k, prob.nx, prob.ny, prob.sub_nx))
        p, F = noalloc(L, torch, prob, stream=stream)
        pc, Fc = with_context(L, torch, prob)
        assert np.array_equal(p, pc) and np.array_equal(F, Fc), k
        ref = mrcm_solve(prob)
        assert rel_l2(p, ref.p) <= TOL and rel_l2(F, ref.F) <= TOL


def test_null_stream_zero_source_and_neumann(env):
    """The null stream, a NULL source, 8-cell subdomains (the particular
    solve as its own launch) and an all-Neumann five-spot (zero-mean gauge)."""
    L, torch = env
    for prob, src in ((make_problem(64, b=8, seg=2, log_var=1.0, seed=93), False),
                      (make_problem(128, b=16, seg=4, bc="fivespot", log_var=2.0, seed=94), True)):
        say("[gpu] noalloc null stream b %d" % prob.sub_nx)
        p, F = noalloc(L, torch, prob, source=src)
        pc, Fc = with_context(L, torch, prob)
        assert np.array_equal(p, pc) and np.array_equal(F, Fc)


def test_rejections(env):
    L, torch = env
    from paper_2009_07965_amd import RMRCMError
    prob = make_problem(64, b=16, seg=4, seed=95)
    K, bt, q, bv, pd, fd = dev(torch, prob)
    say("[gpu] noalloc rejections")
    with pytest.raises(RMRCMError) as ei:          # host permeability
        L.rmrcm_step_noalloc(params(L, prob), prob.K, prob.bc_type, q, bv, pd, fd)
    assert ei.value.status == -1
    p = params(L, prob)
    p.precision = 1
    with pytest.raises(RMRCMError) as ei:
        L.rmrcm_step_noalloc(p, K, prob.bc_type, q, bv, pd, fd)
    assert ei.value.status == -7
    # 4096^2 cells need several GB: rejected before any device work (the
    # arrays passed are never touched, so small ones suffice)
    p = params(L, prob)
    p.nx = p.ny = 4096
    p.sub_nx = p.sub_ny = 32
    p.seg = 8
    bt_big = np.ones(4 * 4096, dtype=np.int8)
    with pytest.raises(RMRCMError) as ei:
        L.rmrcm_step_noalloc(p, K, bt_big, q, bv, pd, fd)
    assert ei.value.status == -8
    # a non-positive permeability is found on the device
    Kbad = K.clone()
    Kbad[3, 5] = -1.0
    with pytest.raises(RMRCMError) as ei:
        L.rmrcm_step_noalloc(params(L, prob), Kbad, prob.bc_type, q, bv, pd, fd)
    assert ei.value.status == -1
    pn, Fn = noalloc(L, torch, prob)
    ref = mrcm_solve(prob)
    assert rel_l2(pn, ref.p) <= TOL and rel_l2(Fn, ref.F) <= TOL
