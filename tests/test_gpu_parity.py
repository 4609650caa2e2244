"""FP64 GPU path (through the C ABI) against the CPU oracle.

Element by element on the same seeded inputs: cell pressures and the four
one-sided outward face fluxes of every cell, plus the interface values
(U, P) per segment.  Bar: relative L2 error <= 1e-10 for pressure and flux
(the FP64 target), 1e-9 for U (it is a difference of the two one-sided
Robin data divided by 2 beta).

Sizes: the oracle finishes each case in seconds; cases span many
subdomains, every supported subdomain width, rectangular grids and
subdomains, segment lengths from one face to a whole side, the degenerate
single-subdomain and two-subdomain decompositions, interfaces of 256 to 1024
segments (the merges whose blocks exceed one workgroup's registers), and the
full 1024^2
workload (32^2 subdomains of 32^2 cells, 10 levels) in the launch
configuration the benchmark times.
"""

import sys

import numpy as np
import pytest

from helpers import make_problem
from oracle.fine import fine_solve
from oracle.metrics import rel_l2, cell_balance, cell_backward_error, interface_residual
from oracle.mrcm import mrcm_solve
from workloads import config_problem

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def Solver():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2009_07965_amd import Solver as S
    return S


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(Solver, prob, name):
    say("[gpu] %s nx=%d ny=%d sub=%dx%d seg=%d alpha=%g" % (
        name, prob.nx, prob.ny, prob.sub_nx, prob.sub_ny, prob.seg, prob.alpha))
    S = Solver.from_problem(prob)
    try:
        p, F = S.solve(prob.q, prob.bc_value)
        U, P = S.interface()
    finally:
        S.close()
    return p, F, U, P


CASES = {
    "cfg1_64": lambda: config_problem(1),
    "tiny_b4_seg2": lambda: make_problem(8, b=4, seg=2),
    "tiny_b4_seg1": lambda: make_problem(8, b=4, seg=1, alpha=0.3),
    "tiny_b4_seg4": lambda: make_problem(8, b=4, seg=4, alpha=10.0),
    "rect_64x32_b16": lambda: make_problem(64, ny=32, b=16, seg=4, log_var=2.0),
    "rect_sub_16x8": lambda: make_problem(64, ny=64, b=16, by=8, seg=4, source=True),
    "rect_sub_8x32": lambda: make_problem(32, ny=128, b=8, by=32, seg=4, bc="mixed"),
    "b32_128": lambda: make_problem(128, b=32, seg=8, log_var=3.0, lam=0.1),
    "b8_64x128_src_mixed": lambda: make_problem(64, ny=128, b=8, seg=2, source=True,
                                                bc="mixed", log_var=2.0),
    "b32_seg1": lambda: make_problem(64, b=32, seg=1, log_var=1.0),
    "alpha_1e3": lambda: make_problem(64, b=16, seg=4, alpha=1e3),
    "alpha_1e-2": lambda: make_problem(64, b=16, seg=4, alpha=1e-2),
    "high_contrast": lambda: make_problem(64, b=16, seg=4, log_var=9.0, lam=0.05),
    "two_subdomains": lambda: make_problem(64, ny=32, b=32, seg=8),
    "two_subdomains_y": lambda: make_problem(32, ny=64, b=32, seg=16, source=True),
    "single_subdomain": lambda: make_problem(32, b=32, seg=8, source=True),
    "all_neumann_fivespot_b8": lambda: make_problem(64, b=8, seg=2, bc="fivespot", log_var=2.0),
    "all_neumann_fivespot_b32": lambda: make_problem(256, b=32, seg=8, bc="fivespot", log_var=3.0),
    "all_neumann_fivespot_big_root": lambda: make_problem(256, b=8, seg=2, bc="fivespot",
                                                          log_var=1.0, lam=0.1),
    # ten levels of 16-cell subdomains with 4-cell segments: merges of up to
    # 16 segments fused per level, 32 and 64 with the column apply and
    # traces fused (row tiles over two and three workgroups), the deepest
    # five depths of the downward pass in one launch
    "b16_512_seg4": lambda: make_problem(512, b=16, seg=4, log_var=3.0, lam=0.05),
    "rect_512x256_b16_src": lambda: make_problem(512, ny=256, b=16, seg=4, source=True, log_var=2.0),
    # 256 gamma segments at the two top levels: the merges with blocks in
    # global memory (2 x 2 split inverses, matrix-product applies)
    "gamma256": lambda: make_problem(256, b=8, seg=1, log_var=2.0, lam=0.1, source=True),
    "gamma256_all_neumann": lambda: make_problem(256, b=8, seg=1, bc="fivespot", log_var=1.0,
                                                 lam=0.1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp64_matches_oracle(Solver, name):
    prob = CASES[name]()
    ref = mrcm_solve(prob)
    p, F, U, P = run_gpu(Solver, prob, name)
    assert rel_l2(p, ref.p) <= TOL, rel_l2(p, ref.p)
    assert rel_l2(F, ref.F) <= TOL, rel_l2(F, ref.F)
    if ref.dec.nseg:
        assert rel_l2(P, ref.P) <= TOL
        assert rel_l2(U, ref.U) <= 10 * TOL


@pytest.mark.parametrize("b", [4, 8, 32])
def test_seg1_equals_fine_solution(Solver, b):
    """One fine face per segment: the method reproduces the fine solve."""
    prob = make_problem(64, b=b, seg=1, log_var=2.0, source=True)
    pf, Ff = fine_solve(prob)
    p, F, U, P = run_gpu(Solver, prob, "seg1_b%d" % b)
    assert rel_l2(p, pf) <= TOL and rel_l2(F, Ff) <= TOL


@pytest.mark.parametrize("nx,ny,b,bc", [(512, 512, 16, "we"), (1024, 512, 32, "we"),
                                        (512, 512, 16, "fivespot"), (1024, 1024, 32, "we")])
def test_long_gamma_seg1_equals_fine_solution(Solver, nx, ny, b, bc):
    """Interfaces of 512 and 1024 segments (one fine face each) at the top
    levels: the merges with blocks in global memory (recursively split
    inverses, matrix-product applies and parent traces) reproduce the fine
    solve, with Dirichlet data and all-Neumann (the pinned top)."""
    prob = make_problem(nx, ny=ny, b=b, seg=1, log_var=2.0, lam=0.1, source=(bc == "we"), bc=bc)
    pf, Ff = fine_solve(prob)
    p, F, U, P = run_gpu(Solver, prob, "gamma_long_%dx%d_b%d_%s" % (nx, ny, b, bc))
    assert rel_l2(p, pf) <= TOL, rel_l2(p, pf)
    assert rel_l2(F, Ff) <= TOL, rel_l2(F, Ff)


def test_invariants_on_gpu_output(Solver):
    """Per-cell conservation and the interface equations eq. 13.2 / 14.2 on
    the GPU's own output."""
    prob = make_problem(128, b=16, seg=4, log_var=3.0, source=True, bc="mixed")
    p, F, U, P = run_gpu(Solver, prob, "invariants")
    assert cell_balance(F, prob.q) < 1e-12
    from oracle.decomp import Decomposition
    r13, r14 = interface_residual(Decomposition(prob), F, U)
    assert r13 < 1e-12 and r14 < 1e-11


def test_context_reuse_many_right_hand_sides(Solver):
    """One setup, several solves with different sources and boundary data."""
    prob = make_problem(64, b=16, seg=4, log_var=2.0)
    S = Solver.from_problem(prob)
    try:
        rng = np.random.default_rng(0)
        for k in range(3):
            q = rng.standard_normal(prob.q.shape) / prob.ncells
            bcv = prob.bc_value.copy()
            bcv[:prob.ny] = 1.0 + k
            pr = prob.with_(q=q, bc_value=bcv)
            say("[gpu] reuse solve %d" % k)
            p, F = S.solve(q, bcv)
            ref = mrcm_solve(pr)
            assert rel_l2(p, ref.p) <= TOL and rel_l2(F, ref.F) <= TOL
    finally:
        S.close()


def test_device_pointers_and_reproducibility(Solver):
    """Inputs and outputs as device tensors give the host result, and two
    runs agree bit for bit (no floating-point atomics)."""
    import torch
    prob = make_problem(128, b=32, seg=8, log_var=2.0, source=True)
    say("[gpu] device pointers")
    dev = torch.device("cuda:0")
    K = torch.from_numpy(prob.K).to(dev)
    bt = torch.from_numpy(prob.bc_type).to(dev)
    S = Solver(prob.nx, prob.ny, K, bt, prob.sub_nx, prob.sub_ny, prob.seg, alpha=prob.alpha)
    try:
        q = torch.from_numpy(prob.q).to(dev)
        bv = torch.from_numpy(prob.bc_value).to(dev)
        pd = torch.zeros((prob.ny, prob.nx), dtype=torch.float64, device=dev)
        fd = torch.zeros((4, prob.ny, prob.nx), dtype=torch.float64, device=dev)
        S.solve(q, bv, pd, fd)
        torch.cuda.synchronize()
        p1, F1 = pd.cpu().numpy().copy(), fd.cpu().numpy().copy()
        S.solve(q, bv, pd, fd)
        torch.cuda.synchronize()
        assert np.array_equal(p1, pd.cpu().numpy()) and np.array_equal(F1, fd.cpu().numpy())
    finally:
        S.close()
    ph, Fh, _u, _p = run_gpu(Solver, prob, "host pointers")
    assert np.array_equal(ph, p1) and np.array_equal(Fh, F1)


def test_full_size_1024(Solver):
    """The 1024^2 workload (32x32 subdomains of 32^2 cells, 8-cell segments,
    10 levels) compared element by element with the oracle."""
    prob = config_problem(2)
    ref = mrcm_solve(prob)
    p, F, U, P = run_gpu(Solver, prob, "full 1024^2")
    assert rel_l2(p, ref.p) <= TOL, rel_l2(p, ref.p)
    assert rel_l2(F, ref.F) <= TOL, rel_l2(F, ref.F)
    assert rel_l2(P, ref.P) <= TOL
    # conservation: backward error per cell (contrast ~5e6 here)
    assert cell_backward_error(prob, p, F) < 1e-12
    assert cell_backward_error(prob, ref.p, ref.F) < 1e-12


def test_async_refactor_new_field(Solver):
    """rmrcm_refactor is asynchronous; a solve that returns host arrays waits
    for it and gives the oracle's answer for the new field."""
    p1 = make_problem(128, b=16, seg=4, log_var=2.0, seed=11)
    p2 = make_problem(128, b=16, seg=4, log_var=4.0, lam=0.05, seed=12, source=True)
    S = Solver.from_problem(p1)
    try:
        say("[gpu] async refactor")
        S.refactor(p2.K, wait=False)
        p, F = S.solve(p2.q, p2.bc_value)
        ref = mrcm_solve(p2)
        assert rel_l2(p, ref.p) <= TOL and rel_l2(F, ref.F) <= TOL
    finally:
        S.close()


def test_bad_permeability_reported_at_sync(Solver):
    """A non-positive permeability passed to refactor is found on the device
    and returned by the next sync (EINVAL); the next valid refactor
    restores the context."""
    from paper_2009_07965_amd import RMRCMError
    prob = make_problem(64, b=16, seg=4, log_var=1.0)
    S = Solver.from_problem(prob)
    try:
        say("[gpu] bad permeability")
        Kbad = prob.K.copy()
        Kbad[5, 7] = -1.0
        S.refactor(Kbad, wait=False)
        with pytest.raises(RMRCMError) as ei:
            S.sync()
        assert ei.value.status == -1
        S.sync()                                   # the status was consumed
        S.refactor(prob.K)
        p, F = S.solve(prob.q, prob.bc_value)
        ref = mrcm_solve(prob)
        assert rel_l2(p, ref.p) <= TOL and rel_l2(F, ref.F) <= TOL
    finally:
        S.close()
