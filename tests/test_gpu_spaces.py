"""General MRCM interface spaces on the GPU (U_H and P_H piecewise constant
on segments of different lengths; Section 2 leaves them free, Section 4's
MuMM takes them equal) against the oracle's general non-recursive MRCM
(oracle.mrcm, pinned by the face-by-face brute force of oracle.monolithic).

The GPU path solves the local problems per piece (the shorter segment) and
restricts every merge to the spaces (the merge factor of k_merge.hip's
general-spaces path); the column kernels, the downward pass and the
reconstruction are those of the MuMM spaces.  Checked element by element
at the FP64 bar (pressures, fluxes, interface U and P per piece against the
oracle's per segment), for U coarser and P coarser, 8-, 16- and 32-cell
subdomains, Dirichlet, mixed and all-Neumann data and alpha over six
decades; merges of every column tier (gamma up to 256 pieces, the blocks in
global memory) on 512^2 and 1024^2 fields; the replayed step graph; the
mixed precision mode.
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
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2009_07965_amd as lib
    return lib


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(L, prob, **kw):
    S = L.Solver.from_problem(prob, **kw)
    try:
        p, F = S.solve(prob.q, prob.bc_value)
        U, P = S.interface()
    finally:
        S.close()
    return p, F, U, P


def check(prob, p, F, U, P, tol=TOL):
    ref = mrcm_solve(prob)
    dec = ref.dec
    ep, ef = rel_l2(p, ref.p), rel_l2(F, ref.F)
    eu = rel_l2(U, ref.U[dec.seg_useg])
    eP = rel_l2(P, ref.P[dec.seg_pseg])
    say("    p %.2e F %.2e U %.2e P %.2e" % (ep, ef, eu, eP))
    assert ep <= tol and ef <= tol, (ep, ef)
    assert eu <= 1e3 * tol and eP <= 1e3 * tol, (eu, eP)
    # U constant on every U-segment, P on every P-segment
    for arr, seg in ((U, dec.seg_useg), (P, dec.seg_pseg)):
        spread = np.zeros(seg.max() + 1)
        lo = np.full(seg.max() + 1, np.inf)
        hi = np.full(seg.max() + 1, -np.inf)
        np.minimum.at(lo, seg, arr)
        np.maximum.at(hi, seg, arr)
        assert (hi - lo).max() <= 1e-9 * max(np.abs(arr).max(), 1e-300)


CASES = [
    # n, b, seg_u, seg_p
    (64, 8, 4, 2), (64, 8, 2, 8),
    (128, 16, 8, 4), (128, 16, 4, 16), (128, 16, 16, 4),
    (256, 32, 16, 8), (256, 32, 8, 32),
]


@pytest.mark.parametrize("n,b,su,sp", CASES)
@pytest.mark.parametrize("bc", ["we", "mixed"])
def test_general_spaces_match_oracle(L, n, b, su, sp, bc):
    prob = make_problem(n, b=b, seg=min(su, sp), log_var=3.0, lam=0.1, seed=21 + n, bc=bc,
                        source=True).with_(seg_u=su, seg_p=sp)
    say("[gpu] spaces %d^2 b %d seg_u %d seg_p %d %s" % (n, b, su, sp, bc))
    check(prob, *run(L, prob))


@pytest.mark.parametrize("su,sp", [(8, 4), (4, 16)])
def test_general_spaces_all_neumann(L, su, sp):
    prob = make_problem(128, b=16, seg=4, log_var=2.0, seed=8, bc="fivespot").with_(seg_u=su, seg_p=sp)
    say("[gpu] spaces all-Neumann seg_u %d seg_p %d" % (su, sp))
    check(prob, *run(L, prob))


@pytest.mark.parametrize("alpha", [1e-3, 1e3])
def test_general_spaces_alpha(L, alpha):
    prob = make_problem(128, b=16, seg=4, alpha=alpha, log_var=3.0, seed=12,
                        source=True).with_(seg_u=16, seg_p=4)
    say("[gpu] spaces alpha %g" % alpha)
    check(prob, *run(L, prob))


@pytest.mark.parametrize("n,b,su,sp", [(512, 16, 8, 4), (1024, 16, 4, 8)])
def test_general_spaces_large_interfaces(L, n, b, su, sp):
    """Top interfaces of 128 (512^2) and 256 (1024^2) pieces."""
    prob = make_problem(n, b=b, seg=4, log_var=3.0, lam=0.1, seed=3, source=True).with_(seg_u=su, seg_p=sp)
    say("[gpu] spaces %d^2 seg_u %d seg_p %d" % (n, su, sp))
    check(prob, *run(L, prob))


def test_general_spaces_step_graph(L):
    """rmrcm_step on device arrays (the captured and replayed chain, the
    particular column carried through the merges) equals the oracle."""
    import torch
    prob = make_problem(256, b=32, seg=8, log_var=3.0, seed=17, source=True).with_(seg_u=32, seg_p=8)
    say("[gpu] spaces, step graph")
    d = torch.device("cuda:0")
    K = torch.from_numpy(prob.K).to(d)
    q = torch.from_numpy(prob.q).to(d)
    bv = torch.from_numpy(prob.bc_value).to(d)
    pd = torch.zeros((prob.ny, prob.nx), dtype=torch.float64, device=d)
    fd = torch.zeros((4, prob.ny, prob.nx), dtype=torch.float64, device=d)
    torch.cuda.synchronize()
    S = L.Solver.from_problem(prob)
    try:
        for _ in range(2):
            S.step(K, q, bv, pd, fd)
        S.sync()
        U, P = S.interface()
    finally:
        S.close()
    torch.cuda.synchronize()
    check(prob, pd.cpu().numpy(), fd.cpu().numpy(), U, P)


def test_general_spaces_mixed_precision(L):
    prob = make_problem(128, b=16, seg=4, log_var=3.0, seed=19, source=True).with_(seg_u=4, seg_p=16)
    say("[gpu] spaces, mixed precision")
    p, F, U, P = run(L, prob, precision=1)
    ref = mrcm_solve(prob)
    assert rel_l2(p, ref.p) <= 1e-9 and rel_l2(F, ref.F) <= 1e-9
