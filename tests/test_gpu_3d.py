"""The 3D method on the GPU (the paper's experiments: seven-point scheme,
columns of sub_nx x sub_ny x nz cells with no z-division, Hbar_z = H_z)
against the 3D oracle (oracle/three_d.py: the plain non-recursive MRCM on
the columns' local problems, pinned by closed forms, the 2D method on
z-independent problems and a face-by-face brute force), element by
element at the FP64 bar: pressures, the six one-sided fluxes of every
cell, and the interface U and P.  Columns whose row blocks have 16 to 64
cells (sub_nx * nz), Dirichlet, mixed and all-Neumann data, alpha over six
decades, the replayed step on device arrays, and a 256 x 256 x 8 grid of
1024 columns (interfaces up to 128 segments)."""

import sys

import numpy as np
import pytest

from helpers import make_problem3d
from oracle.metrics import rel_l2
from oracle.three_d import mrcm_solve3d

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


def check(prob, p, F, U, P, tol=TOL):
    rp, rF, rU, rP, _dec = mrcm_solve3d(prob)
    ep, ef = rel_l2(p, rp), rel_l2(F, rF)
    eu, eP = rel_l2(U, rU), rel_l2(P, rP)
    say("    p %.2e F %.2e U %.2e P %.2e" % (ep, ef, eu, eP))
    assert ep <= tol and ef <= tol, (ep, ef)
    assert eu <= 100 * tol and eP <= 100 * tol, (eu, eP)


def run(L, prob):
    S = L.Solver.from_problem(prob)
    try:
        p, F = S.solve(prob.q, prob.bc_value)
        U, P = S.interface()
    finally:
        S.close()
    return p, F, U, P


SHAPES = [
    # nx, ny, nz, b, seg
    (16, 16, 3, 8, 2), (32, 32, 4, 8, 4), (32, 32, 8, 8, 2), (64, 64, 4, 16, 4), (64, 64, 2, 32, 8),
    (32, 64, 16, 4, 2),
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("bc", ["we", "mixed"])
def test_3d_matches_oracle(L, shape, bc):
    nx, ny, nz, b, seg = shape
    prob = make_problem3d(nx, ny, nz, b=b, seg=seg, bc=bc, seed=nx + nz)
    say("[gpu] 3d %dx%dx%d b %d seg %d %s" % (nx, ny, nz, b, seg, bc))
    check(prob, *run(L, prob))


def test_3d_all_neumann(L):
    prob = make_problem3d(32, 32, 4, b=8, seg=4, bc="neumann")
    say("[gpu] 3d all-Neumann")
    check(prob, *run(L, prob))


@pytest.mark.parametrize("alpha", [1e-3, 1e3])
def test_3d_alpha(L, alpha):
    prob = make_problem3d(32, 32, 4, b=8, seg=4, alpha=alpha, log_var=3.0)
    say("[gpu] 3d alpha %g" % alpha)
    check(prob, *run(L, prob))


def test_3d_step_graph(L):
    import torch
    prob = make_problem3d(64, 64, 4, b=16, seg=4, seed=9)
    say("[gpu] 3d step graph")
    d = torch.device("cuda:0")
    K = torch.from_numpy(prob.K).to(d)
    q = torch.from_numpy(prob.q).to(d)
    bv = torch.from_numpy(prob.bc_value).to(d)
    pd = torch.zeros(prob.K.shape, dtype=torch.float64, device=d)
    fd = torch.zeros((6,) + prob.K.shape, dtype=torch.float64, device=d)
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


def test_3d_larger_grid(L):
    prob = make_problem3d(256, 256, 8, b=8, seg=4, log_var=3.0, lam=0.1, seed=5)
    say("[gpu] 3d 256x256x8")
    check(prob, *run(L, prob))
