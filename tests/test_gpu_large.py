"""The benchmarked step at the large workloads' shapes.

``rmrcm_step`` replays one captured graph in which the particular problem
is carried as one more column through the local sweeps and through every
merge below the top (the column ``nslot`` of each trace matrix).  At the
interface sizes of the 1024^2, 2048^2 and 8192^2 workloads that column goes
through the 32-, 64- and 128-segment register tiers and, beyond 128
segments, through the merges whose blocks live in global memory.  Checked
here, in the launch configuration the benchmark times (device arrays, a
caller stream, autotuned merge column tiles, the replayed graph):

* against the oracle (plain non-recursive MRCM, FP64) element by element
  on grids it finishes in seconds: 512^2 and 1024^2 random fields with
  32^2 subdomains, the full 1024^2 workload, and 1024^2 crops of the
  2048^2 and 8192^2 fields with those workloads' subdomain and segment
  sizes (Algorithm 1 with eq. particular: the recursive result equals the
  non-recursive one to round-off);
* at the full 2048^2 and 8192^2 sizes, where the oracle cannot run, by
  properties that hold at any size: the cell-wise backward error of the
  mass balance (eq. 12.2), the interface conditions eq. 13.2 and eq. 14.2
  on the GPU's own fluxes and interface values, agreement of the step with
  a separate setup + solve (the particular chain of its own), and the
  pressure range [0, 1] of the Dirichlet data (observed on these fields:
  the fine scheme and every local Robin problem obey a discrete maximum
  principle, the coupled multiscale solution is not proven to).
"""

import sys

import numpy as np
import pytest

from helpers import make_problem
from oracle.metrics import rel_l2, cell_backward_error
from oracle.mrcm import mrcm_solve
from workloads import config_problem

pytestmark = pytest.mark.gpu

TOL = 1e-10
# step (particular column carried through the merges) vs setup + solve (a
# particular chain of its own): each is within about 1e-11 of the exact
# discrete solution on these fields, so they agree to that order
STEP_TOL = 1e-11


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


def crop(prob, n):
    """The n x n lower-left corner of a workload's field with its subdomain
    and segment sizes and the same boundary-condition pattern."""
    from workloads import dirichlet_we
    t, v = dirichlet_we(n, n)
    return prob.with_(nx=n, ny=n, K=np.ascontiguousarray(prob.K[:n, :n]),
                      q=np.zeros((n, n)), bc_type=t, bc_value=v)


def bench_step(L, torch, prob, autotune=True):
    """The benchmark's launch configuration: device arrays, a caller
    stream, autotuned merge tiles, rmrcm_step replayed as a graph (two
    steps, the second on the captured graph)."""
    d = torch.device("cuda:0")
    K = torch.from_numpy(prob.K).to(d)
    q = torch.from_numpy(prob.q).to(d)
    bv = torch.from_numpy(prob.bc_value).to(d)
    bt = torch.from_numpy(prob.bc_type).to(d)
    pd = torch.zeros((prob.ny, prob.nx), dtype=torch.float64, device=d)
    fd = torch.zeros((4, prob.ny, prob.nx), dtype=torch.float64, device=d)
    torch.cuda.synchronize()
    S = L.Solver(prob.nx, prob.ny, K, bt, prob.sub_nx, prob.sub_ny, prob.seg, alpha=prob.alpha)
    stream = torch.cuda.Stream()
    try:
        S.set_stream(stream.cuda_stream)
        if autotune:
            S.autotune()
        for _ in range(2):
            S.step(K, q, bv, pd, fd)
        S.sync()
        torch.cuda.synchronize()
        U, P = S.interface()
    finally:
        S.close()
    out = pd.cpu().numpy(), fd.cpu().numpy(), U, P
    del K, q, bv, bt, pd, fd
    torch.cuda.empty_cache()
    return out


def eager(L, prob):
    S = L.Solver.from_problem(prob)
    try:
        return S.solve(prob.q, prob.bc_value)
    finally:
        S.close()


def interface_residuals(prob, p, F, U):
    """Backward errors of eq. 13.2 (the sum of the two one-sided fluxes of a
    segment) and eq. 14.2 divided by beta (their difference minus 2 |e| U)
    for every segment (documented order): each residual divided by the size
    of the terms that cancel in it, the segment's Robin face conductances
    |f| / (rho + beta) on both sides times max |p| (the one-sided fluxes
    are those conductances times pressure differences)."""
    nx, ny, bx, by, sg = prob.nx, prob.ny, prob.sub_nx, prob.sub_ny, prob.seg
    mx, my = nx // bx, ny // by
    hx, hy = prob.lx / nx, prob.ly / ny
    K = prob.K
    # vertical lines I = 1..mx-1: E faces of column I bx - 1, W faces of I bx
    flo_v = F[1][:, bx - 1:nx - 1:bx].reshape(ny // sg, sg, mx - 1).sum(1).T.ravel()
    fhi_v = F[0][:, bx:nx:bx].reshape(ny // sg, sg, mx - 1).sum(1).T.ravel()
    flo_h = F[3][by - 1:ny - 1:by, :].reshape(my - 1, nx // sg, sg).sum(2).ravel()
    fhi_h = F[2][by:ny:by, :].reshape(my - 1, nx // sg, sg).sum(2).ravel()

    # conductance sums per segment
    klo = K[:, bx - 1:nx - 1:bx]                      # (ny, mx-1)
    khi = K[:, bx:nx:bx]
    keff = (2 * klo * khi / (klo + khi)).reshape(ny // sg, sg, mx - 1).mean(1)   # (lines, mx-1)
    beta = prob.alpha * sg * hy / keff
    bf = np.repeat(beta, sg, axis=0)                  # per face (ny, mx-1)
    cs_v = (hy / (hx / (2 * klo) + bf) + hy / (hx / (2 * khi) + bf))
    cs_v = cs_v.reshape(ny // sg, sg, mx - 1).sum(1).T.ravel()
    klo = K[by - 1:ny - 1:by, :]                      # (my-1, nx)
    khi = K[by:ny:by, :]
    keff = (2 * klo * khi / (klo + khi)).reshape(my - 1, nx // sg, sg).mean(2)
    beta = prob.alpha * sg * hx / keff
    bf = np.repeat(beta, sg, axis=1)
    cs_h = (hx / (hy / (2 * klo) + bf) + hx / (hy / (2 * khi) + bf))
    cs_h = cs_h.reshape(my - 1, nx // sg, sg).sum(2).ravel()
    flo = np.concatenate([flo_v, flo_h])
    fhi = np.concatenate([fhi_v, fhi_h])
    scale = np.concatenate([cs_v, cs_h]) * np.abs(p).max()
    length = np.concatenate([np.full(flo_v.size, sg * hy), np.full(flo_h.size, sg * hx)])
    r13 = (np.abs(flo + fhi) / scale).max()
    r14 = (np.abs(flo - fhi - 2.0 * length * U) / scale).max()
    return r13, r14


@pytest.mark.parametrize("n", [512, 1024])
def test_step_32_64_128_segment_tiers_match_oracle(env, n):
    """32^2 subdomains with 8-cell segments: interfaces of 4 .. n/8 segments,
    i.e. the 32-, 64- and (at 1024^2) 128-segment merges carrying the
    particular column inside the replayed step."""
    L, torch = env
    prob = make_problem(n, b=32, seg=8, log_var=4.0, lam=0.05, seed=70 + n, source=True)
    say("[gpu] step tiers n %d" % n)
    p, F, U, P = bench_step(L, torch, prob)
    pe, Fe = eager(L, prob)
    assert rel_l2(p, pe) <= STEP_TOL and rel_l2(F, Fe) <= STEP_TOL
    ref = mrcm_solve(prob)
    assert rel_l2(p, ref.p) <= TOL, rel_l2(p, ref.p)
    assert rel_l2(F, ref.F) <= TOL, rel_l2(F, ref.F)
    assert rel_l2(P, ref.P) <= TOL


def test_benchmarked_step_full_1024_matches_oracle(env):
    """The 1024^2 workload exactly as the benchmark times it."""
    L, torch = env
    prob = config_problem(2)
    say("[gpu] benchmarked step, full 1024^2")
    p, F, U, P = bench_step(L, torch, prob)
    ref = mrcm_solve(prob)
    assert rel_l2(p, ref.p) <= TOL, rel_l2(p, ref.p)
    assert rel_l2(F, ref.F) <= TOL, rel_l2(F, ref.F)
    assert rel_l2(P, ref.P) <= TOL
    assert cell_backward_error(prob, p, F) < 1e-12


@pytest.fixture(scope="module")
def big():
    return {}


def workload(big, k):
    if k not in big:
        say("[gpu] generating workload %d" % k)
        big[k] = config_problem(k)
    return big[k]


@pytest.mark.parametrize("k", [4, 5])
def test_crop_of_large_workload_matches_oracle(env, big, k):
    """1024^2 crops of the 2048^2 (16^2 subdomains, 4-cell segments: top
    interfaces of 256 segments, the global-memory merges) and 8192^2
    (channel field, 32^2 subdomains, 8-cell segments) workloads."""
    L, torch = env
    prob = crop(workload(big, k), 1024)
    say("[gpu] crop of workload %d" % k)
    p, F, U, P = bench_step(L, torch, prob)
    ref = mrcm_solve(prob)
    assert rel_l2(p, ref.p) <= TOL, rel_l2(p, ref.p)
    assert rel_l2(F, ref.F) <= TOL, rel_l2(F, ref.F)
    assert rel_l2(P, ref.P) <= TOL


@pytest.mark.parametrize("k", [4, 5])
def test_full_size_invariants(env, big, k):
    """Full 2048^2 (14 levels, top interface 512 segments) and 8192^2
    (16 levels, 67M cells, top interface 1024 segments)."""
    L, torch = env
    prob = workload(big, k)
    say("[gpu] full workload %d: step" % k)
    p, F, U, P = bench_step(L, torch, prob)
    assert np.isfinite(p).all() and np.isfinite(F).all()
    assert cell_backward_error(prob, p, F) < 1e-12
    r13, r14 = interface_residuals(prob, p, F, U)
    say("[gpu] interface backward errors %.3e %.3e" % (r13, r14))
    assert r13 < 1e-12 and r14 < 1e-12, (r13, r14)
    assert p.min() >= -1e-9 and p.max() <= 1.0 + 1e-9, (p.min(), p.max())
    say("[gpu] full workload %d: setup + solve" % k)
    pe, Fe = eager(L, prob)
    assert rel_l2(p, pe) <= STEP_TOL and rel_l2(F, Fe) <= STEP_TOL
    if k == 5:
        del big[k]


def test_step_single_subdomain(env):
    """One subdomain with Dirichlet faces (no merge, no interface): the step
    is the local solve alone, and equals the oracle (the fine solve)."""
    L, torch = env
    prob = make_problem(32, b=32, seg=8, source=True, log_var=2.0)
    say("[gpu] step, one subdomain")
    p, F, U, P = bench_step(L, torch, prob, autotune=False)
    ref = mrcm_solve(prob)
    assert rel_l2(p, ref.p) <= TOL and rel_l2(F, ref.F) <= TOL
