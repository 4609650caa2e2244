"""Learned mode (RMRCM_MIXED_LEARNED): the surrogate's bases behind the
FP64 residual gate.

A small network is trained on the GPU on pairs from the local solver, then
used by the solver.  An accepted prediction (gate residual within
gate_tol) is the starting iterate of the FP64-residual refinement of its
subdomain, so every basis still meets ir_tol.  Checked here:

* the gate residual of every subdomain, read back through rmrcm_get_gate,
  against the residual of the local Robin system built by the oracle
  (oracle.local's face conductances and transmissibilities) for the
  prediction of the oracle's network (oracle/cnn.py, FP64, same weights,
  on the oracle's features): the two networks differ by FP32 rounding only;
* with every interior subdomain accepted, the solution against the oracle
  MRCM at the mixed bar;
* gate_tol = 0 accepts nothing and gives RMRCM_MIXED bit for bit;
  acceptance grows with the gate, and the flux error against the FP64 path
  stays within 1e-6 at every gate (the refinement takes the accepted
  predictions to ir_tol).
"""

import os
import sys
import tempfile

import numpy as np
import pytest

from helpers import make_problem
from oracle import cnn as ref_cnn
from oracle.decomp import Decomposition
from oracle.local import local_solve
from oracle.metrics import rel_l2
from oracle.mrcm import mrcm_solve
from oracle.tpfa import block_matrix

pytestmark = pytest.mark.gpu

S_, C_, L_, R_ = 16, 16, 5, 16
MIXED_TOL = 1e-9


@pytest.fixture(scope="module")
def weights():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2009_07965_amd import Net, learned
    print("[gpu] learned: training a small surrogate", flush=True)
    x, t = learned.generate_pairs(6000, m=8, seed=4200)
    net = Net(S_, C_, L_, R_, max_batch=128)
    d = tempfile.mkdtemp()
    path = os.path.join(d, "cnn16.bin")
    try:
        net.set_params(learned.init_params(S_, C_, L_, R_, seed=2))
        learned.train(net, x, t, epochs=6, batch=128, lr=2e-3, seed=0)
        net.save(path)
    finally:
        net.close()
    yield path
    os.remove(path)
    os.rmdir(d)


def run(prob, **kw):
    from paper_2009_07965_amd import Solver, rmrcm_get_gate, RMRCM_MIXED_LEARNED
    S = Solver.from_problem(prob, **kw)
    try:
        p, F = S.solve(prob.q, prob.bc_value)
        st = S.stats()
        gate = None
        if kw.get("precision") == RMRCM_MIXED_LEARNED:
            gate = rmrcm_get_gate(S.ctx, (prob.nx // prob.sub_nx) * (prob.ny // prob.sub_ny))
    finally:
        S.close()
    return p, F, st, gate


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


PROB = dict(nx=128, b=16, seg=4, log_var=3.0, lam=0.1, seed=31)


def problem():
    return make_problem(PROB["nx"], b=PROB["b"], seg=PROB["seg"], log_var=PROB["log_var"],
                        lam=PROB["lam"], seed=PROB["seed"])


def test_gate_residuals_match_oracle(weights):
    """Gate residual of every interior subdomain vs the oracle's |A y - e| /
    |e| for the oracle network's prediction on the oracle's features."""
    from paper_2009_07965_amd import Net, RMRCM_MIXED_LEARNED
    prob = problem()
    say("[gpu] learned gate residuals")
    _p, _F, st, (gres, acc) = run(prob, precision=RMRCM_MIXED_LEARNED, cnn_weights=weights.encode(),
                                  gate_tol=1e30)
    net = Net.load(weights, max_batch=8)
    try:
        theta = net.get_params().astype(np.float64)
    finally:
        net.close()
    dec = Decomposition(prob)
    b = prob.sub_nx
    checked = 0
    for J in range(dec.my):
        for I in range(dec.mx):
            k = J * dec.mx + I
            slots = dec.subdomain_slots(I, J)
            if any(e < 0 for (e, *_r) in slots):
                assert np.isinf(gres[k]) and acc[k] == 0
                continue
            beta = np.array([dec.seg_beta[e] for (e, *_r) in slots]).reshape(4, b // prob.seg)
            x = ref_cnn.features(prob.K[J * b:(J + 1) * b, I * b:(I + 1) * b], beta, prob.seg)
            y, _ = ref_cnn.forward(theta, x[None], S_, C_, L_, R_)
            y = y[0].reshape(R_, b * b)
            r = local_solve(prob, dec, I, J, with_particular=False)
            A = block_matrix(r.tx, r.ty, r.robin_c.sum(axis=2) + r.ext_c.sum(axis=2))
            worst = 0.0
            for a, (e, _sg, side, s) in enumerate(r.slots):
                ea = np.zeros(b * b)
                t = np.arange(s * prob.seg, (s + 1) * prob.seg)
                cells = ([(0, j) for j in t] if side == 0 else [(b - 1, j) for j in t] if side == 1
                         else [(i, 0) for i in t] if side == 2 else [(i, b - 1) for i in t])
                for (i, j) in cells:
                    ea[j * b + i] += r.robin_c[j, i, side]
                worst = max(worst, np.linalg.norm(A @ y[a] - ea) / np.linalg.norm(ea))
            assert abs(gres[k] - worst) <= 1e-4 * worst, (I, J, gres[k], worst)
            assert acc[k] == 1
            checked += 1
    assert checked == 36 and st["surrogate_accepted_subdomains"] == 36


def test_accepted_predictions_refined_match_oracle(weights):
    """Every interior subdomain starts its refinement from the prediction;
    the result meets the mixed bar against the oracle."""
    from paper_2009_07965_amd import RMRCM_MIXED_LEARNED
    prob = problem()
    say("[gpu] learned, all accepted")
    p, F, st, (gres, acc) = run(prob, precision=RMRCM_MIXED_LEARNED, cnn_weights=weights.encode(),
                                gate_tol=1e30)
    ref = mrcm_solve(prob)
    ep, ef = rel_l2(p, ref.p), rel_l2(F, ref.F)
    say("    accepted %d, ir %s/%s, p %.2e F %.2e" % (acc.sum(), st["ir_iters_setup"],
                                                     st["ir_iters_solve"], ep, ef))
    assert acc.sum() == 36 and st["surrogate_accepted_subdomains"] == 36
    assert ep <= MIXED_TOL and ef <= MIXED_TOL


def test_strict_gate_equals_mixed(weights):
    from paper_2009_07965_amd import RMRCM_MIXED, RMRCM_MIXED_LEARNED
    prob = problem()
    say("[gpu] learned gate 0")
    p0, f0, st0, _g = run(prob, precision=RMRCM_MIXED_LEARNED, cnn_weights=weights.encode(), gate_tol=0.0)
    p1, f1, _, _g = run(prob, precision=RMRCM_MIXED)
    assert st0["surrogate_accepted_subdomains"] == 0
    assert np.array_equal(p0, p1) and np.array_equal(f0, f1)


def test_acceptance_and_error_against_gate(weights):
    from paper_2009_07965_amd import RMRCM_FP64, RMRCM_MIXED_LEARNED
    prob = problem()
    pr, fr, _, _g = run(prob, precision=RMRCM_FP64)
    acc, errs = [], []
    for tau in (1e-8, 1e-1, 0.5, 1.0, 1e30):
        say("[gpu] learned gate %g" % tau)
        p, f, st, _g = run(prob, precision=RMRCM_MIXED_LEARNED, cnn_weights=weights.encode(),
                           gate_tol=tau)
        acc.append(st["surrogate_accepted_subdomains"])
        errs.append(rel_l2(f, fr))
        say("    accepted %d of 36 interior subdomains, ir %s/%s, flux rel err vs FP64 %.3e"
            % (acc[-1], st["ir_iters_setup"], st["ir_iters_solve"], errs[-1]))
        assert np.all(np.isfinite(p)) and np.all(np.isfinite(f))
    assert acc == sorted(acc)               # monotone in the gate
    assert acc[-1] == 36                    # 8x8 subdomains: 6x6 interior ones
    assert max(errs) <= 1e-6                # refined to ir_tol at every gate
