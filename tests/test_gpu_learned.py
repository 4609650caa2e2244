"""Learned mode (RMRCM_MIXED_LEARNED): the surrogate's bases behind the
FP64 residual gate.

A small network is trained on the GPU on pairs from the local solver, then
used by the solver: with gate_tol = 0 nothing is accepted and the result is
that of RMRCM_MIXED bit for bit; with an unbounded gate every interior
subdomain takes the network's basis; acceptance grows with gate_tol; and at
the strict gate the end-to-end flux error against the FP64 path stays
within 1e-6 (the errors at looser gates are printed).
"""

import os
import sys
import tempfile

import numpy as np
import pytest

from helpers import make_problem
from oracle.metrics import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def weights():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2009_07965_amd import Net, learned
    print("[gpu] learned: training a small surrogate", flush=True)
    x, t = learned.generate_pairs(6000, m=8, seed=4200)
    net = Net(16, 16, 5, 16, max_batch=128)
    d = tempfile.mkdtemp()
    path = os.path.join(d, "cnn16.bin")
    try:
        net.set_params(learned.init_params(16, 16, 5, 16, seed=2))
        learned.train(net, x, t, epochs=6, batch=128, lr=2e-3, seed=0)
        net.save(path)
    finally:
        net.close()
    yield path
    os.remove(path)
    os.rmdir(d)


def run(prob, **kw):
    from paper_2009_07965_amd import Solver
    S = Solver.from_problem(prob, **kw)
    try:
        p, F = S.solve(prob.q, prob.bc_value)
        st = S.stats()
    finally:
        S.close()
    return p, F, st


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


PROB = dict(nx=128, b=16, seg=4, log_var=3.0, lam=0.1, seed=31)


def test_strict_gate_equals_mixed(weights):
    from paper_2009_07965_amd import RMRCM_MIXED, RMRCM_MIXED_LEARNED
    prob = make_problem(PROB["nx"], b=PROB["b"], seg=PROB["seg"], log_var=PROB["log_var"],
                        lam=PROB["lam"], seed=PROB["seed"])
    say("[gpu] learned gate 0")
    p0, f0, st0 = run(prob, precision=RMRCM_MIXED_LEARNED, cnn_weights=weights.encode(), gate_tol=0.0)
    p1, f1, _ = run(prob, precision=RMRCM_MIXED)
    assert st0["surrogate_accepted_subdomains"] == 0
    assert np.array_equal(p0, p1) and np.array_equal(f0, f1)


def test_acceptance_and_error_against_gate(weights):
    from paper_2009_07965_amd import RMRCM_FP64, RMRCM_MIXED_LEARNED
    prob = make_problem(PROB["nx"], b=PROB["b"], seg=PROB["seg"], log_var=PROB["log_var"],
                        lam=PROB["lam"], seed=PROB["seed"])
    pr, fr, _ = run(prob, precision=RMRCM_FP64)
    acc, errs = [], []
    for tau in (1e-8, 1e-2, 1e-1, 1.0, 1e30):
        say("[gpu] learned gate %g" % tau)
        p, f, st = run(prob, precision=RMRCM_MIXED_LEARNED, cnn_weights=weights.encode(),
                       gate_tol=tau)
        acc.append(st["surrogate_accepted_subdomains"])
        errs.append(rel_l2(f, fr))
        say("    accepted %d of 36 interior subdomains, flux rel err vs FP64 %.3e" % (acc[-1], errs[-1]))
        assert np.all(np.isfinite(p)) and np.all(np.isfinite(f))
    assert acc == sorted(acc)               # monotone in the gate
    assert acc[-1] == 36                    # 8x8 subdomains: 6x6 interior ones
    assert errs[0] <= 1e-6                  # the strict gate keeps the 1e-6 target
