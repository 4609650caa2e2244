"""The seeded input generators: determinism and the statistics they
promise (zero-mean, unit-variance exponential-covariance field)."""

import numpy as np

from workloads import gaussian_field_exp, lognormal_grf, channelized, ensemble_member, config_problem


def test_grf_deterministic_and_seeded():
    a = gaussian_field_exp(64, 32, 0.1, seed=5)
    b = gaussian_field_exp(64, 32, 0.1, seed=5)
    c = gaussian_field_exp(64, 32, 0.1, seed=6)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.shape == (32, 64)


def test_grf_statistics():
    """Pointwise mean ~0 and variance ~1 over many samples; the lag-one
    correlation along x matches exp(-h / lam)."""
    n, lam = 64, 0.1
    xs = np.stack([gaussian_field_exp(n, n, lam, seed=s) for s in range(200)])
    assert abs(xs.mean()) < 0.05
    assert abs(xs.var() - 1.0) < 0.08
    h = 1.0 / n
    corr = np.mean(xs[:, :, 1:] * xs[:, :, :-1]) / xs.var()
    assert abs(corr - np.exp(-h / lam)) < 0.03


def test_lognormal_and_channel_fields_positive():
    K = lognormal_grf(32, 32, 0.05, 4.0, seed=2)
    assert np.all(K > 0) and np.all(np.isfinite(K))
    C = channelized(128, seed=5)
    assert np.all(C > 0)
    lk = np.log(C)
    # bimodal: most cells near log 1 or log 1000
    near = (np.abs(lk) < 1.5) | (np.abs(lk - np.log(1000)) < 1.5)
    assert near.mean() > 0.97
    assert (np.abs(lk - np.log(1000)) < 1.5).mean() > 0.05


def test_configs_and_ensemble_members():
    P = config_problem(1)
    assert P.K.shape == (64, 64) and P.sub_nx == 16 and P.seg == 4
    m = ensemble_member(0)
    assert m.nx in (128, 256, 512) and m.sub_nx in (8, 16, 32)
    assert m.seg == m.sub_nx // 4
    assert abs(m.q.sum()) < 1e-15 and np.all(m.bc_type == 0)
