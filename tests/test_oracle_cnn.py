"""Pins of the CPU reference network (oracle/cnn.py) against independent
definitions: SciPy's 2D correlation, central differences of the loss,
torch's bfloat16 rounding, and the scale invariance of the features."""

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def test_conv3x3_matches_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 7, 7))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = cnn.conv3x3(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, c], W[o, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.allclose(y[n, o], ref, rtol=0, atol=1e-12)


def test_conv3x3_delta_kernel_is_a_shift():
    x = np.arange(25.0).reshape(1, 1, 5, 5)
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 1, 2] = 1.0          # reads the right neighbour
    y = cnn.conv3x3(x, W, np.zeros(1))
    assert np.array_equal(y[0, 0, :, :-1], x[0, 0, :, 1:])
    assert np.all(y[0, 0, :, -1] == 0.0)


def test_conv_gradients_central_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 5))
    W = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    dy = rng.standard_normal((2, 2, 5, 5))
    f = lambda xx, WW, bb: float(np.sum(dy * cnn.conv3x3(xx, WW, bb)))  # noqa: E731
    gx, gW, gb = cnn.conv3x3_grads(x, W, dy)
    h = 1e-6
    for idx in [(0, 1, 2, 3), (1, 0, 0, 0), (1, 2, 4, 4)]:
        e = np.zeros_like(x); e[idx] = h
        assert abs((f(x + e, W, b) - f(x - e, W, b)) / (2 * h) - gx[idx]) < 1e-7
    for idx in [(0, 1, 0, 2), (1, 2, 1, 1)]:
        e = np.zeros_like(W); e[idx] = h
        assert abs((f(x, W + e, b) - f(x, W - e, b)) / (2 * h) - gW[idx]) < 1e-7
    e = np.zeros_like(b); e[1] = h
    assert abs((f(x, W, b + e) - f(x, W, b - e)) / (2 * h) - gb[1]) < 1e-7


def test_network_gradient_central_differences():
    S, C, L, R = 6, 4, 3, 5
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(cnn.num_params(S, C, L, R)) * 0.3
    x = rng.standard_normal((3, 2, S, S))
    t = rng.standard_normal((3, R, S, S))
    loss, g = cnn.loss_and_grad(theta, x, t, S, C, L, R, round_weights=False)
    h = 1e-6
    for k in rng.choice(theta.size, 25, replace=False):
        e = np.zeros_like(theta); e[k] = h
        lp, _ = cnn.loss_and_grad(theta + e, x, t, S, C, L, R, round_weights=False)
        lm, _ = cnn.loss_and_grad(theta - e, x, t, S, C, L, R, round_weights=False)
        assert abs((lp - lm) / (2 * h) - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k


def test_bf16_rounding_matches_torch_and_ties_to_even():
    torch = pytest.importorskip("torch")
    one = 1.0
    cases = np.array([one, one + 2.0 ** -8, one + 2.0 ** -8 + 2.0 ** -20,
                      one + 2.0 ** -7 + 2.0 ** -8, -3.14159, 1e-20, 65504.0], dtype=np.float32)
    r = cnn.bf16_round(cases)
    assert r[0] == 1.0 and r[1] == 1.0                       # tie to even (down)
    assert r[2] == 1.0 + 2.0 ** -7                          # above the tie
    assert r[3] == 1.0 + 2.0 ** -6                          # tie to even (up)
    rng = np.random.default_rng(3)
    v = (rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(v), ref)


def test_features_scale_invariance_and_homogeneous_patch():
    rng = np.random.default_rng(4)
    K = np.exp(rng.standard_normal((8, 8)))
    beta = np.exp(rng.standard_normal((4, 2)))
    f1 = cnn.features(K, beta, 4)
    f2 = cnn.features(7.5 * K, beta / 7.5, 4)
    assert np.allclose(f1, f2, atol=1e-13)
    fh = cnn.features(np.full((8, 8), 3.0), np.full((4, 2), 0.5), 4)
    assert np.all(fh[0] == 0.0)
    assert np.allclose(fh[1][0, :], np.log(1.5)) and np.all(fh[1][1:-1, 1:-1] == 0.0)
