"""Pins of the FP64 selector oracle: finite differences, a closed-form loss
and gradient, the closed form of Adam's first step, and min-max scaling."""
import math

import numpy as np

import oracle
from paper_1805_11938_amd import synth


def _params(seed=1):
    return synth.mlp_init(seed)


def test_init_shapes_and_bounds():
    p = _params()
    assert [a.shape for a in p] == [(12, 64), (64,), (64, 64), (64,), (64, 5), (5,)]
    assert np.abs(p[0]).max() <= math.sqrt(6 / 12) and np.abs(p[2]).max() <= math.sqrt(6 / 64)
    assert all(np.all(b == 0) for b in p[1::2])


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    p = _params(3)
    p = [a + 0.05 * rng.standard_normal(a.shape) for a in p]  # nonzero biases too
    X = rng.random((9, 12))
    y = rng.integers(0, 5, 9)
    _, g = oracle.mlp_loss_and_grads(p, X, y)
    h = 1e-6
    for li, a in enumerate(p):
        flat = a.ravel()
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            pp = [b.copy() for b in p]
            pm = [b.copy() for b in p]
            pp[li].ravel()[idx] += h
            pm[li].ravel()[idx] -= h
            num = (oracle.mlp_loss_and_grads(pp, X, y)[0] - oracle.mlp_loss_and_grads(pm, X, y)[0]) / (2 * h)
            ana = g[li].ravel()[idx]
            assert abs(num - ana) <= 1e-6 * max(1e-3, abs(ana)) + 1e-9, (li, idx, num, ana)


def test_zero_output_layer_closed_form():
    rng = np.random.default_rng(1)
    p = _params(5)
    p[4] = np.zeros_like(p[4])
    p[5] = np.zeros_like(p[5])
    B = 7
    X = rng.random((B, 12))
    y = rng.integers(0, 5, B)
    loss, g = oracle.mlp_loss_and_grads(p, X, y)
    assert abs(loss - math.log(5)) < 1e-15
    onehot = np.eye(5)[y]
    dz = (0.2 - onehot) / B
    assert np.allclose(g[5], dz.sum(0), atol=1e-16, rtol=0)
    z, (X_, a1, h1, a2, h2) = oracle.mlp_forward(p, X)
    assert np.allclose(g[4], h2.T @ dz, atol=1e-15, rtol=0)
    # no gradient reaches the hidden layers through a zero W3
    assert np.all(g[0] == 0) and np.all(g[2] == 0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    p = [rng.standard_normal((3, 4))]
    g = [rng.standard_normal((3, 4))]
    m = [np.zeros((3, 4))]
    v = [np.zeros((3, 4))]
    lr, eps = 1e-3, 1e-8
    (p1,), (m1,), (v1,) = oracle.adam_step(p, g, m, v, 1, lr=lr, eps=eps)
    # bias-corrected first step: m_hat = g, v_hat = g^2
    assert np.allclose(p1, p[0] - lr * g[0] / (np.abs(g[0]) + eps), rtol=1e-13, atol=0)
    assert np.allclose(m1, 0.1 * g[0], rtol=1e-15) and np.allclose(v1, 0.001 * g[0] ** 2, rtol=1e-13)


def test_minmax_and_transform():
    F = np.array([[1.0, 10, 100, 0.5, 1, 2, 3, 4, 0.1, 1, 7, 0.2],
                  [3.0, 30, 300, 0.25, 2, 4, 5, 6, 0.3, 2, 9, 0.4]])
    T = oracle.feature_transform(F)
    assert T[0, 0] == 1.0 and T[1, 0] == 2.0  # log2(1 + 1), log2(1 + 3)
    assert T[0, 3] == -1.0 and T[1, 3] == -2.0  # log2 of the fraction
    assert T[0, 8] == 0.1 and T[1, 11] == 0.4  # untouched
    lo, hi = oracle.minmax_fit(T)
    S = oracle.minmax_apply(T, lo, hi)
    assert np.all((S == 0) | (S == 1))
    # no clamping outside the training range
    out = oracle.minmax_apply(T[:1] * 0 + hi + (hi - lo), lo, hi)
    assert np.allclose(out[0][hi > lo], 2.0)


def test_forward_by_hand():
    # A two-sample network with hand-chosen weights, worked on paper; every value is exact in
    # binary, so the comparison is exact.  Hidden unit 0 of layer 1 is cut by the ReLU for the
    # second sample, unit 1 for the second sample as well; unit 0 of layer 2 for the first.
    W1 = np.zeros((12, 64)); b1 = np.zeros(64)
    W2 = np.zeros((64, 64)); b2 = np.zeros(64)
    W3 = np.zeros((64, 5)); b3 = np.zeros(5)
    W1[0, 0], W1[1, 0], b1[0] = 1.0, -2.0, 0.5      # a1_0 = x0 - 2 x1 + 0.5
    W1[2, 1], b1[1] = 3.0, -1.0                      # a1_1 = 3 x2 - 1
    W2[0, 0], W2[1, 0], b2[0] = 2.0, -5.0, 0.25      # a2_0 = 2 h1_0 - 5 h1_1 + 0.25
    W2[0, 1], b2[1] = 1.0, -0.75                     # a2_1 = h1_0 - 0.75
    b2[2] = 1.5                                      # a2_2 = 1.5
    W3[0, 0] = 4.0                                   # z0 = 4 h2_0
    W3[1, 1], b3[1] = 8.0, 0.5                       # z1 = 8 h2_1 + 0.5
    W3[2, 2] = 2.0                                   # z2 = 2 h2_2
    W3[2, 4], b3[4] = -1.0, -3.0                     # z4 = -h2_2 - 3
    X = np.full((2, 12), 7.0)                        # features with zero weights still present
    X[0, :3] = [1.0, 0.25, 0.5]
    X[1, :3] = [0.0, 1.0, 0.0]
    z, (_, a1, h1, a2, h2) = oracle.mlp_forward([W1, b1, W2, b2, W3, b3], X)
    # sample 0: a1 = [1, 0.5]; a2 = [2 - 2.5 + 0.25, 1 - 0.75, 1.5] = [-0.25 (cut), 0.25, 1.5]
    # sample 1: a1 = [-1.5, -1] (both cut); a2 = [0.25, -0.75 (cut), 1.5]
    assert a1[:, :2].tolist() == [[1.0, 0.5], [-1.5, -1.0]]
    assert h1[:, :2].tolist() == [[1.0, 0.5], [0.0, 0.0]]
    assert a2[:, :3].tolist() == [[-0.25, 0.25, 1.5], [0.25, -0.75, 1.5]]
    assert h2[:, :3].tolist() == [[0.0, 0.25, 1.5], [0.25, 0.0, 1.5]]
    assert np.all(a1[:, 2:] == 0) and np.all(a2[:, 3:] == 0)
    assert z.tolist() == [[0.0, 2.5, 3.0, 0.0, -4.5], [1.0, 0.5, 3.0, 0.0, -4.5]]
