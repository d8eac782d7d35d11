"""Pins of the FP64 warm-start network reference (oracle/mlp.py) on the CPU."""

import numpy as np

from oracle import mlp as M


def _params(shp, seed, scale=0.7):
    rng = np.random.default_rng(seed)
    Ws = [rng.normal(0, scale / np.sqrt(i), (o, i)) for o, i in shp]
    bs = [rng.normal(0, 0.3, o) for o, _ in shp]
    return M.pack(Ws, bs)


def test_gradient_matches_central_differences():
    shp = M.shapes(3, 5, 2)
    p = _params(shp, 0)
    rng = np.random.default_rng(1)
    x = rng.normal(size=(7, 3))
    t = rng.normal(size=(7, 2))
    L, g = M.loss_grad(p, shp, x, t)
    assert abs(L - M.loss(p, shp, x, t)) < 1e-15
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (M.loss(p + e, shp, x, t) - M.loss(p - e, shp, x, t)) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * max(1.0, np.abs(g).max())


def test_zero_hidden_weights_closed_form():
    """With W1 = W2 = W3 = 0 every hidden layer is tanh(b_l), so y = W4 tanh(b3) + b4 for every row."""
    shp = M.shapes(4, 6, 3)
    Ws, bs = M.unpack(_params(shp, 2), shp)
    for l in range(3):
        Ws[l][:] = 0.0
    p = M.pack(Ws, bs)
    x = np.random.default_rng(3).normal(size=(5, 4))
    y = M.forward(p, shp, x)[-1]
    expect = Ws[3] @ np.tanh(bs[2]) + bs[3]
    assert np.abs(y - expect[None, :]).max() < 1e-15


def test_first_adam_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2, so the update is -lr g / (|g| + eps)."""
    g = np.array([3.0, -2e-3, 0.0, 1e-9, -7.5])
    p = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    p1, m, v = M.adam_step(p, np.zeros(5), np.zeros(5), 1, g, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_round_bf16_ties_to_even():
    one = 1.0
    vals = np.array([one, one + 2.0 ** -8, one + 3 * 2.0 ** -8, -(one + 2.0 ** -7), 3.0e38, 0.0], dtype=np.float32)
    got = M.round_bf16(vals)
    expect = [one, one, one + 2.0 ** -6, -(one + 2.0 ** -7), None, 0.0]
    for gv, ev in zip(got, expect):
        if ev is not None:
            assert gv == ev
    # 3e38 rounds to a representable bfloat16 close to it
    assert abs(got[4] - 3.0e38) / 3.0e38 < 2 ** -8
