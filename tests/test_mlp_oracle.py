"""Pins of the FP64 network reference: gradients against central finite
differences of the loss, softmax cross-entropy against its closed form on a
constructed case, and the order choice against a hand-computed CDF."""
import numpy as np

from oracle import mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.standard_normal(mlp.NPARAMS) * 0.1
    x = rng.standard_normal((5, mlp.IN))
    y = rng.integers(0, mlp.NCLS, size=(5, 3))
    loss, g = mlp.loss_and_grad(p, x, y)
    B = x.shape[0]
    idx = rng.choice(mlp.NPARAMS, size=60, replace=False)
    # include the biases of every layer
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SHAPES])
    idx = np.concatenate([idx, offs[1:-1] - 1, offs[1:-1]])
    h = 1e-6
    for i in idx:
        dp = np.zeros_like(p)
        dp[i] = h
        lp, _ = mlp.loss_and_grad(p + dp, x, y)
        lm, _ = mlp.loss_and_grad(p - dp, x, y)
        fd = (lp - lm) / (2 * h) / B
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_cross_entropy_closed_form():
    # zero weights: logits = b3; with b3 = 0 every class has probability 1/19
    p = np.zeros(mlp.NPARAMS)
    x = np.ones((3, mlp.IN))
    y = np.array([[0, 5, 18], [1, 1, 1], [7, 3, 2]])
    loss, g = mlp.loss_and_grad(p, x, y)
    assert abs(loss - 3 * 3 * np.log(19)) < 1e-12
    # gradient of b3: mean over samples of (1/19 - onehot)
    gb3 = g[-mlp.OUT:]
    ref = np.full(mlp.OUT, 1.0 / 19)
    for ax in range(3):
        for b in range(3):
            ref[ax * 19 + y[b, ax]] -= 1.0 / 3
    assert np.abs(gb3 - ref).max() < 1e-14


def test_choose_rule():
    z = np.full((1, mlp.OUT), -50.0)
    z[0, 2] = 0.0             # axis 0: all mass on class 2 -> K = 8
    z[0, 19 + 0] = 0.0        # axis 1: two equal classes 0 and 10
    z[0, 19 + 10] = 0.0
    z[0, 38 + 18] = 0.0       # axis 2: class 18 -> K = 24
    q = mlp.choose(z, 0.99)
    assert q.tolist() == [[8, 16, 24]]
    q = mlp.choose(z, 0.4)
    assert q.tolist() == [[8, 6, 24]]


def test_adam_first_step_is_signed_lr():
    p = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    p1, m, v = mlp.adam(p, g, np.zeros(4), np.zeros(4), 1, 0.1)
    assert np.allclose(p1[:3], -0.1 * np.sign(g[:3]), atol=1e-7)
    assert p1[3] == 0.0


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the first and second moments are
    m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the bias-corrected
    estimates are exactly g and g^2 at every step t, and each step moves a
    parameter by lr * g / (|g| + eps): after T steps the displacement is
    T lr g / (|g| + eps).  A wrong bias-correction power, beta or step index
    breaks this from the second step on."""
    rng = np.random.default_rng(11)
    g = rng.standard_normal(16) * np.logspace(-3, 2, 16)
    p0 = rng.standard_normal(16)
    lr, eps = 3e-3, 1e-8
    p, m, v = p0.copy(), np.zeros(16), np.zeros(16)
    for t in range(1, 8):
        p, m, v = mlp.adam(p, g, m, v, t, lr, eps=eps)
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-13, atol=0)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12, atol=0)
        step_ref = p0 - t * lr * g / (np.abs(g) + eps)
        assert np.abs(p - step_ref).max() <= 1e-13 * t
