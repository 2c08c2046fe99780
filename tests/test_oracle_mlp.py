"""CPU pins of the oracle's learned-proposal pieces (features, MLP, loss, Adam, proposal).

The paper does not define a learned proposal, so these are pinned by mathematics:
central finite differences for the backward pass, closed forms of the loss and of
Adam's first step, hand-computed features, and the probability-simplex properties
of the proposal.
"""
import numpy as np
import pytest

from oracle import mlp


def _theta(seed=3):
    th = mlp.init_params(seed)
    rng = np.random.default_rng(seed)
    return th + 0.05 * rng.standard_normal(th.shape)  # nonzero biases too


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    th = _theta()
    Fs = rng.standard_normal((2, 7, mlp.NF))
    cr = np.abs(rng.standard_normal((2, 7))) * (rng.random((2, 7)) < 0.7)
    cr[:, 0] = 1.0
    L, g = mlp.batch_loss_grad(th, Fs, cr)
    sizes = {n: int(np.prod(s)) for n, s in mlp.SIZES}
    offs = np.cumsum([0] + [sizes[n] for n, _ in mlp.SIZES])
    idx = []
    for b in range(len(mlp.SIZES)):  # a sample of every parameter block
        lo, hi = offs[b], offs[b + 1]
        idx += list(rng.choice(np.arange(lo, hi), size=min(40, hi - lo), replace=False))
    h = 1e-6
    worst = 0.0
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.batch_loss_grad(tp, Fs, cr)[0] - mlp.batch_loss_grad(tm, Fs, cr)[0]) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / max(1e-3, np.abs(g).max()))
    assert worst <= 1e-6, worst


def test_loss_closed_forms():
    s = np.array([0.3, -1.0, 2.0, 0.5])
    # one-hot credit: L = -log p_i
    L, ds = mlp.listwise_loss(s, np.array([0.0, 0.0, 5.0, -1.0]))
    p = np.exp(s) / np.exp(s).sum()
    assert np.isclose(L, -np.log(p[2]), rtol=1e-14)
    assert np.allclose(ds, p - np.array([0, 0, 1.0, 0]), atol=1e-15)
    # equal scores: L = log(tau) for any normalised target
    L, ds = mlp.listwise_loss(np.zeros(4), np.array([1.0, 2.0, 3.0, 4.0]))
    assert np.isclose(L, np.log(4.0), rtol=1e-14)
    assert abs(ds.sum()) < 1e-15
    # shifting every score leaves the loss unchanged; no positive credit -> no loss
    L1, _ = mlp.listwise_loss(s, np.array([1.0, 2.0, 0.0, 0.5]))
    L2, _ = mlp.listwise_loss(s + 7.25, np.array([1.0, 2.0, 0.0, 0.5]))
    assert np.isclose(L1, L2, rtol=1e-13)
    L, ds = mlp.listwise_loss(s, np.array([-1.0, 0.0, -2.0, 0.0]))
    assert L == 0.0 and not ds.any()


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.ones(4)
    new, m1, m2 = mlp.adam_step(th, g, np.zeros(4), np.zeros(4), t=1, lr=0.01, eps=1e-8)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def test_adam_constant_gradient_closed_form_every_step():
    """Under a constant gradient g the moments have closed forms m1_t = (1 - b1^t) g and
    m2_t = (1 - b2^t) g^2, so the bias-corrected moments equal g and g^2 at every t and every
    update is -lr g / (|g| + eps). Checked at t = 1, 2, 50 and 1000: an exponent slip in the
    bias correction (b1 instead of b1^t, t - 1 for t) or b1 and b2 swapped fails it at t >= 2."""
    g = np.array([0.5, -2.0, 1e-3, 3.0e-6, -7.25])
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    th = np.linspace(-1.0, 1.0, g.size)
    m1 = np.zeros_like(g)
    m2 = np.zeros_like(g)
    for t in range(1, 1001):
        new, m1, m2 = mlp.adam_step(th, g, m1, m2, t=t, lr=lr, b1=b1, b2=b2, eps=eps)
        if t in (1, 2, 50, 1000):
            np.testing.assert_allclose(m1, (1.0 - b1 ** t) * g, rtol=1e-12, atol=0)
            np.testing.assert_allclose(m2, (1.0 - b2 ** t) * g * g, rtol=1e-12, atol=0)
            np.testing.assert_allclose(new - th, -lr * g / (np.abs(g) + eps), rtol=1e-10, atol=0)
        th = new


def test_proposal_is_a_mixed_distribution():
    rng = np.random.default_rng(1)
    s = 5 * rng.standard_normal(1000)
    q = mlp.proposal(s)
    assert np.isclose(q.sum(), 1.0, rtol=1e-13)
    assert q.min() >= 0.1 / 1000 * (1 - 1e-12)
    assert np.allclose(mlp.proposal(np.full(7, 3.0)), np.full(7, 1 / 7), rtol=1e-14)


def test_init_range_and_reproducibility():
    a = mlp.init_params(11)
    b = mlp.init_params(11)
    c = mlp.init_params(12)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    P = mlp.unpack(a)
    assert np.abs(P["W1"]).max() <= 1 / np.sqrt(6) and np.abs(P["W2"]).max() <= 1 / np.sqrt(128)
    assert np.abs(P["w3"]).max() <= 1 / np.sqrt(128)
    assert not P["b1"].any() and not P["b2"].any() and P["b3"][0] == 0.0
    # uniform on [-s, s]: mean ~ 0, variance ~ s^2 / 3
    w = P["W2"].ravel() * np.sqrt(128)
    assert abs(w.mean()) < 0.02 and abs(w.var() - 1 / 3) < 0.02


def test_features_hand_computed():
    a = np.exp(np.array([0.0, 2.0, 4.0]))
    r = np.array([3.0, 0.0, -4.0])
    rp = np.array([3.0, 1.0, -2.0])
    last = np.array([-1, 5, 6])
    k = 7
    F = mlp.features(a, r, rp, last, k)
    sd = np.sqrt(8.0 / 3.0)
    assert np.allclose(F[:, 0], np.array([-2.0, 0.0, 2.0]) / sd, rtol=1e-14)
    base = -np.log(5.0) + 0.5 * np.log(a.sum())
    assert np.isclose(F[0, 1], np.log(3.0) + base, rtol=1e-14)
    assert F[1, 1] == -30.0  # r_j = 0
    assert np.isclose(F[2, 1], np.log(4.0) - 2.0 + base, rtol=1e-14)
    assert np.allclose(F[:, 2], np.log([1.0 + 8, 1.0 + 2, 1.0 + 1]), rtol=1e-15)
    assert F[0, 3] == -30.0  # r_j unchanged
    assert np.isclose(F[1, 3], np.log(1.0) - np.log(5.0) + 0.5 * np.log(3.0), rtol=1e-14)
    assert np.allclose(F[:, 4], np.log(8.0)) and np.array_equal(F[:, 5], [0.0, 0.0, 1.0])


def test_training_lowers_the_loss_on_a_learnable_signal():
    """Credits that grow with f1 are learnable: 200 Adam steps cut the loss."""
    rng = np.random.default_rng(5)
    th = mlp.init_params(2)
    ns, tau = 8, 16
    Fs = rng.standard_normal((ns, tau, mlp.NF))
    cr = np.exp(2.0 * Fs[:, :, 1])
    L0, _ = mlp.batch_loss_grad(th, Fs, cr)
    m1 = np.zeros_like(th)
    m2 = np.zeros_like(th)
    for t in range(1, 201):
        L, g = mlp.batch_loss_grad(th, Fs, cr)
        th, m1, m2 = mlp.adam_step(th, g, m1, m2, t, lr=3e-3)
    assert L < 0.8 * L0, (L0, L)
