"""Learned proposal for the subsample sketch: coordinate features, a 3-layer MLP,
its listwise loss, backward pass and Adam, all in FP64.

The paper lets the sketch distribution D be any distribution whose expected
projection is positive definite (Sec. 3, Sec. 5) and studies non-uniform
coordinate probabilities, e.g. p_i proportional to A_ii (Sec. 7). It does not
prescribe a learned distribution; everything here is this repository's
proposal, pinned by finite differences and closed forms rather than by the paper.

Features of coordinate j at iteration k (r = r^k = A x^k - b, rp = r^{k-1},
a_j = A_jj, last_j = the latest iteration < k whose sketch held j, or -1):

  f0 = (log a_j - mean_j log a) / std_j log a        (0 if the std is 0)
  f1 = clip(log|r_j| - log(a_j)/2 - log||r|| + log(sum_j a_j)/2, -30, 30)
  f2 = log(1 + k - last_j)
  f3 = clip(log|r_j - rp_j| - log||r|| + log(m)/2, -30, 30)
  f4 = log(k + 1)
  f5 = 1 if last_j == k - 1 else 0

(log 0 = -inf before clipping). f1 compares coordinate j's residual, scaled by
sqrt(a_j), with the average such scaled residual.

Network: s = w3 . relu(W2^T relu(W1^T f + b1) + b2) + b3 with f in R^6, hidden
width 128 (W1: 6 x 128, W2: 128 x 128, row-major [in][out]). Parameters are
packed in the order W1, b1, W2, b2, w3, b3 (17665 values). Initial weights are
uniform on [-1/sqrt(fan_in), 1/sqrt(fan_in)] from Philox4x64-10 with key
(seed, 0) and counter (index, 0, 5, 0): u = ((W0 >> 12) + 0.5) 2^-52,
value = (1/sqrt(fan_in)) (2u - 1); biases start at 0.

Proposal: q = (1 - eps) softmax(s) + eps / m (eps = 0.1), so that every
coordinate keeps probability mass and the expected projection stays positive
definite (the condition of Thm 5.1).

Loss on one recorded iteration with sketch C (tau coordinates) and credits
c_b = delta_b rho_b (their sum is delta^T G delta, the decrease of the squared
A-norm error of that step, eq:gradeqf): t = max(c, 0) / sum max(c, 0),
p = softmax(s[C]) over the sketch only, L = -sum_b t_b log p_b, and
dL/ds[C_b] = p_b - t_b. Iterations whose credits are all <= 0 carry no loss.

Adam: m1 <- b1 m1 + (1 - b1) g, m2 <- b2 m2 + (1 - b2) g^2,
theta <- theta - lr (m1 / (1 - b1^t)) / (sqrt(m2 / (1 - b2^t)) + eps_adam).

Part of the oracle: test infrastructure only.
"""
import numpy as np

from .philox import philox4x64_10

NF = 6
H = 128
SIZES = [("W1", (NF, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)
TAG_INIT = 5
CLIP = 30.0
EPS_MIX = 0.1


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights from the counter RNG, zero biases."""
    idx = np.arange(NPARAMS, dtype=np.uint64)
    w0, _, _, _ = philox4x64_10(idx, np.uint64(0), np.uint64(TAG_INIT), np.uint64(0),
                                np.uint64(seed), np.uint64(0))
    u = ((w0 >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52
    theta = np.zeros(NPARAMS)
    o = 0
    fan = {"W1": NF, "W2": H, "w3": H}
    for name, shape in SIZES:
        n = int(np.prod(shape))
        if name in fan:
            scale = 1.0 / np.sqrt(float(fan[name]))
            theta[o:o + n] = scale * (2.0 * u[o:o + n] - 1.0)
        o += n
    return theta


def features(a, r, rp, last, k):
    """F (m x 6) of every coordinate, as defined in the module docstring."""
    a = np.asarray(a, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    rp = np.asarray(rp, dtype=np.float64)
    last = np.asarray(last, dtype=np.int64)
    m = a.shape[0]
    la = np.log(a)
    mu = la.mean()
    sd = np.sqrt(((la - mu) ** 2).mean())
    F = np.zeros((m, NF))
    F[:, 0] = (la - mu) / sd if sd > 0 else 0.0
    rn = np.linalg.norm(r)
    with np.errstate(divide="ignore"):
        F[:, 1] = np.clip(np.log(np.abs(r)) - 0.5 * la - np.log(rn) + 0.5 * np.log(a.sum()), -CLIP, CLIP)
        F[:, 3] = np.clip(np.log(np.abs(r - rp)) - np.log(rn) + 0.5 * np.log(float(m)), -CLIP, CLIP)
    F[:, 2] = np.log(1.0 + (k - last).astype(np.float64))
    F[:, 4] = np.log(float(k + 1))
    F[:, 5] = (last == k - 1).astype(np.float64)
    return F


def forward(theta, F):
    """Scores s (rows of F) and the activations the backward pass needs."""
    P = unpack(theta)
    z1 = F @ P["W1"] + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(z2, 0.0)
    s = h2 @ P["w3"] + P["b3"][0]
    return s, (F, z1, h1, z2, h2)


def backward(theta, cache, ds):
    """Gradient of sum_i ds_i s_i with respect to the packed parameters."""
    P = unpack(theta)
    F, z1, h1, z2, h2 = cache
    g = {}
    g["w3"] = h2.T @ ds
    g["b3"] = np.array([ds.sum()])
    dh2 = np.outer(ds, P["w3"]) * (z2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ P["W2"].T) * (z1 > 0)
    g["W1"] = F.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return pack(g)


def listwise_loss(s_sel, credits):
    """(L, dL/ds) over one sketch's coordinates; (0, 0) when no credit is positive."""
    c = np.maximum(np.asarray(credits, dtype=np.float64), 0.0)
    tot = c.sum()
    if not tot > 0.0:
        return 0.0, np.zeros_like(s_sel)
    t = c / tot
    z = s_sel - s_sel.max()
    lse = np.log(np.exp(z).sum())
    logp = z - lse
    return float(-(t * logp).sum()), np.exp(logp) - t


def batch_loss_grad(theta, Fs, credits):
    """Mean loss and gradient over samples: Fs (nsamples x tau x 6), credits (nsamples x tau)."""
    ns, tau, _ = Fs.shape
    s, cache = forward(theta, Fs.reshape(ns * tau, NF))
    s = s.reshape(ns, tau)
    ds = np.zeros_like(s)
    L = 0.0
    for i in range(ns):
        li, gi = listwise_loss(s[i], credits[i])
        L += li
        ds[i] = gi
    return L / ns, backward(theta, cache, ds.ravel() / ns)


def adam_step(theta, grad, m1, m2, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t >= 1 counts the steps); returns new (theta, m1, m2)."""
    m1 = b1 * m1 + (1.0 - b1) * grad
    m2 = b2 * m2 + (1.0 - b2) * grad * grad
    mh = m1 / (1.0 - b1 ** t)
    vh = m2 / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m1, m2


def proposal(s, eps=EPS_MIX):
    """q = (1 - eps) softmax(s) + eps / m."""
    s = np.asarray(s, dtype=np.float64)
    z = np.exp(s - s.max())
    return (1.0 - eps) * z / z.sum() + eps / s.shape[0]
