"""FP64 reference of the learned warm start's network (oracle; test
infrastructure only).

A 3-level 3D U-Net on a periodic grid: 3x3x3 convolutions with periodic
padding, ReLU, 2x2x2 average pooling, nearest-neighbour upsampling, skip
connections by channel concatenation, and a 1x1x1 output head.  Fields are
channels-last arrays of shape (n, n, n, C).  A convolution weight has shape
(27, Cin, Cout) with tap t = (di+1)*9 + (dj+1)*3 + (dk+1), and computes
  y[v, o] = b[o] + sum_t sum_c x[v + d_t, c] W[t, c, o].
Backward passes are written out by hand and pinned by finite differences in
tests/test_oracle_unet.py.
"""
from __future__ import annotations

import numpy as np

TAPS = [(di, dj, dk) for di in (-1, 0, 1) for dj in (-1, 0, 1) for dk in (-1, 0, 1)]

# (name, Cin, Cout) of the 3x3x3 convolutions in execution order
LAYERS = [
    ("l1a", 4, 16), ("l1b", 16, 16),
    ("l2a", 16, 32), ("l2b", 32, 32),
    ("l3a", 32, 64), ("l3b", 64, 64),
    ("l4a", 96, 32), ("l4b", 32, 32),
    ("l5a", 48, 16), ("l5b", 16, 16),
]


def shift(x, d):
    """x[v + d] on the periodic grid (x has spatial axes 0..2)."""
    return np.roll(x, (-d[0], -d[1], -d[2]), axis=(0, 1, 2))


def conv3(x, W, b):
    y = np.zeros(x.shape[:3] + (W.shape[2],))
    for t, d in enumerate(TAPS):
        y += shift(x, d) @ W[t]
    return y + b


def conv3_backward(x, W, dy):
    """Gradients of conv3 w.r.t. its input, weight and bias."""
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t, d in enumerate(TAPS):
        dW[t] = shift(x, d).reshape(-1, x.shape[3]).T @ dy.reshape(-1, dy.shape[3])
        dx += shift(dy @ W[t].T, (-d[0], -d[1], -d[2]))
    return dx, dW, dy.sum(axis=(0, 1, 2))


def pool(x):
    n = x.shape[0] // 2
    return x.reshape(n, 2, n, 2, n, 2, -1).mean(axis=(1, 3, 5))


def pool_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_backward(dy):
    n = dy.shape[0] // 2
    return dy.reshape(n, 2, n, 2, n, 2, -1).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


def init_params(seed=0):
    """He-normal weights, zero biases, head weight ~ N(0, 1/16)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co in LAYERS:
        p[name + ".w"] = rng.standard_normal((27, ci, co)) * np.sqrt(2.0 / (27 * ci))
        p[name + ".b"] = np.zeros(co)
    p["head.w"] = rng.standard_normal(16) * 0.25
    p["head.b"] = np.zeros(1)
    return p


class _NoCache(dict):
    def __setitem__(self, key, value):
        pass


def forward(p, x0, keep=True):
    """Returns (yhat (n,n,n), cache) for the input x0 (n,n,n,4).  With
    keep=False the activations are not kept (cache is empty), which bounds
    the memory of large grids."""
    c = {"x0": x0} if keep else _NoCache()
    a = relu(conv3(x0, p["l1a.w"], p["l1a.b"]))
    c["a1"] = a
    s1 = relu(conv3(a, p["l1b.w"], p["l1b.b"]))
    c["s1"] = s1
    a = pool(s1)
    c["p1"] = a
    a = relu(conv3(a, p["l2a.w"], p["l2a.b"]))
    c["a2"] = a
    s2 = relu(conv3(a, p["l2b.w"], p["l2b.b"]))
    c["s2"] = s2
    a = pool(s2)
    c["p2"] = a
    a = relu(conv3(a, p["l3a.w"], p["l3a.b"]))
    c["a3"] = a
    a = relu(conv3(a, p["l3b.w"], p["l3b.b"]))
    c["b3"] = a
    cat2 = np.concatenate([up(a), s2], axis=3)
    c["c2"] = cat2
    a = relu(conv3(cat2, p["l4a.w"], p["l4a.b"]))
    c["a4"] = a
    a = relu(conv3(a, p["l4b.w"], p["l4b.b"]))
    c["b4"] = a
    cat1 = np.concatenate([up(a), s1], axis=3)
    c["c1"] = cat1
    a = relu(conv3(cat1, p["l5a.w"], p["l5a.b"]))
    c["a5"] = a
    a = relu(conv3(a, p["l5b.w"], p["l5b.b"]))
    c["b5"] = a
    y = a @ p["head.w"] + p["head.b"][0]
    return y, c


def backward(p, c, dy, rnd=None):
    """Gradients of all parameters for the output gradient dy (n,n,n).

    ``rnd`` (default: none) is applied to every activation gradient a layer
    hands to the layer below -- the head's, each convolution's input
    gradient, each upsampling adjoint and each pooling adjoint plus its skip
    gradient -- so that a caller can reproduce a narrower storage format of
    those tensors; the parameter gradients are never rounded."""
    if rnd is None:
        rnd = _identity
    g = {}
    g["head.w"] = np.tensordot(c["b5"], dy, axes=([0, 1, 2], [0, 1, 2]))
    g["head.b"] = np.array([dy.sum()])
    d = rnd(dy[..., None] * p["head.w"][None, None, None, :])

    def back(name, x, out, d):
        d = d * (out > 0)
        dx, g[name + ".w"], g[name + ".b"] = conv3_backward(x, p[name + ".w"], d)
        return rnd(dx)

    d = back("l5b", c["a5"], c["b5"], d)
    d = back("l5a", c["c1"], c["a5"], d)
    d_up1, d_s1 = d[..., :32], d[..., 32:]
    d = rnd(up_backward(d_up1))
    d = back("l4b", c["a4"], c["b4"], d)
    d = back("l4a", c["c2"], c["a4"], d)
    d_up2, d_s2 = d[..., :64], d[..., 64:]
    d = rnd(up_backward(d_up2))
    d = back("l3b", c["a3"], c["b3"], d)
    d = back("l3a", c["p2"], c["a3"], d)
    d = rnd(pool_backward(d) + d_s2)
    d = back("l2b", c["a2"], c["s2"], d)
    d = back("l2a", c["p1"], c["a2"], d)
    d = rnd(pool_backward(d) + d_s1)
    d = back("l1b", c["a1"], c["s1"], d)
    back("l1a", c["x0"], c["a1"], d)
    return g


def _identity(x):
    return x


def adam_step(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_clip=0.0):
    """One step of Adam (Kingma and Ba, "Adam: a method for stochastic
    optimization", 2015, Algorithm 1), preceded by global-norm clipping of
    the gradient when grad_clip > 0: g <- g min(1, grad_clip / ||g||_2).
    ``step`` is t >= 1, the number of the update.  Returns (w, m, v, ||g||_2
    before clipping) as new arrays."""
    g = np.asarray(g, dtype=np.float64)
    gnorm = float(np.sqrt(np.sum(g * g)))
    if grad_clip > 0.0 and gnorm > grad_clip:
        g = g * (grad_clip / gnorm)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1**step)
    v_hat = v / (1.0 - beta2**step)
    w = np.asarray(w, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return w, m, v, gnorm


def input_features(rho, alpha_b0, alpha_m0, a):
    """Input channels: standardised l = ln(1 + delta + 1e-3), delta = rho -
    <rho>, and the three broadcast parameters alpha_B0, alpha_M0, a."""
    rho = np.asarray(rho, dtype=np.float64)
    delta = rho - rho.mean()
    lr = np.log(np.maximum(1.0 + delta, 0.0) + 1e-3)
    lr = (lr - lr.mean()) / lr.std()
    n = lr.shape[0]
    x = np.empty((n, n, n, 4))
    x[..., 0] = lr
    x[..., 1] = alpha_b0
    x[..., 2] = alpha_m0
    x[..., 3] = a
    return x


def source_target(chi, rho, s_mu_chi):
    """The nonlinear part of the scalar field's normalised source,
    t = lap_h chi / (s mu_chi) - delta (7-point periodic Laplacian, h = 1/n):
    zero where chi obeys the linearised equation lap chi = mu_chi s delta."""
    chi = np.asarray(chi, dtype=np.float64)
    n = chi.shape[0]
    lap = -6.0 * chi
    for ax in range(3):
        lap += np.roll(chi, 1, ax) + np.roll(chi, -1, ax)
    rho = np.asarray(rho, dtype=np.float64)
    return lap * n * n / s_mu_chi - (rho - rho.mean())
