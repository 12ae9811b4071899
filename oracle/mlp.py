"""FP64 forward/backward of the first-floor selector network.

Architecture (learned first-floor selection): x(8) -> Linear(64) -> GELU ->
Linear(64) -> GELU -> Linear(4) -> softmax over ladder rungs; loss = mean
cross-entropy against the lowest admissible rung.  GELU is the exact erf form
0.5 x (1 + erf(x / sqrt 2)).  Prediction = argmax, ties -> lower rung
(preservation first).  Weights are stored row-major as W[out][in].

Adam (lr, beta1=0.9, beta2=0.999, eps=1e-8) is the textbook update, pinned by
its closed forms: the first step and every step under a constant gradient move
each parameter by lr * g / (|g| + eps), and the moments equal the geometric
averages of the gradients seen.
"""
import math

import numpy as np
from scipy.special import erf

SIZES = (8, 64, 64, 4)


def init_params(seed, sizes=SIZES):
    """He-normal weights from numpy default_rng(seed), zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        W = rng.standard_normal((fo, fi)) * math.sqrt(2.0 / fi)
        params += [W, np.zeros(fo)]
    return params


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx GELU = Phi(x) + x phi(x)."""
    Phi = 0.5 * (1.0 + erf(x / math.sqrt(2.0)))
    phi = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return Phi + x * phi


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    a1 = X @ W1.T + b1
    h1 = gelu(a1)
    a2 = h1 @ W2.T + b2
    h2 = gelu(a2)
    logits = h2 @ W3.T + b3
    return logits, (X, a1, h1, a2, h2)


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_grads(params, X, y):
    """Mean softmax cross-entropy and its gradients w.r.t. every parameter."""
    W1, b1, W2, b2, W3, b3 = params
    logits, (X, a1, h1, a2, h2) = forward(params, X)
    B = X.shape[0]
    P = softmax(logits)
    loss = float(-np.mean(np.log(P[np.arange(B), y])))
    dlog = P.copy()
    dlog[np.arange(B), y] -= 1.0
    dlog /= B
    gW3 = dlog.T @ h2
    gb3 = dlog.sum(axis=0)
    dh2 = dlog @ W3
    da2 = dh2 * gelu_grad(a2)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * gelu_grad(a1)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def predict(params, X):
    logits, _ = forward(params, X)
    return np.argmax(logits, axis=1)     # first maximum = lower rung on ties


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam; state = dict(t, m, v)."""
    if not state:
        state.update(t=0, m=[np.zeros_like(p) for p in params],
                     v=[np.zeros_like(p) for p in params])
    state["t"] += 1
    t = state["t"]
    for p, g, m, v in zip(params, grads, state["m"], state["v"]):
        m *= b1
        m += (1 - b1) * g
        v *= b2
        v += (1 - b2) * g * g
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p -= lr * mh / (np.sqrt(vh) + eps)
