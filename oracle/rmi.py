"""Float64 reference for the index network and its training step.  TEST INFRASTRUCTURE.

Not in the paper.  The learned index is a two-stage recursive model index
(Kraska et al., "The Case for Learned Index Structures", 2018): stage 1 picks
one of E experts, the chosen stage-2 expert predicts a position.  Every
network here is a one-input, one-output perceptron with H ReLU hidden units:

    f(u) = sum_i w2[i] * relu(w1[i] * u + b1[i]) + b2

with the parameter vector laid out as [w1 (H), b1 (H), w2 (H), b2].  The loss
of one network over its N samples is the mean squared error

    L = (1 / N) * sum_n (f(u_n) - t_n)^2

and a stage of E experts minimises the sum of the experts' own losses, each
averaged over that expert's samples.  The ReLU derivative at 0 is taken as 0.
The optimiser is Adam (Kingma and Ba, 2015) with bias correction.
"""

from __future__ import annotations

import numpy as np


def n_params(hidden: int) -> int:
    return 3 * hidden + 1


def split(theta: np.ndarray, hidden: int):
    t = np.asarray(theta, dtype=np.float64)
    return t[:hidden], t[hidden:2 * hidden], t[2 * hidden:3 * hidden], t[3 * hidden]


def forward(theta, u, hidden: int):
    """f(u) for a vector of inputs u (float64)."""
    w1, b1, w2, b2 = split(theta, hidden)
    u = np.asarray(u, dtype=np.float64)
    z = np.outer(u, w1) + b1
    h = np.maximum(z, 0.0)
    return h @ w2 + b2


def loss(theta, u, t, hidden: int) -> float:
    y = forward(theta, u, hidden)
    t = np.asarray(t, dtype=np.float64)
    return float(np.mean((y - t) ** 2)) if t.size else 0.0


def grad(theta, u, t, hidden: int) -> np.ndarray:
    """dL/dtheta of one network's MSE, by the chain rule written out term by term."""
    w1, b1, w2, b2 = split(theta, hidden)
    u = np.asarray(u, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = u.shape[0]
    g = np.zeros(n_params(hidden))
    if n == 0:
        return g
    z = np.outer(u, w1) + b1                 # (n, H)
    h = np.maximum(z, 0.0)
    y = h @ w2 + b2
    d = 2.0 * (y - t) / n                    # dL/dy_n
    g[2 * hidden:3 * hidden] = h.T @ d       # dL/dw2
    g[3 * hidden] = d.sum()                  # dL/db2
    dz = np.outer(d, w2) * (z > 0.0)         # dL/dz
    g[:hidden] = dz.T @ u                    # dL/dw1
    g[hidden:2 * hidden] = dz.sum(axis=0)    # dL/db1
    return g


def stage_grad(thetas, u, t, expert, hidden: int) -> np.ndarray:
    """Gradients of a stage of E experts; sample n trains expert ``expert[n]``."""
    thetas = np.asarray(thetas, dtype=np.float64)
    out = np.zeros_like(thetas)
    expert = np.asarray(expert)
    for e in range(thetas.shape[0]):
        sel = expert == e
        out[e] = grad(thetas[e], np.asarray(u)[sel], np.asarray(t)[sel], hidden)
    return out


def adam(theta, g, m, v, step: int, lr: float, beta1: float = 0.9,
         beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update; returns (theta, m, v) as new float64 arrays. ``step`` counts from 1."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * np.asarray(g, np.float64)
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * np.asarray(g, np.float64) ** 2
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return np.asarray(theta, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v
