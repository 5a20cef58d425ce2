"""Learned warm start of the PDIP: per-contact features, a 3x128 MLP, its
gradients and Adam, plain FP64 NumPy.

The paper starts every PDIP from tangential impulses 0 and a preset normal
impulse, because warm-starting an interior-point method is hard: a point near
the optimum but off the central path makes the method take short steps
(Sec. 3.3, "Re-using information across timesteps").  The learned warm start
predicts the impulses of each contact from local features and starts the PDIP
from that prediction, placed strictly inside the cone and on the central path
of a chosen t0; the cold start stays as the fallback and the reference.

Readings (the design is not in the paper)
-----------------------------------------
* Features per contact, scaled units (velocities over g h, lengths over the
  mean radius r_bar):
    0      Phi / (h g h)                 (the b_i term of r, Sec. 2.3)
    1..3   D_i^T v / (g h)               relative velocity in (n, t1, t2)
    4..6   n
    7, 8   r_a / r_bar, r_b / r_bar      (r_b = 0 for a wall)
    9, 10  contacts of body a, of body b (0 for a wall)
* Network: 11 -> 128 -> 128 -> 128 -> 3, tanh hidden layers, linear output
  p = (p0, p1, p2).  Prediction gamma_n = exp(p0), gamma_t =
  0.9 mu gamma_n (p1, p2) / max(1, |(p1, p2)|).
* Targets from a solved step: y0 = log(max(gamma_n, 1e-6)),
  (y1, y2) = gamma_t / (mu gamma_n) clipped to the unit disc.
* Loss: mean over the batch of sum_k (p_k - y_k)^2 / 3.
* Adam (Kingma & Ba 2015): lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8.
* Features are z-scored with the training set's mean and deviation.
"""

from __future__ import annotations

import numpy as np

from . import assembly

LAYERS = (11, 128, 128, 128, 3)


def features(scene, contacts):
    """[Nc][11] features of the ordered contacts (see module readings)."""
    D = assembly.jacobian(scene, contacts)
    vel = D.T @ assembly.generalized_velocity(scene)
    vbar = float(np.linalg.norm(scene.gravity)) * scene.h
    rbar = float(scene.radius.mean())
    nc = contacts.nc
    F = np.zeros((nc, 11))
    F[:, 0] = contacts.phi / scene.h / vbar
    F[:, 1:4] = vel.reshape(-1, 3) / vbar
    F[:, 4:7] = contacts.frame[:, 0, :]
    wall = contacts.is_wall
    F[:, 7] = scene.radius[contacts.a] / rbar
    F[:, 8] = np.where(wall, 0.0, scene.radius[np.where(wall, 0, contacts.b)] / rbar)
    deg = np.zeros(scene.M, dtype=np.int64)
    np.add.at(deg, contacts.a, 1)
    np.add.at(deg, contacts.b[~wall], 1)
    F[:, 9] = deg[contacts.a]
    F[:, 10] = np.where(wall, 0, deg[np.where(wall, 0, contacts.b)])
    return F


def targets(gamma_scaled, mu):
    g = gamma_scaled.reshape(-1, 3)
    gn = np.maximum(g[:, 0], 1e-6)
    y = np.zeros_like(g)
    y[:, 0] = np.log(gn)
    q = g[:, 1:] / (mu * g[:, 0:1])
    nq = np.maximum(1.0, np.linalg.norm(q, axis=1))
    y[:, 1:] = q / nq[:, None]
    return y


def forward(params, X):
    """Returns the outputs and the activations of every layer."""
    acts = [X]
    h = X
    nl = len(params) // 2
    for l in range(nl):
        W, b = params[2 * l], params[2 * l + 1]
        z = h @ W + b
        h = np.tanh(z) if l < nl - 1 else z
        acts.append(h)
    return h, acts


def loss_and_grad(params, X, Y):
    """MSE loss (mean over rows of the mean over the 3 outputs) and gradients."""
    P, acts = forward(params, X)
    B = X.shape[0]
    diff = P - Y
    loss = float((diff * diff).sum() / (3.0 * B))
    g = 2.0 * diff / (3.0 * B)
    grads = [None] * len(params)
    nl = len(params) // 2
    for l in range(nl - 1, -1, -1):
        hin = acts[l]
        grads[2 * l] = hin.T @ g
        grads[2 * l + 1] = g.sum(axis=0)
        if l > 0:
            g = (g @ params[2 * l].T) * (1.0 - acts[l] ** 2)
    return loss, grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state = (m, v, t)."""
    m, v, t = state
    t += 1
    for i, (p, g) in enumerate(zip(params, grads)):
        m[i] = b1 * m[i] + (1 - b1) * g
        v[i] = b2 * v[i] + (1 - b2) * g * g
        mh = m[i] / (1 - b1 ** t)
        vh = v[i] / (1 - b2 ** t)
        p -= lr * mh / (np.sqrt(vh) + eps)
    return (m, v, t)


def predict_gamma(params, Xn, mu):
    """Scaled impulses [Nc][3] strictly inside the cone."""
    P, _ = forward(params, Xn)
    gn = np.exp(P[:, 0])
    q = P[:, 1:]
    nq = np.maximum(1.0, np.linalg.norm(q, axis=1))
    gt = 0.9 * mu * gn[:, None] * q / nq[:, None]
    return np.concatenate([gn[:, None], gt], axis=1)
