"""FP64 reference of the learned bracket predictor (test infrastructure only).

The predictor maps the features of an element to its integration bracket
(the range [t0, t1] of Section 2.1, Eq. (7)-(8), as found by the method's own
range finder):

    features   z = ((log max(v, v_floor) - m_v) / s_v,  (log x - m_x) / s_x)
    network    h1 = clamp(W1 z + b1, -1, 1)   W1: 64 x 2,  b1: 64
               h2 = phi(W2 h1 + b2)           W2: 64 x 64, b2: 64
               y  = W3 h2 + b3                W3: 2 x 64,  b3: 2
    activations  the clamp (derivative 1 inside, 0 outside) and
               phi(a) = u (3 - u^2) / 2,  u = clamp(a / 1.5, -1, 1)
               (a cubic sigmoid shaped like tanh: odd, phi'(0) = 1, constant
               +-1 beyond |a| = 1.5, continuously differentiable), with
               phi'(a) = 1 - u^2 inside and 0 outside
    targets    y0* = t0 / t1,  y1* = log t1
    loss       L = (1/B) sum_s 1/2 (w0 e0^2 + w1 e1^2),  e = y - y*,
               w0 = alpha if e0 > 0 else 1   (t0 predicted too large is unsafe)
               w1 = alpha if e1 < 0 else 1   (t1 predicted too small is unsafe)

Parameter vector (float, 4482 trainable values) in this order:
W1 (row-major 64 x 2), b1, W2 (row-major 64 x 64, W2[i, j] multiplies h1[j]),
b2, W3 (row-major 2 x 64), b3.

Nothing here is shared with the GPU library; it is written from the definition
above and pinned by central differences in tests/test_mlp_ref.py.
"""

from __future__ import annotations

import numpy as np

H = 64
NPARAMS = 2 * H + H + H * H + H + 2 * H + 2  # 4482
V_FLOOR = 1e-3


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == NPARAMS
    o = 0
    W1 = p[o:o + 2 * H].reshape(H, 2); o += 2 * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + 2 * H].reshape(2, H); o += 2 * H
    b3 = p[o:o + 2]; o += 2
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, np.ravel(W3), b3]).astype(np.float64)


def features(v, x, norm):
    """norm = (m_v, s_v, m_x, s_x)."""
    v = np.abs(np.asarray(v, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    lv = np.log(np.maximum(v, V_FLOOR))
    lx = np.log(x)
    return np.stack([(lv - norm[0]) / norm[1], (lx - norm[2]) / norm[3]], axis=1)


ACT_C = 1.5


def phi(a):
    """The activation and its derivative, elementwise."""
    u = np.clip(np.asarray(a, dtype=np.float64) / ACT_C, -1.0, 1.0)
    return 0.5 * u * (3.0 - u * u), (1.5 / ACT_C) * (1.0 - u * u)


def hard_clamp(a):
    """The first layer's activation clamp(a, -1, 1) and its derivative."""
    a = np.asarray(a, dtype=np.float64)
    return np.clip(a, -1.0, 1.0), (np.abs(a) < 1.0).astype(np.float64)


def forward(p, z):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1, d1 = hard_clamp(z @ W1.T + b1)
    h2, d2 = phi(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    return y, (z, h1, h2, d1, d2)


def targets(t0, t1):
    t0 = np.asarray(t0, dtype=np.float64)
    t1 = np.asarray(t1, dtype=np.float64)
    return np.stack([t0 / t1, np.log(t1)], axis=1)


def loss_and_grad(p, z, ystar, alpha):
    """Mean asymmetric squared loss and its gradient with respect to p."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (z, h1, h2, d1, d2) = forward(p, z)
    B = z.shape[0]
    e = y - ystar
    w = np.ones_like(e)
    w[:, 0] = np.where(e[:, 0] > 0, alpha, 1.0)
    w[:, 1] = np.where(e[:, 1] < 0, alpha, 1.0)
    L = 0.5 * np.sum(w * e * e) / B
    dy = w * e / B                      # B x 2
    gW3 = dy.T @ h2                     # 2 x 64
    gb3 = dy.sum(axis=0)
    da2 = (dy @ W3) * d2                # B x 64
    gW2 = da2.T @ h1                    # 64 x 64
    gb2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * d1
    gW1 = da1.T @ z                     # 64 x 2
    gb1 = da1.sum(axis=0)
    return L, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(p, g, m, s, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); step counts from 1.  Returns (p, m, s)."""
    m = beta1 * m + (1 - beta1) * g
    s = beta2 * s + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** step)
    shat = s / (1 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(shat) + eps), m, s


def bracket_from_outputs(y, margin_t1, margin_t0):
    """Predicted bracket after widening: t0 = max(0, y0 - margin_t0) exp(y1),
    t1 = exp(y1 + margin_t1)."""
    t1 = np.exp(y[:, 1])
    t0 = np.maximum(0.0, y[:, 0] - margin_t0) * t1
    return t0, t1 * np.exp(margin_t1)
