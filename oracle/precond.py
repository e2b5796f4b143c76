"""Learned Davidson preconditioner: plain reference of what the library's
kernels compute.  Test infrastructure only.

The paper leaves the local solver open (Sec. 2.3); the method's solver here
is a Davidson iteration whose correction step is normally the diagonal
preconditioner t = -r / (diag H_eff - theta diag N_eff).  The learned
variant replaces it by a two-layer perceptron applied to every element of
the site tensor separately:

  features  f0 = |r_i| / rms(r)
            f1 = asinh(d_i),            d_i = dh_i - theta dn_i
            f2 = asinh(dn_i)
            f3 = asinh(-f0 / d_i'),     d_i' = d_i floored to |d_i| >= floor
            f4 = sign(r_i) t_i / rms(t), t = -r / d' (the diagonal correction)
  model     g(f) = w2 . relu(W1 f + b1) + b2
  correction t_i = sign(r_i) g(f)

The correction is odd in r, as a linear preconditioner is, so the sign of
the Ritz vector (free in an eigensolver) does not matter; the diagonal rule
is the special case g = f4 (up to scale).  The Davidson step normalises t,
so only its direction matters.  Training pairs come from the solver itself:
at iteration j of a converged local solve with Ritz vector x_j (unit norm)
and final vector x*, the exact correction is e_j = x*/(x_j . x*) - x_j, the
step after which the search space holds x*; sign(r_i) e_ij / rms(e_j) is
the target of g at element i.  Loss: mean squared error; optimiser: Adam
(Kingma and Ba, 2015).

Per-N-block scope (``groups`` given: one label per element, elements of one
label forming one N-block of the site tensor, i.e. sharing the particle
numbers of both bonds): the model sees the residual restricted to one
block.  The root mean squares in f0 and f4 are taken over the element's
block, the correction is sign(r_i) g(f) rms_b(t) (the model shapes the
correction inside a block, the diagonal rule keeps the weight of the
block), and the target divides e by its rms over the element's block.
Everything here is FP64 and element-by-element plain numpy.
"""
from __future__ import annotations

import numpy as np


def rms_over(v, groups=None):
    """Root mean square of v over the whole vector (groups None) or, element
    by element, over the element's group."""
    v = np.asarray(v, dtype=float)
    if groups is None:
        return np.full(v.size, np.sqrt(np.sum(v * v) / v.size))
    groups = np.asarray(groups)
    out = np.empty(v.size)
    for g in np.unique(groups):
        sel = groups == g
        out[sel] = np.sqrt(np.sum(v[sel] ** 2) / np.count_nonzero(sel))
    return out


def _safe_div(a, b):
    return np.where(b > 0, a / np.where(b > 0, b, 1.0), 0.0)


def diagonal_correction(r, dh, dn, theta, floor=1e-8):
    """t = -r / d' with d = dh - theta dn floored to |d'| >= floor."""
    d = dh - theta * dn
    dfl = np.where(np.abs(d) < floor, np.where(d < 0, -floor, floor), d)
    return -np.asarray(r, dtype=float) / dfl, d, dfl


def features(r, dh, dn, theta, floor=1e-8, groups=None):
    """Five features per element (n x 5); rms over the vector, or over the
    element's N-block when ``groups`` is given."""
    r = np.asarray(r, dtype=float)
    t, d, dfl = diagonal_correction(r, dh, dn, theta, floor)
    f0 = _safe_div(np.abs(r), rms_over(r, groups))
    f4 = _safe_div(np.sign(r) * t, rms_over(t, groups))
    return np.stack([f0, np.arcsinh(d), np.arcsinh(dn), np.arcsinh(-f0 / dfl), f4], axis=1)


def correction(p, r, dh, dn, theta, floor=1e-8, groups=None):
    """The learned correction t = sign(r) g(f(r)); per N-block it is scaled
    by the block rms of the diagonal correction."""
    y = np.sign(r) * forward(p, features(r, dh, dn, theta, floor, groups))
    if groups is not None:
        y = y * rms_over(diagonal_correction(r, dh, dn, theta, floor)[0], groups)
    return y


def target(r, x, xstar, groups=None):
    """Training target of g at every element: sign(r_i) e_i / rms(e), the
    rms over the vector or over the element's N-block."""
    return np.sign(r) * exact_correction(x, xstar, groups)


def forward(p, F):
    """Model output for feature rows F (n x 5)."""
    z = F @ np.asarray(p["W1"], float).T + np.asarray(p["b1"], float)[None, :]
    h = np.maximum(z, 0.0)
    return h @ np.asarray(p["w2"], float) + float(p["b2"])


def loss_and_grads(p, F, Y):
    """Mean squared error 0.5 * mean((y - Y)^2) and its gradients with
    respect to W1, b1, w2, b2 by the chain rule."""
    W1 = np.asarray(p["W1"], float)
    b1 = np.asarray(p["b1"], float)
    w2 = np.asarray(p["w2"], float)
    n = F.shape[0]
    z = F @ W1.T + b1[None, :]
    h = np.maximum(z, 0.0)
    y = h @ w2 + float(p["b2"])
    dy = (y - Y) / n
    loss = 0.5 * float(np.mean((y - Y) ** 2))
    g_w2 = h.T @ dy
    g_b2 = float(np.sum(dy))
    dz = np.outer(dy, w2) * (z > 0.0)
    g_W1 = dz.T @ F
    g_b1 = dz.sum(axis=0)
    return loss, {"W1": g_W1, "b1": g_b1, "w2": g_w2, "b2": g_b2}


def adam_step(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with bias correction; ``state`` holds m, v per
    parameter and the step count t (created on the first call)."""
    if not state:
        state.update({k: (np.zeros_like(np.asarray(v, float)), np.zeros_like(np.asarray(v, float)))
                      for k, v in p.items()})
        state["t"] = 0
    state["t"] += 1
    t = state["t"]
    out = {}
    for k in ("W1", "b1", "w2", "b2"):
        m, v = state[k]
        gk = np.asarray(g[k], float)
        m = beta1 * m + (1 - beta1) * gk
        v = beta2 * v + (1 - beta2) * gk * gk
        state[k] = (m, v)
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        out[k] = np.asarray(p[k], float) - lr * mh / (np.sqrt(vh) + eps)
    out["b2"] = float(out["b2"])
    return out


def exact_correction(x, xstar, groups=None):
    """e = x*/(x . x*) - x for unit x, divided by its rms over the vector or
    over each element's N-block (zero where that rms is zero)."""
    e = xstar / float(x @ xstar) - x
    return _safe_div(e, rms_over(e, groups))
