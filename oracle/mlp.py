"""Learned warm start of the Newton solve (oracle).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP network kernels; never imported
by the product path.

The paper solves each implicit step by Newton's method from the previous state.  The warm
start predicts each node's displacement over the step with a small network and hands it to
Newton as the initial guess; Newton still decides convergence.  Definitions (the network is
not in the paper; these are the build's own, stated in the design notes):

* features of node i of a rod (26; a missing neighbour at a rod end replicated):
  v_{i-1} - v_i, v_{i+1} - v_i, v_i, the velocity change over the last step a_i = v_i - v_prev_i,
  x_{i-1} - 2 x_i + x_{i+1}, log10 E, the radius, the mean rest length of the edges at node i,
  the natural curvature at node i in 1/m (the nearest interior node's at the rod ends), the
  change of the velocity change j_i = a_i - (v_prev_i - v_prev2_i), and a_{i-1} - 2 a_i + a_{i+1};
* standardisation: z = (f - mean) / std per feature, computed in float64, rounded to float32;
* network 26 -> 256 -> 256 -> 3 with ReLU; every GEMM input (activations, weights and
  back-propagated gradients) is rounded to bfloat16 (round to nearest, ties to even); products
  of bfloat16 values are exact and are accumulated here in float64 (the kernels accumulate in
  float32); biases and master weights are float32;
* output: the displacement beyond the third-order extrapolation, dx = dt (v_i + a_i + j_i) + s y,
  with s the per-component root-mean-square of (dx - dt (v + a + j)) over the training data;
* loss: mean over the batch of the squared error summed over the three components; Adam
  (beta 0.9 / 0.999, eps 1e-8) on the float32 master weights.

Pinned by tests/test_oracle_mlp.py: the rounding against the library conversion, the
backward pass (without rounding) against automatic differentiation, Adam's first step against
its closed form, and the rounded forward pass against the unrounded one within the bfloat16
error bound.
"""
from __future__ import annotations

import numpy as np
import torch

N_IN, N_HID, N_OUT = 26, 256, 3


# ---------------------------------------------------------------------------
# bfloat16 rounding
# ---------------------------------------------------------------------------

def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32:
    keep the upper 16 bits of the float32 pattern after adding 0x7FFF plus the lowest kept
    bit; NaN stays NaN."""
    a = np.asarray(a, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def to_f32(a):
    """float64 -> float32, round to nearest even (numpy's conversion)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32)


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------

def rod_features(x, v, v_prev, v_prev2, kbar, E, h, ebar):
    """Features (N, 26) of one rod: x, v, v_prev, v_prev2 (N, 3) at the start of the step
    (v_prev the velocity before the previous step, v_prev2 the one before that), kbar (N-2, 2)
    in 1/m (or None for zero), E, h scalars, ebar (N-1,) rest edge lengths."""
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    vp = np.asarray(v_prev, dtype=np.float64)
    a = v - vp
    a_prev = vp - np.asarray(v_prev2, dtype=np.float64)
    n = x.shape[0]
    f = np.zeros((n, N_IN))
    for i in range(n):
        im, ip = max(i - 1, 0), min(i + 1, n - 1)
        f[i, 0:3] = v[im] - v[i]
        f[i, 3:6] = v[ip] - v[i]
        f[i, 6:9] = v[i]
        f[i, 9:12] = a[i]
        f[i, 12:15] = x[im] - 2.0 * x[i] + x[ip]
        f[i, 15] = np.log10(E)
        f[i, 16] = h
        f[i, 17] = ebar[0] if i == 0 else (ebar[n - 2] if i == n - 1 else 0.5 * (ebar[i - 1] + ebar[i]))
        if n >= 3 and kbar is not None:
            f[i, 18:20] = kbar[min(max(i, 1), n - 2) - 1]
        f[i, 20:23] = a[i] - a_prev[i]
        f[i, 23:26] = a[im] - 2.0 * a[i] + a[ip]
    return f


def standardise(f, mean, std):
    """z = (f - mean)/std in float64, rounded to float32."""
    return to_f32((np.asarray(f, dtype=np.float64) - mean) / std)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def init_params(seed=0):
    """He-uniform initial weights (float32 master copies), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def layer(n_out, n_in):
        lim = np.sqrt(6.0 / n_in)
        return rng.uniform(-lim, lim, size=(n_out, n_in)).astype(np.float32), np.zeros(n_out, dtype=np.float32)
    W1, b1 = layer(N_HID, N_IN)
    W2, b2 = layer(N_HID, N_HID)
    W3, b3 = layer(N_OUT, N_HID)
    return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "W3": W3, "b3": b3}


def _r(a, rounding):
    return bf16_round(a).astype(np.float64) if rounding else np.asarray(a, dtype=np.float64)


def forward(p, X, rounding=True):
    """Y (B, 3) and the cache of GEMM inputs.  X is the standardised float32 input."""
    x0 = _r(X, rounding)
    h1 = np.maximum(x0 @ _r(p["W1"], rounding).T + p["b1"].astype(np.float64), 0.0)
    h1 = to_f32(h1) if rounding else h1
    a1 = _r(h1, rounding)
    h2 = np.maximum(a1 @ _r(p["W2"], rounding).T + p["b2"].astype(np.float64), 0.0)
    h2 = to_f32(h2) if rounding else h2
    a2 = _r(h2, rounding)
    y = a2 @ _r(p["W3"], rounding).T + p["b3"].astype(np.float64)
    y = to_f32(y) if rounding else y
    return y, {"x0": x0, "a1": a1, "a2": a2, "h1": h1, "h2": h2}


def loss_and_backward(p, X, T, rounding=True):
    """Loss (mean over the batch of the summed squared error) and parameter gradients."""
    B = X.shape[0]
    y, c = forward(p, X, rounding)
    d = np.asarray(y, dtype=np.float64) - np.asarray(T, dtype=np.float64)
    L = float((d * d).sum() / B)
    dy = 2.0 * d / B
    dy = to_f32(dy) if rounding else dy
    g_y = _r(dy, rounding)
    dh2 = (g_y @ _r(p["W3"], rounding)) * (c["h2"] > 0)
    dh2 = to_f32(dh2) if rounding else dh2
    g_h2 = _r(dh2, rounding)
    dh1 = (g_h2 @ _r(p["W2"], rounding)) * (c["h1"] > 0)
    dh1 = to_f32(dh1) if rounding else dh1
    g_h1 = _r(dh1, rounding)
    grads = {
        "W3": g_y.T @ c["a2"], "b3": g_y.sum(0),
        "W2": g_h2.T @ c["a1"], "b2": g_h2.sum(0),
        "W1": g_h1.T @ c["x0"], "b1": g_h1.sum(0),
    }
    return L, y, grads


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step count t >= 1) of float32 master weights, in place."""
    for k in p:
        gk = np.asarray(g[k], dtype=np.float64)
        m[k] = b1 * m[k] + (1.0 - b1) * gk
        v[k] = b2 * v[k] + (1.0 - b2) * gk * gk
        mh = m[k] / (1.0 - b1 ** t)
        vh = v[k] / (1.0 - b2 ** t)
        p[k] = to_f32(p[k].astype(np.float64) - lr * mh / (np.sqrt(vh) + eps))
    return p, m, v


def zeros_like(p):
    return {k: np.zeros(a.shape, dtype=np.float64) for k, a in p.items()}


def autograd_reference(p, X, T):
    """float64 automatic differentiation of the unrounded network and loss (a pin)."""
    tp = {k: torch.tensor(a, dtype=torch.float64, requires_grad=True) for k, a in p.items()}
    x = torch.tensor(X, dtype=torch.float64)
    h1 = torch.relu(x @ tp["W1"].T + tp["b1"])
    h2 = torch.relu(h1 @ tp["W2"].T + tp["b2"])
    y = h2 @ tp["W3"].T + tp["b3"]
    L = ((y - torch.tensor(T, dtype=torch.float64)) ** 2).sum() / X.shape[0]
    L.backward()
    return float(L), {k: t.grad.numpy() for k, t in tp.items()}
