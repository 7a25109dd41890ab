"""FP64 reference of the learned-proposal network (not part of the paper).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
CPU-baseline leg of the benchmark are the only callers.

The network maps the 16 per-variable features X (``features`` in the C part
of this package) to one logit per variable:

    xq  = bf16(X)                         W1q, W2q, w3q = bf16(W1, W2, w3)
    a1  = xq @ W1q + b1                   h1 = relu(a1),  h1q = bf16(h1)
    a2  = h1q @ W2q + b2                  h2 = relu(a2)
    out = h2 @ w3q + b3                   (one logit per row)

bf16() rounds to the nearest bfloat16 value, ties to even, directly from the
real value.  Loss: mean binary cross-entropy with logits against labels y in
{0, 1}, optionally weighted per row.  Gradients are those of this function
with the rounded tensors held fixed: the gradient with respect to a master
weight is the gradient with respect to its rounded copy, and the derivative
of relu at h1q is taken as [h1q > 0].  Everything here is float64 and written
as the plain matrix products; a library matmul is the only primitive.
"""
from __future__ import annotations

import numpy as np

D_IN, D_HID = 16, 128
SHAPES = {"W1": (D_IN, D_HID), "b1": (D_HID,), "W2": (D_HID, D_HID), "b2": (D_HID,), "w3": (D_HID,), "b3": (1,)}
ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")
NUM_PARAMS = sum(int(np.prod(s)) for s in SHAPES.values())


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significant bits), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)  # x = m * 2^e, 0.5 <= |m| < 1
    scale = np.ldexp(1.0, e - 8)
    out = np.round(x / scale) * scale  # np.round: halves to even
    return np.where(x == 0, 0.0, out)


def init_params(seed: int) -> dict:
    """He-style initialisation (float32 master values, returned as float64)."""
    g = np.random.default_rng(seed)
    p = {
        "W1": g.normal(0, np.sqrt(2.0 / D_IN), SHAPES["W1"]),
        "b1": np.zeros(D_HID),
        "W2": g.normal(0, np.sqrt(2.0 / D_HID), SHAPES["W2"]),
        "b2": np.zeros(D_HID),
        "w3": g.normal(0, np.sqrt(1.0 / D_HID), SHAPES["w3"]),
        "b3": np.zeros(1),
    }
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in ORDER])


def unflatten(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == NUM_PARAMS
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = flat[o:o + n].reshape(SHAPES[k]).copy()
        o += n
    return out


def forward(p: dict, X, quantize: bool = True) -> dict:
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    xq = q(X)
    W1q, W2q, w3q = q(p["W1"]), q(p["W2"]), q(p["w3"])
    a1 = xq @ W1q + p["b1"]
    h1q = q(np.maximum(a1, 0.0))
    a2 = h1q @ W2q + p["b2"]
    h2 = np.maximum(a2, 0.0)
    out = h2 @ w3q + p["b3"][0]
    return dict(xq=xq, W1q=W1q, W2q=W2q, w3q=w3q, a1=a1, h1q=h1q, a2=a2, h2=h2, out=out)


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss_and_grad(p: dict, X, y, w=None, quantize: bool = True):
    """Mean weighted BCE-with-logits and its gradient with respect to every
    parameter (dict of float64 arrays shaped like the parameters)."""
    f = forward(p, X, quantize)
    y = np.asarray(y, dtype=np.float64)
    B = y.size
    w = np.ones(B) if w is None else np.asarray(w, dtype=np.float64)
    out = f["out"]
    loss = float(np.sum(w * (softplus(out) - y * out)) / B)
    dout = w * (sigmoid(out) - y) / B
    g = {"w3": f["h2"].T @ dout, "b3": np.array([dout.sum()])}
    da2 = dout[:, None] * f["w3q"][None, :] * (f["a2"] > 0)
    g["W2"] = f["h1q"].T @ da2
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ f["W2q"].T) * (f["h1q"] > 0)
    g["W1"] = f["xq"].T @ da1
    g["b1"] = da1.sum(axis=0)
    return loss, g, f


def abs_grad_bound(p: dict, X, y, w=None):
    """The same products as loss_and_grad with every factor replaced by its
    absolute value: the scale of the rounding error of any ordering of the sums."""
    f = forward(p, X, True)
    y = np.asarray(y, dtype=np.float64)
    B = y.size
    w = np.ones(B) if w is None else np.asarray(w, dtype=np.float64)
    dout = np.abs(w * (sigmoid(f["out"]) - y)) / B + np.abs(w) / B * 1e-7
    g = {"w3": f["h2"].T @ dout, "b3": np.array([dout.sum()])}
    da2 = dout[:, None] * np.abs(f["w3q"])[None, :] * (f["a2"] > 0)
    g["W2"] = f["h1q"].T @ da2
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ np.abs(f["W2q"]).T) * (f["h1q"] > 0)
    g["W1"] = np.abs(f["xq"]).T @ da1
    g["b1"] = da1.sum(axis=0)
    return g


def fragile_rows(p: dict, X, rel: float = 1e-6) -> np.ndarray:
    """Rows whose rounding or relu decisions could go either way under FP32
    accumulation: a pre-activation within rel of its absolute-sum scale from 0,
    or h1 within that distance of a bfloat16 rounding midpoint."""
    f = forward(p, X, True)
    s1 = np.abs(f["xq"]) @ np.abs(f["W1q"]) + np.abs(p["b1"])
    s2 = f["h1q"] @ np.abs(f["W2q"]) + np.abs(p["b2"])
    bad = (np.abs(f["a1"]) <= rel * s1).any(axis=1) | (np.abs(f["a2"]) <= rel * s2).any(axis=1)
    h1 = np.maximum(f["a1"], 0.0)
    m, e = np.frexp(h1)
    step = np.ldexp(1.0, e - 8)
    frac = h1 / step - np.floor(h1 / step)  # 0.5 = exactly between two bf16 values
    near = (np.abs(frac - 0.5) * step <= rel * s1) & (h1 > 0)
    return bad | near.any(axis=1)


def adam(p: dict, g: dict, m: dict, v: dict, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma and Ba, 2015) on each parameter; t is the 1-based step."""
    for k in ORDER:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
