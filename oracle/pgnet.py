"""Learned multigrid initial guess: FP64 reference of the small 3-D conv net (test infrastructure).

Not part of the paper's method: an extension that predicts the pressure
initial guess of the multigrid solve from the solver's own history.  The
reference computes in FP64 on inputs and weights that are already rounded to
bfloat16, so the GPU's BF16-storage / FP32-accumulate kernels can be compared
with it at a tolerance set by the BF16 activations.

Net (readings of the extension): input channels
    [(p_{m-1} - mu)/s, (p_{m-2} - mu)/s, z_m/(w dt s)]  (zero outside the box
    and on solid cells), mu and s the mean and RMS deviation of p_{m-1} over
    the active cells;
layers conv3^3(3->16) + ReLU, conv3^3(16->16) + ReLU, conv3^3(16->1), each a
cross-correlation  out[p] = b + sum_taps W[tap]^T in[p + off(tap)]  with zero
padding at the box faces; taps ordered tap = 9 (dz+1) + 3 (dy+1) + (dx+1);
weights W[tap][c_in][c_out].  Output d = (p_m - p_{m-1})/s; guess
p = p_{m-1} + s d.  Loss: mean over the loss mask of (e - mean(e))^2 with
e = d - d*, the mean removed because the pressure gauge is free.  Adam with
an FP32 master copy.

Arrays are channel-first [C, X, Y, Z] float64.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(a, dx, dy, dz):
    """b[..., x, y, z] = a[..., x+dx, y+dy, z+dz], zero outside the box."""
    out = np.zeros_like(a)
    X, Y, Z = a.shape[-3:]

    def rng(d, n):
        src = slice(max(d, 0), n + min(d, 0))
        dst = slice(max(-d, 0), n + min(-d, 0))
        return src, dst
    sx, tx = rng(dx, X)
    sy, ty = rng(dy, Y)
    sz, tz = rng(dz, Z)
    out[..., tx, ty, tz] = a[..., sx, sy, sz]
    return out


def conv3d(x, W, b):
    """Cross-correlation with 27 taps: out[o, p] = b[o] + sum_t sum_c W[t, c, o] x[c, p + off(t)]."""
    cout = W.shape[2]
    out = np.zeros((cout,) + x.shape[1:])
    for t, (dx, dy, dz) in enumerate(TAPS):
        xs = shift(x, dx, dy, dz)
        out += np.einsum("cxyz,co->oxyz", xs, W[t])
    return out + b[:, None, None, None]


def conv3d_input_grad(g, W):
    """Gradient of sum(g * conv3d(x, W, b)) w.r.t. x (the transposed correlation)."""
    cin = W.shape[1]
    out = np.zeros((cin,) + g.shape[1:])
    for t, (dx, dy, dz) in enumerate(TAPS):
        out += np.einsum("oxyz,co->cxyz", shift(g, -dx, -dy, -dz), W[t])
    return out


def conv3d_weight_grad(x, g):
    """Gradients of sum(g * conv3d(x, W, b)) w.r.t. W [27, cin, cout] and b [cout]."""
    dW = np.zeros((27, x.shape[0], g.shape[0]))
    for t, (dx, dy, dz) in enumerate(TAPS):
        dW[t] = np.einsum("cxyz,oxyz->co", shift(x, dx, dy, dz), g)
    return dW, g.sum(axis=(1, 2, 3))


def init_weights(seed=0, hidden=16, cin=3):
    """Kaiming-uniform init (bound sqrt(6/fan_in)) from a seeded numpy generator; biases 0."""
    rng = np.random.default_rng(seed)
    shapes = [(27, cin, hidden), (27, hidden, hidden), (27, hidden, 1)]
    params = []
    for s in shapes:
        bound = np.sqrt(6.0 / (27 * s[1]))
        params.append(rng.uniform(-bound, bound, size=s))
        params.append(np.zeros(s[2]))
    return params  # [W1, b1, W2, b2, W3, b3]


def forward(params, x, bf16=True):
    """Returns (y, cache). With bf16, inputs, weights and stored activations are BF16-rounded."""
    W1, b1, W2, b2, W3, b3 = params
    r = bf16_round if bf16 else (lambda a: a)
    x = r(x)
    z1 = conv3d(x, r(W1), r(b1))
    a1 = r(np.maximum(z1, 0.0))
    z2 = conv3d(a1, r(W2), r(b2))
    a2 = r(np.maximum(z2, 0.0))
    y = conv3d(a2, r(W3), r(b3))[0]
    return y, (x, a1, a2)


def loss_and_grad(y, target, mask):
    """Mean-removed MSE over mask and its gradient w.r.t. y."""
    n = int(mask.sum())
    e = np.where(mask, y - target, 0.0)
    ebar = e[mask].mean() if n else 0.0
    d = np.where(mask, e - ebar, 0.0)
    loss = float(np.sum(d * d) / max(n, 1))
    return loss, 2.0 * d / max(n, 1)


def backward(params, cache, dy, bf16=True):
    """Gradients [dW1, db1, dW2, db2, dW3, db3] of the loss given dL/dy."""
    W1, b1, W2, b2, W3, b3 = params
    r = bf16_round if bf16 else (lambda a: a)
    x, a1, a2 = cache
    g3 = dy[None]
    dW3, db3 = conv3d_weight_grad(a2, g3)
    g2 = conv3d_input_grad(g3, r(W3)) * (a2 > 0)
    dW2, db2 = conv3d_weight_grad(a1, g2)
    g1 = conv3d_input_grad(g2, r(W2)) * (a1 > 0)
    dW1, db1 = conv3d_weight_grad(x, g1)
    return [dW1, db1, dW2, db2, dW3, db3]


def adam(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the master weights (state: dict with t, m, v)."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    if "m" not in state:
        state["m"] = [np.zeros_like(p) for p in params]
        state["v"] = [np.zeros_like(p) for p in params]
    out = []
    for k, (p, g) in enumerate(zip(params, grads)):
        m = b1 * state["m"][k] + (1 - b1) * g
        v = b2 * state["v"][k] + (1 - b2) * g * g
        state["m"][k], state["v"][k] = m, v
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out


def features(p1, p2, z, wdt, active):
    """Normalised input channels and (mu, s) from the previous two pressures and the divergence."""
    n = int(active.sum())
    mu = float(p1[active].mean()) if n else 0.0
    s = float(np.sqrt(np.mean((p1[active] - mu) ** 2))) if n else 0.0
    if s == 0.0:
        s = 1.0
    f = np.zeros((3,) + p1.shape)
    f[0] = np.where(active, (p1 - mu) / s, 0.0)
    f[1] = np.where(active, (p2 - mu) / s, 0.0)
    f[2] = np.where(active, z / (wdt * s), 0.0)
    return f, mu, s
