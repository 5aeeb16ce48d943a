"""Warm-start network oracle (FP64, optional BF16 rounding), test infrastructure.

The network predicts a tile's solution from its normalised blurred input
(a learned initialisation for the Local-Solver; the plain iterations always
follow it, so it only changes the starting point of Algorithm 1):

    a1 = relu(conv1(x)),  a2 = relu(conv2(a1)),  a3 = relu(conv3(a2)),
    out = x + conv4(a3)

with 3x3 convolutions (cross-correlation, zero padding, stride 1) of
1 -> 32 -> 32 -> 32 -> 1 channels and biases.  Loss = mean over pixels of
(out - target)^2.  Optimiser: Adam.

With ``bf16=True`` values are rounded to bfloat16 (round to nearest even,
through float32) at the points where the GPU kernels store BF16: the
network input x, every weight tensor used by a convolution, the
activations a1..a3, and the masked gradients dp1..dp3 that feed the
backward convolutions and weight gradients.  Everything else is FP64 here
(FP32 accumulate on the GPU).

Arrays are channel-last: images [B, H, W], activations [B, H, W, C],
weights [C_out, C_in, 3, 3].
"""
from __future__ import annotations

import numpy as np

CH = 32
LAYERS = [(1, CH), (CH, CH), (CH, CH), (CH, 1)]


def n_params():
    return sum(co * ci * 9 + co for ci, co in LAYERS)


def init_params(seed, scale_last=1.0):
    """He-initialised weights, zero biases; list of (W, b) per layer."""
    rng = np.random.default_rng(seed)
    params = []
    for li, (ci, co) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (ci * 9))
        if li == len(LAYERS) - 1:
            std *= scale_last
        params.append((rng.standard_normal((co, ci, 3, 3)) * std, np.zeros(co)))
    return params


def flatten(params):
    """Flat FP64 vector: per layer W (C_out, C_in, 3, 3) row-major, then b."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(vec):
    out, o = [], 0
    for ci, co in LAYERS:
        nw = co * ci * 9
        W = np.asarray(vec[o:o + nw], dtype=np.float64).reshape(co, ci, 3, 3)
        o += nw
        b = np.asarray(vec[o:o + co], dtype=np.float64)
        o += co
        out.append((W, b))
    return out


def round_bf16(a):
    """Round to bfloat16 (nearest, ties to even) via float32; returns float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(a, W, b):
    """out[n,y,x,o] = b[o] + sum_{c,dy,dx} W[o,c,dy,dx] a_pad[n, y+dy, x+dx, c]."""
    B, H, Wd, C = a.shape
    ap = np.zeros((B, H + 2, Wd + 2, C))
    ap[:, 1:-1, 1:-1, :] = a
    out = np.broadcast_to(b, (B, H, Wd, W.shape[0])).copy()
    for dy in range(3):
        for dx in range(3):
            out += ap[:, dy:dy + H, dx:dx + Wd, :] @ W[:, :, dy, dx].T
    return out


def conv3x3_grads(a, dp, W):
    """Gradients of conv3x3 w.r.t. its input, weights and bias given dL/dout = dp."""
    B, H, Wd, C = a.shape
    ap = np.zeros((B, H + 2, Wd + 2, C))
    ap[:, 1:-1, 1:-1, :] = a
    dap = np.zeros_like(ap)
    dW = np.zeros_like(W)
    for dy in range(3):
        for dx in range(3):
            patch = ap[:, dy:dy + H, dx:dx + Wd, :]
            dW[:, :, dy, dx] = np.einsum("nyxo,nyxc->oc", dp, patch)
            dap[:, dy:dy + H, dx:dx + Wd, :] += dp @ W[:, :, dy, dx]
    return dap[:, 1:-1, 1:-1, :], dW, dp.sum(axis=(0, 1, 2))


def forward(params, x, bf16=False):
    """x: [B, H, W] -> (out [B, H, W], cache)."""
    rnd = round_bf16 if bf16 else (lambda v: v)
    Ws = [rnd(W) for W, _ in params]
    bs = [b for _, b in params]
    x = np.asarray(x, dtype=np.float64)
    a0 = rnd(x)[..., None]
    acts, pres = [a0], []
    a = a0
    for li in range(3):
        p = conv3x3(a, Ws[li], bs[li])
        a = rnd(np.maximum(p, 0.0))
        pres.append(p)
        acts.append(a)
    r = conv3x3(a, Ws[3], bs[3])[..., 0]
    out = x + r
    return out, {"acts": acts, "Ws": Ws, "bf16": bf16}


def loss_and_grads(params, x, target, bf16=False):
    """Loss mean((out - target)^2) and its gradients (list of (dW, db))."""
    out, cache = forward(params, x, bf16)
    rnd = round_bf16 if bf16 else (lambda v: v)
    d = out - target
    loss = float(np.mean(d * d))
    dout = (2.0 / d.size) * d
    acts, Ws = cache["acts"], cache["Ws"]
    grads = [None] * 4
    dp = dout[..., None]
    da, dW, db = conv3x3_grads(acts[3], dp, Ws[3])
    grads[3] = (dW, db)
    for li in (2, 1, 0):
        dp = rnd(da * (acts[li + 1] > 0))
        da, dW, db = conv3x3_grads(acts[li], dp, Ws[li])
        grads[li] = (dW, db)
    return loss, grads, out


def adam_step(flat_params, flat_grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) of a flat parameter vector; returns
    (params, m, v).  step counts from 1."""
    m = b1 * m + (1 - b1) * flat_grad
    v = b2 * v + (1 - b2) * flat_grad * flat_grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat_params - lr * mh / (np.sqrt(vh) + eps), m, v
