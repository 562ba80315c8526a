"""FP64 oracle of the neural density field (test infrastructure only).

The field is not part of the paper: it is a small Fourier-feature MLP that is
trained on the (position, normalised density) pairs the method produces and
then answers density queries at arbitrary surface points.  This module is the
plain reference for the GPU kernels: the same network evaluated in FP64 with
bfloat16 round-to-nearest-even applied at the points where the GPU stores
bfloat16 values (features, weights, hidden activations, the back-propagated
pre-activation gradients that feed the matrix cores).  With ``bf16=False`` it is
the exact FP64 network, which its finite-difference pin checks.

Network: x -> x~ = (x - lo) / ext in [0,1]^3 -> 96 features
[sin, cos](2 pi f_b x~_a), f_b = max_cycles^(b/15), b = 0..15, a = x,y,z, feature
index 6b + 2a + (0 sin | 1 cos) -> 4 x (64, ReLU) -> 1 -> softplus.
Loss: mean squared error against the normalised density.
Parity status: pinned (central finite differences in FP64, closed forms of the
features and softplus; Adam: the first step, a constant gradient over ten steps
and two steps with changing gradients worked out by hand).
"""
from __future__ import annotations

import numpy as np

BANDS = 16
WIDTH = 64
FEAT = 6 * BANDS
LAYERS = 4
SHAPES = [("W1", (FEAT, WIDTH)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (WIDTH, WIDTH)), ("b4", (WIDTH,)),
          ("w5", (WIDTH,)), ("b5", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


MAX_CYCLES = 32.0


def freqs(max_cycles=None):
    mc = MAX_CYCLES if max_cycles is None else float(max_cycles)
    b = np.arange(BANDS, dtype=np.float64)
    return np.power(mc, b / (BANDS - 1)).astype(np.float32).astype(np.float64)


def bf16(x):
    """Round to bfloat16 (round-to-nearest-even on the float32 value), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def unflatten(flat):
    flat = np.asarray(flat, np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in SHAPES])


def features(x, lo, ext, bf=True, max_cycles=None):
    """[n][96] features of world points x [n][3] for a field box with corner lo and edge ext."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    xt = (x - np.asarray(lo, np.float64)) / float(ext)
    arg = 2.0 * np.pi * xt[:, None, :] * freqs(max_cycles)[None, :, None]        # [n][band][axis]
    phi = np.stack([np.sin(arg), np.cos(arg)], -1).reshape(len(x), FEAT)  # 6b + 2a + c
    return bf16(phi) if bf else phi


def softplus(o):
    return np.logaddexp(0.0, o)


def forward(flat, x, lo, ext, bf=True, max_cycles=None):
    """Returns (y [n], cache)."""
    p = unflatten(flat)
    q = (lambda a: bf16(a)) if bf else (lambda a: a)
    h = features(x, lo, ext, bf, max_cycles)
    hs, zs = [h], []
    for L in range(1, LAYERS + 1):
        z = h @ q(p[f"W{L}"]) + p[f"b{L}"]
        zs.append(z)
        h = q(np.maximum(z, 0.0))
        hs.append(h)
    o = h @ p["w5"] + p["b5"][0]
    y = softplus(o)
    return y, {"hs": hs, "zs": zs, "o": o, "p": p, "q": q}


def loss_and_grad(flat, x, target, lo, ext, bf=True, max_cycles=None):
    """Mean squared error over the batch and its gradient with respect to the flat parameters."""
    y, c = forward(flat, x, lo, ext, bf, max_cycles)
    t = np.asarray(target, np.float64).reshape(-1)
    B = len(t)
    loss = np.mean((y - t) ** 2)
    dy = 2.0 * (y - t) / B
    do = dy / (1.0 + np.exp(-c["o"]))                 # softplus' = sigmoid
    p, q, hs, zs = c["p"], c["q"], c["hs"], c["zs"]
    g = {"w5": hs[LAYERS].T @ do, "b5": np.array([do.sum()])}
    dh = np.outer(do, p["w5"])
    for L in range(LAYERS, 0, -1):
        dz = q(dh * (zs[L - 1] > 0.0))               # bf16 operand of the matrix products
        g[f"W{L}"] = hs[L - 1].T @ dz
        g[f"b{L}"] = dz.sum(axis=0)
        if L > 1:
            dh = dz @ q(p[f"W{L}"]).T
    return loss, flatten(g), y


def adam_step(flat, m, v, grad, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step counts from 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-uniform weights, zero biases (a plain reference initialisation)."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, shape in SHAPES:
        if name.startswith("W") or name == "w5":
            fan_in = shape[0]
            lim = np.sqrt(6.0 / fan_in)
            out[name] = rng.uniform(-lim, lim, shape)
        else:
            out[name] = np.zeros(shape)
    return flatten(out)
