"""FP64 CPU oracle of the learned kernel generator (the surrogate of the
window FD), test infrastructure only.

The surrogate is not in the paper (arXiv 2408.11376 computes P by explicit FD,
Sec. 3.1); it is the learned extension of the hot path.  Its definition, which
the GPU path implements in BF16 / FP32:

Features of the window of source s (W = 2r + 1 cells per axis, z, y, x relative
to s - r), three channels per cell:
    f0 = 1 if the cell is inside the domain and D > 0, else 0
    f1 = (max(log10 D, -12) + 6) / 6 inside the domain, -1 outside
    f2 = log(max(U, 1e-30)) / 20, U = the uniform-D window kernel (same r, n,
         lambda = 0.9 / 6, reflecting window walls), i.e. the prior
Network: five 3x3x3 convolutions with zero "same" padding,
    3 -> 16 -> 16 -> 16 -> 16 -> 1 channels, SiLU after the first four;
    logits = 20 * f2 + conv5 output (residual on the prior log-kernel).
Kernel: G = softmax of the logits over the structural support S (cells
reachable from s through faces with lambda > 0 inside the window, in at most
n_sub face crossings); G = 0 outside S.
Loss per window: KL(q || G) + sum |q - G| over S, with q the FD kernel
normalised to unit mass; a batch takes the mean.

Weights: layer l has w[l] of shape [co][ci][3][3][3] (tap order z, y, x) and
b[l] of shape [co].
"""
from __future__ import annotations

import numpy as np

CHANNELS = (3, 16, 16, 16, 16, 1)
PRIOR_SCALE = 20.0
LOGD_FLOOR = -12.0


def param_shapes():
    shapes = []
    for l in range(5):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        shapes.append(((co, ci, 3, 3, 3), (co,)))
    return shapes


def num_params():
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes())


def unflatten(theta):
    """Flat FP32/FP64 vector -> list of (w, b) in layer order (w then b)."""
    out, o = [], 0
    for ws, bs in param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((np.asarray(theta[o:o + nw], dtype=np.float64).reshape(ws),
                    np.asarray(theta[o + nw:o + nw + nb], dtype=np.float64)))
        o += nw + nb
    return out


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def silu(x):
    return x / (1.0 + np.exp(-x))


def silu_grad(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def conv3(x, w, b):
    """x [ci][W][W][W], w [co][ci][3][3][3], b [co] -> [co][W][W][W]; zero
    'same' padding; y[co, z, y, x] = b[co] + sum w[co, ci, dz, dy, dx] *
    x[ci, z + dz - 1, y + dy - 1, x + dx - 1]."""
    ci, n = x.shape[0], x.shape[1]
    xp = np.zeros((ci, n + 2, n + 2, n + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    y = np.zeros((w.shape[0], n, n, n)) + b[:, None, None, None]
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                patch = xp[:, dz:dz + n, dy:dy + n, dx:dx + n]          # [ci][n][n][n]
                y += np.tensordot(w[:, :, dz, dy, dx], patch, axes=(1, 0))
    return y


def conv3_backward(x, w, dy):
    """Gradients of conv3 wrt x, w, b given dy [co][W][W][W]."""
    ci, n = x.shape[0], x.shape[1]
    xp = np.zeros((ci, n + 2, n + 2, n + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for dz in range(3):
        for dy_ in range(3):
            for dx in range(3):
                patch = xp[:, dz:dz + n, dy_:dy_ + n, dx:dx + n]
                dw[:, :, dz, dy_, dx] = np.tensordot(dy, patch, axes=([1, 2, 3], [1, 2, 3]))
                dxp[:, dz:dz + n, dy_:dy_ + n, dx:dx + n] += np.tensordot(w[:, :, dz, dy_, dx], dy, axes=(0, 0))
    db = dy.sum(axis=(1, 2, 3))
    return dxp[:, 1:-1, 1:-1, 1:-1], dw, db


def forward(params, feat):
    """feat [3][W][W][W] -> (logits [W][W][W], cache)."""
    acts, pre = [feat], []
    h = feat
    for l, (w, b) in enumerate(params):
        z = conv3(h, w, b)
        pre.append(z)
        h = silu(z) if l < 4 else z
        acts.append(h)
    logits = PRIOR_SCALE * feat[2] + h[0]
    return logits, (acts, pre)


def masked_softmax(logits, support):
    s = support.astype(bool)
    g = np.zeros_like(logits)
    if not s.any():
        return g
    z = logits[s]
    z = z - z.max()
    e = np.exp(z)
    g[s] = e / e.sum()
    return g


def loss_and_dlogits(g, q, support):
    """Loss KL(q || g) + L1(q, g) over the support and its gradient wrt the
    logits of the masked softmax g = softmax(logits | support)."""
    s = support.astype(bool)
    gs, qs = g[s], q[s]
    with np.errstate(divide="ignore", invalid="ignore"):
        kl = np.where(qs > 0, qs * (np.log(np.where(qs > 0, qs, 1.0)) - np.log(gs)), 0.0).sum()
    l1 = np.abs(qs - gs).sum()
    sign = np.sign(qs - gs)
    sbar = (sign * gs).sum()
    dz = np.zeros_like(g)
    dz[s] = (gs - qs) + gs * (sbar - sign)
    return kl + l1, dz


def backward(params, cache, dlogits):
    """Gradients of the parameters given d loss / d logits."""
    acts, pre = cache
    grads = [None] * 5
    dh = dlogits[None]                                   # d/d conv5 output [1][W][W][W]
    for l in range(4, -1, -1):
        w, b = params[l]
        dz = dh if l == 4 else dh * silu_grad(pre[l])
        dx, dw, db = conv3_backward(acts[l], w, dz)
        grads[l] = (dw, db)
        dh = dx
    return grads


def init_params(seed: int, scale: float = 1.0):
    """Deterministic initialisation from a SplitMix64 stream (He-style for
    the SiLU layers, a small last layer so the start is the prior)."""
    import synth
    params, o = [], 0
    for l, (ws, bs) in enumerate(param_shapes()):
        nw = int(np.prod(ws))
        fan_in = ws[1] * 27
        std = scale * np.sqrt(2.0 / fan_in) * (0.1 if l == 4 else 1.0)
        w = synth.normal(seed * 10 + l, nw).reshape(ws) * std
        params.append((w, np.zeros(bs)))
    return params


# ----------------------------------------------------------------- features

def window_features(label, d_phase, s, r, prior_logu):
    """Three feature channels [3][W][W][W] of the window of source s."""
    nz, ny, nx = label.shape
    W = 2 * r + 1
    sz, rem = divmod(int(s), nx * ny)
    sy, sx = divmod(rem, nx)
    f = np.zeros((3, W, W, W))
    f[1] = -1.0
    for wz in range(W):
        Z = sz - r + wz
        if not 0 <= Z < nz:
            continue
        for wy in range(W):
            Y = sy - r + wy
            if not 0 <= Y < ny:
                continue
            for wx in range(W):
                X = sx - r + wx
                if not 0 <= X < nx:
                    continue
                D = d_phase[label[Z, Y, X]]
                f[0, wz, wy, wx] = 1.0 if D > 0 else 0.0
                f[1, wz, wy, wx] = (max(np.log10(D), LOGD_FLOOR) if D > 0 else LOGD_FLOOR) / 6.0 + 1.0
    f[2] = prior_logu / PRIOR_SCALE
    return f


def prior_log_uniform(r, n_sub):
    """log of the uniform-D kernel of an unclipped window (lambda = 0.15 on
    every face, reflecting walls), from the oracle's own window FD."""
    import oracle
    W = 2 * r + 1
    label = np.zeros((W, W, W), dtype=np.uint8)
    p = oracle.Problem(label, np.array([1.0]), r, n_sub, 1.0, 0.0)
    G, _ = p.kernels([((r * W) + r) * W + r])
    return np.log(np.maximum(G[0], 1e-30))
