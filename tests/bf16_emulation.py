"""BF16-rounding emulation of the learned kernel generator (test
infrastructure; no GPU code).

The library's network rounds to BF16 (8 significant bits, round to nearest
even) at fixed points and nowhere else:

* the three input features of every window cell (the prior feature is the
  FP32 product prior * (1/20) before it is rounded);
* every weight (the FP32 master copy is rounded when packed for MFMA);
* every hidden activation, SiLU(pre-activation) of the first four layers;
* d loss / d logits (the FP64 expression, times 1 / batch, in FP32);
* every back-propagated gradient after the SiLU derivative.

Products of BF16 operands are exact in FP32 and are accumulated in FP32;
biases, pre-activations, the last layer's output, the logits (prior + output,
FP32) and the softmax / loss (FP64 from the FP32 logits) are never rounded to
BF16.  This module replays exactly those roundings in FP64 on top of the
oracle's convolutions, so the GPU's results can be held to the small
differences that accumulation order and width leave (~1e-4 relative), while
the plain FP64 oracle differs from both by the roundings themselves (~1e-2).
"""
from __future__ import annotations

import numpy as np

from oracle import surrogate as su


def bf16(x):
    """Round to BF16 (round to nearest even, through FP32) and widen to FP64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def features(label, d_phase, s, r, prior64):
    """The BF16 input features of the window of source s (channels 0..2)."""
    f = su.window_features(label, d_phase, s, r, prior64)
    p32 = np.asarray(prior64, dtype=np.float32)
    f2 = (p32 * np.float32(1.0 / su.PRIOR_SCALE)).astype(np.float64)
    return np.stack([bf16(f[0]), bf16(f32(f[1])), bf16(f2)])


def forward(params, feat, prior64):
    """FP32 logits and the cache of a BF16 network.  params: (w, b) per layer
    holding FP32 values; feat: the BF16 features."""
    acts, pre = [feat], []
    h = feat
    for l, (w, b) in enumerate(params):
        z = f32(su.conv3(h, bf16(w), b))
        pre.append(z)
        h = bf16(su.silu(z)) if l < 4 else z
        acts.append(h)
    logits = f32(np.asarray(prior64, dtype=np.float32) + np.asarray(h[0], dtype=np.float32))
    return logits, (acts, pre)


def backward(params, cache, dlogits, scale):
    """Gradients of the parameters of one window: d loss / d logits is scaled
    by the FP32 ``scale`` (1 / batch) and rounded, then back-propagated with
    the BF16 weights, each layer's gradient rounded after the SiLU
    derivative."""
    acts, pre = cache
    grads = [None] * 5
    dz = bf16(f32(np.asarray(dlogits, dtype=np.float64) * float(np.float32(scale))))[None]
    for l in range(4, -1, -1):
        w, _ = params[l]
        dx, dw, db = su.conv3_backward(acts[l], bf16(w), dz)
        grads[l] = (dw, db)
        if l == 0:
            break
        p = np.asarray(pre[l - 1], dtype=np.float32)
        s = np.float32(1.0) / (np.float32(1.0) + np.exp(-p))
        sg = s * (np.float32(1.0) + p * (np.float32(1.0) - s))
        dz = bf16(np.asarray(dx, dtype=np.float32) * sg)
    return grads
