"""Test helpers: device marshalling and result comparison (no method arithmetic)."""
from __future__ import annotations

import numpy as np


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def place(shape, s, G):
    """Scatter a W^3 window (z, y, x relative to s - r) into a zero grid."""
    nz, ny, nx = shape
    W = G.shape[0]
    r = W // 2
    sz, rem = divmod(int(s), nx * ny)
    sy, sx = divmod(rem, nx)
    out = np.zeros(shape, dtype=G.dtype)
    for wz in range(W):
        Z = sz - r + wz
        if not 0 <= Z < nz:
            continue
        for wy in range(W):
            Y = sy - r + wy
            if not 0 <= Y < ny:
                continue
            xs = [(sx - r + wx, wx) for wx in range(W) if 0 <= sx - r + wx < nx]
            for X, wx in xs:
                out[Z, Y, X] = G[wz, wy, wx]
    return out


def rel_l1(a, b):
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def window_sources(shape, point, r):
    """Linear indices of every source whose window contains ``point`` (z, y, x)."""
    nz, ny, nx = shape
    z, y, x = point
    zs = range(max(0, z - r), min(nz, z + r + 1))
    ys = range(max(0, y - r), min(ny, y + r + 1))
    xs = range(max(0, x - r), min(nx, x + r + 1))
    return np.array([(sz * ny + sy) * nx + sx for sz in zs for sy in ys for sx in xs], dtype=np.int64)


def oracle_point(problem, c_old, point):
    """c_new at one cell from the oracle's kernels of all sources that reach it."""
    r = problem.r
    shape = problem.label.shape
    src = window_sources(shape, point, r)
    src = src[c_old.ravel()[src] != 0.0]
    if src.size == 0:
        return 0.0
    G, _ = problem.kernels(src)
    nz, ny, nx = shape
    z, y, x = point
    total = 0.0
    for k, s in enumerate(src):
        sz, rem = divmod(int(s), nx * ny)
        sy, sx = divmod(rem, nx)
        total += c_old.ravel()[s] * G[k, z - sz + r, y - sy + r, x - sx + r]
    return total
