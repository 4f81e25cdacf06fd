"""Window kernels with 16-bit neighbour copies: the arithmetic of the
reduced-precision modes, with the state kept exact.

TEST INFRASTRUCTURE ONLY: the tests use it; the product library never loads,
links or calls it, and it shares no code with the HIP path.

What it computes.  The window kernel of Sec. 3.1 (the column of P: an
explicit 7-point finite-difference solution from a unit point source, the
same scheme, walls and face coefficients as the FP64 oracle) where every
sub-step publishes the state as copies rounded to the nearest value of a
16-bit format (ties to even) and each face moves lambda_f (copy of the
neighbour - copy of the cell).  The state itself stays in FP64 here (FP32 on
the device).  Because the two cells of a face use the same two copies, the
amounts they exchange are equal and opposite, so the kernel keeps its mass
whatever the rounding (Sec. 3.3 relies on mass conservation to accept reduced
precision).  The device modes FP16X32 / BF16X32 also divide the kernel by its
mass at the end; ``kernels`` returns the mass beside the kernel.  With
``state=True`` the state itself is rounded to the format after every sub-step
(the FP16_STATE / BF16_STATE control modes: the copies are then the state).

Formats: FP16 (11 significant bits, smallest normal 2^-14, subnormal step
2^-24) and BF16 (8 significant bits, smallest normal 2^-126, subnormal step
2^-133), values of the kernels stay inside [0, 1], far from either format's
overflow.  ``FP64`` (53 bits) leaves every value unchanged and reduces the
scheme to the FP64 oracle's.
"""
import math

import numpy as np

# (significant bits, exponent of the smallest normal number)
FP16 = (11, -14)
BF16 = (8, -126)
FP64 = (53, -1022)


def round_to_format(x, fmt):
    """Round FP64 values to the nearest number of the binary format ``fmt``
    (significant bits, smallest normal exponent), ties to even.  The step of
    the format at |x| is 2^(max(e, emin) - (bits - 1)) with e the exponent of
    x's leading bit; dividing and multiplying by a power of two are exact."""
    bits, emin = fmt
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)                     # |x| = m 2^e, m in [0.5, 1): leading bit 2^(e - 1)
    lead = np.maximum(e - 1, emin)
    step = np.ldexp(1.0, lead - (bits - 1))
    out = np.rint(x / step) * step         # rint: nearest, ties to even
    return np.where(x == 0.0, x, out)


def _substeps(g, lx, ly, lz, n_sub, fmt, state=False):
    """n_sub sub-steps on a box (z, y, x) with no flux through its walls;
    lx / ly / lz: the box's owned +x / +y / +z face coefficients (0 on the
    box's last plane of each axis).  Terms per cell in the order -x, +x, -y,
    +y, -z, +z, each lambda (copy of the neighbour - copy of the cell);
    state: the new state is rounded to the format as well."""
    for _ in range(n_sub):
        h = round_to_format(g, fmt)
        acc = g.copy()
        acc[:, :, 1:] += lx[:, :, :-1] * (h[:, :, :-1] - h[:, :, 1:])
        acc[:, :, :-1] += lx[:, :, :-1] * (h[:, :, 1:] - h[:, :, :-1])
        acc[:, 1:, :] += ly[:, :-1, :] * (h[:, :-1, :] - h[:, 1:, :])
        acc[:, :-1, :] += ly[:, :-1, :] * (h[:, 1:, :] - h[:, :-1, :])
        acc[1:, :, :] += lz[:-1, :, :] * (h[:-1, :, :] - h[1:, :, :])
        acc[:-1, :, :] += lz[:-1, :, :] * (h[1:, :, :] - h[:-1, :, :])
        g = round_to_format(acc, fmt) if state else acc
    return g


def kernels(problem, src, fmt, state=False):
    """Window kernels of the sources ``src`` of an ``oracle.Problem`` with
    copies in ``fmt`` (and the state rounded too if ``state``): G [n_src, W,
    W, W] (z, y, x relative to s - r, zeros outside the domain) and the
    masses [n_src] (not divided out)."""
    p = problem
    src = np.asarray(src, dtype=np.int64).ravel()
    W, r = p.W, p.r
    nz, ny, nx = p.label.shape
    shape = (nz, ny, nx)
    lx, ly, lz = (a.reshape(shape) for a in (p.lx, p.ly, p.lz))
    G = np.zeros((src.size, W, W, W))
    mass = np.zeros(src.size)
    for q, s in enumerate(src):
        sx, sy, sz = int(s % nx), int((s // nx) % ny), int(s // (nx * ny))
        lo = [max(0, c - r) for c in (sz, sy, sx)]
        hi = [min(n - 1, c + r) for c, n in zip((sz, sy, sx), shape)]
        box = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
        # the box's own faces: the last plane of each axis is the window wall
        bx, by, bz = lx[box].copy(), ly[box].copy(), lz[box].copy()
        bx[:, :, -1] = 0.0
        by[:, -1, :] = 0.0
        bz[-1, :, :] = 0.0
        g = np.zeros(tuple(b - a + 1 for a, b in zip(lo, hi)))
        g[sz - lo[0], sy - lo[1], sx - lo[2]] = 1.0
        g = _substeps(g, bx, by, bz, p.n_sub, fmt, state)
        w0 = [a - (c - r) for a, c in zip(lo, (sz, sy, sx))]
        G[q, w0[0]:w0[0] + g.shape[0], w0[1]:w0[1] + g.shape[1], w0[2]:w0[2] + g.shape[2]] = g
        mass[q] = math.fsum(g.ravel())
    return G, mass


def error_bound(n_sub, lam_max, fmt, state=False):
    """Largest |G_copies - G_exact| after n_sub sub-steps for kernels inside
    [0, 1]: the exact update is a convex combination (6 lambda <= 1), so it
    carries an earlier difference over without growth, and each sub-step adds
    at most sum_f lambda_f (|copy - value| of both cells) <= 12 lambda_max u,
    u = 2^-bits the copies' relative rounding bound; rounding the state adds u
    more per sub-step (values <= 1)."""
    bits, _ = fmt
    u = 2.0 ** (-bits)
    return n_sub * (12.0 * lam_max * u + (u if state else 0.0))
