"""Pins of the oracle's steady-flow kernels (first-order upwind advection added
to the explicit diffusion; the flow extension of P, Sec. 5) against results it
does not compute itself: binomial and shift closed forms of pure upwind
advection, mirror symmetry, dense powers of a whole-domain operator built here
face by face, mass conservation, and the flow-free kernels.  CPU only."""
from math import comb

import numpy as np
import pytest

import oracle
import synth


def _lin(shape, z, y, x):
    return (z * shape[1] + y) * shape[2] + x


def test_zero_flow_is_the_plain_kernel():
    d = synth.random_small((6, 7, 8), 3, r=2, n_sub=7, seed=31)
    src = np.arange(0, d.label.size, 5)
    plain = oracle.Problem(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)
    flow = oracle.Problem(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt, velocity=np.zeros((3,) + d.label.shape))
    assert np.array_equal(plain.kernels(src)[0], flow.kernels(src)[0])


@pytest.mark.parametrize("nu,n", [(0.5, 6), (1.0, 5), (0.25, 7)])
def test_pure_advection_closed_forms(nu, n):
    # one phase with D = 0 (no diffusion), u = nu h / dt towards +x: the upwind
    # scheme moves a binomial share nu per sub-step one cell downstream
    L = 24
    label = np.zeros((1, 1, L), dtype=np.uint8)
    u = np.zeros((3, 1, 1, L))
    u[0] = nu / 0.5
    p = oracle.Problem(label, np.array([0.0]), 8, n, 1.0, 0.5, velocity=u)
    s = 6
    G, mass = p.kernels([s])
    got = G[0, 8, 8, :]                                  # the x line through the source
    want = np.zeros(17)
    for k in range(n + 1):
        want[8 + k] = comb(n, k) * nu ** k * (1 - nu) ** (n - k)
    assert np.max(np.abs(got - want)) <= 1e-15
    assert abs(mass[0] - 1.0) <= 1e-15


def test_reversed_flow_mirrors_the_kernel():
    label = np.zeros((9, 9, 9), dtype=np.uint8)
    u = np.zeros((3, 9, 9, 9))
    u[0], u[1], u[2] = 0.3, -0.2, 0.1
    fwd = oracle.Problem(label, np.array([1.0]), 3, 6, 1.0, 0.1, velocity=u)
    bwd = oracle.Problem(label, np.array([1.0]), 3, 6, 1.0, 0.1, velocity=-u)
    s = _lin(label.shape, 4, 4, 4)
    a = fwd.kernels([s])[0][0]
    b = bwd.kernels([s])[0][0]
    assert np.max(np.abs(a - b[::-1, ::-1, ::-1])) <= 1e-15


def _dense_flow_operator(label, d_phase, dt, h, u):
    """One sub-step of diffusion + upwind advection on the whole domain as a
    dense matrix (column j = where the mass of cell j goes), face by face."""
    nz, ny, nx = label.shape
    N = label.size
    A = np.eye(N)

    def idx(x, y, z):
        return (z * ny + y) * nx + x

    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                i = idx(x, y, z)
                for ax, (x2, y2, z2) in enumerate(((x + 1, y, z), (x, y + 1, z), (x, y, z + 1))):
                    if x2 >= nx or y2 >= ny or z2 >= nz:
                        continue
                    j = idx(x2, y2, z2)
                    da, db = d_phase[label[z, y, x]], d_phase[label[z2, y2, x2]]
                    lam = (2 * da * db / (da + db)) * dt / (h * h) if da > 0 and db > 0 else 0.0
                    # diffusion between i and j
                    A[i, i] -= lam
                    A[j, i] += lam
                    A[j, j] -= lam
                    A[i, j] += lam
                    # upwind advection through the face, Courant number v
                    v = u[ax, z, y, x] * dt / h
                    if v > 0:
                        A[i, i] -= v
                        A[j, i] += v
                    else:
                        A[j, j] += v
                        A[i, j] -= v
    return A


def test_kernels_are_columns_of_the_dense_flow_operator_power():
    d = synth.random_small((3, 4, 5), 3, r=5, n_sub=6, seed=32, d_zero_phase=False)
    rng = np.random.default_rng(5)
    u = rng.uniform(-0.4, 0.4, size=(3,) + d.label.shape)
    p = oracle.Problem(d.label, d.d_phase, d.r, d.n_sub, d.h, 0.05, velocity=u)
    M = np.linalg.matrix_power(_dense_flow_operator(d.label, d.d_phase, p.dt, p.h, u), d.n_sub)
    src = np.arange(d.label.size)
    G, mass = p.kernels(src)
    nz, ny, nx = d.label.shape
    for q, s in enumerate(src):
        sz, sy, sx = np.unravel_index(s, d.label.shape)
        W, r = p.W, p.r
        win = G[q][r - sz:r - sz + nz, r - sy:r - sy + ny, r - sx:r - sx + nx]
        assert np.max(np.abs(win.ravel() - M[:, s])) <= 1e-14
        assert abs(mass[q] - 1.0) <= 1e-13
