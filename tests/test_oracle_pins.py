"""Pins of the CPU oracle against results fixed by the mathematics.

Each test checks the oracle against something it does not compute itself:
closed forms of the explicit scheme, exact rational brute force, dense matrix
powers of the whole-domain operator, and invariants (mass, positivity,
symmetry, linearity).  No GPU is involved.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from closed_forms import (dense_operator, matpow_exact, two_cell, uniform_box_kernel,
                          uniform_line_kernel)


def _uniform_problem(shape, r, n, dt=0.15):
    label = np.zeros(shape, dtype=np.uint8)
    return oracle.Problem(label, np.array([1.0]), r, n, 1.0, dt)


def _lin(shape, z, y, x):
    return (z * shape[1] + y) * shape[2] + x


# ------------------------------------------------------------------ coefficients

def test_dt_from_stability_limit():
    label = np.zeros((3, 3, 3), dtype=np.uint8)
    label[1, 1, 1] = 1
    # Dmax = 4 -> 0.9 h^2 / (6 * 4) with h = 0.5
    assert oracle.resolve_dt(label, np.array([1.0, 4.0]), 0.5, 0.0) == (0.9 * 0.25) / 24.0
    assert oracle.resolve_dt(label, np.array([1.0, 4.0]), 0.5, 0.01) == 0.01
    # a table entry no cell uses does not count
    assert oracle.resolve_dt(np.zeros((2, 2, 2), np.uint8), np.array([1.0, 9.0])) == 0.9 / 6.0


def test_face_coefficients_special_cases():
    # cells along x: D = 1, 1, 1e-6, 0
    label = np.array([[[0, 0, 1, 2]]], dtype=np.uint8)
    lx, ly, lz, dt = oracle.coefficients(label, np.array([1.0, 1e-6, 0.0]), 1.0, 0.15)
    assert dt == 0.15
    assert lx[0, 0, 0] == 0.15                       # uniform: D dt / h^2
    # harmonic mean of (1, 1e-6), exact rational value rounded once to FP64
    d1, d2 = Fraction(1), Fraction(1e-6)
    exact = 2 * d1 * d2 / (d1 + d2) * Fraction(0.15)
    assert abs(Fraction(lx[0, 0, 1]) - exact) <= Fraction(2 ** -52) * exact
    assert lx[0, 0, 2] == 0.0                        # impermeable neighbour
    assert lx[0, 0, 3] == 0.0                        # domain wall
    assert np.all(ly == 0.0) and np.all(lz == 0.0)   # single-cell thick in y, z


def test_two_cell_closed_form_pins_harmonic_mean():
    for d1, d2, n in [(1.0, 1e-6, 7), (0.3, 2.0, 25), (1.0, 1.0, 40), (1.0, 0.0, 5)]:
        label = np.array([[[0, 1]]], dtype=np.uint8)
        p = oracle.Problem(label, np.array([d1, d2]), r=1, n_sub=n, h=0.7, dt=0.05)
        G, m = p.kernels([0])
        g1, g2 = two_cell(n, d1, d2, 0.05, 0.7)
        # window (3x3x3) around source 0: source at centre (1,1,1), neighbour +x
        assert G[0, 1, 1, 1] == pytest.approx(g1, abs=1e-15)
        assert G[0, 1, 1, 2] == pytest.approx(g2, abs=1e-15)
        assert abs(m[0] - 1.0) < 1e-15


# ------------------------------------------------------------------ window kernels

def test_zero_substeps_is_identity():
    d = synth.random_small((5, 6, 7), 3, r=2, n_sub=0, seed=3)
    p = oracle.Problem.from_domain(d)
    G, m = p.kernels([0, 17, 100, 209])
    W = p.W
    for g in G:
        e = np.zeros((W, W, W))
        e[2, 2, 2] = 1.0
        assert np.array_equal(g, e)
    c_new, _, _ = p.step(d.c0)
    assert np.array_equal(c_new, d.c0)


def test_one_substep_weights():
    d = synth.random_small((6, 6, 6), 3, r=2, n_sub=1, seed=5)
    p = oracle.Problem.from_domain(d)
    s = _lin(d.shape, 3, 2, 4)
    G, _ = p.kernels([s])
    g = G[0]
    lam = {(0, 0, -1): p.lx[3, 2, 3], (0, 0, 1): p.lx[3, 2, 4],
           (0, -1, 0): p.ly[3, 1, 4], (0, 1, 0): p.ly[3, 2, 4],
           (-1, 0, 0): p.lz[2, 2, 4], (1, 0, 0): p.lz[3, 2, 4]}
    c = 2
    for (dz, dy, dx), l in lam.items():
        assert g[c + dz, c + dy, c + dx] == l
    assert g[c, c, c] == pytest.approx(1.0 - sum(lam.values()), abs=6e-16)
    assert np.count_nonzero(g) <= 7


@pytest.mark.parametrize("n,r", [(5, 3), (12, 3), (40, 3), (20, 4)])
def test_uniform_interior_window_matches_multinomial_closed_form(n, r):
    W = 2 * r + 1
    shape = (W + 6, W + 4, W + 5)
    p = _uniform_problem(shape, r, n)
    s = _lin(shape, r + 3, r + 2, r + 2)                 # window fully inside the domain
    G, m = p.kernels([s])
    ref = uniform_box_kernel(n, 0.15, (W, W, W), (r, r, r))
    assert np.max(np.abs(G[0] - ref)) <= 1e-14
    assert abs(m[0] - 1.0) <= 1e-13


def test_uniform_clipped_window_matches_closed_form():
    # source 1 cell from the x=0 wall and 2 from the top z wall: clipped box
    r, n = 4, 30
    shape = (12, 11, 10)
    p = _uniform_problem(shape, r, n)
    sz, sy, sx = 9, 5, 1
    G, _ = p.kernels([_lin(shape, sz, sy, sx)])
    zlo, zhi = sz - r, min(shape[0] - 1, sz + r)
    ylo, yhi = sy - r, sy + r
    xlo, xhi = 0, sx + r
    box = (zhi - zlo + 1, yhi - ylo + 1, xhi - xlo + 1)
    ref = uniform_box_kernel(n, 0.15, box, (sz - zlo, sy - ylo, sx - xlo))
    W = 2 * r + 1
    full = np.zeros((W, W, W))
    full[zlo - (sz - r):zhi - (sz - r) + 1, ylo - (sy - r):yhi - (sy - r) + 1,
         xlo - (sx - r):xhi - (sx - r) + 1] = ref
    assert np.max(np.abs(G[0] - full)) <= 1e-14


def test_line_domain_is_exact_1d_kernel():
    L, r, n = 15, 7, 60
    p = _uniform_problem((1, 1, L), r, n, dt=0.2)
    for pos in (0, 3, 7, 14):
        G, _ = p.kernels([pos])
        lo = max(0, pos - r)
        hi = min(L - 1, pos + r)
        ref = uniform_line_kernel(n, 0.2, hi - lo + 1, pos - lo)
        got = G[0][r, r, lo - (pos - r): hi - (pos - r) + 1]
        assert np.max(np.abs(got - ref)) <= 1e-14
        assert np.count_nonzero(G[0]) == np.count_nonzero(got)


def test_kernel_mass_nonnegativity_and_impermeable_source():
    d = synth.random_small((9, 8, 10), 4, r=3, n_sub=40, seed=21)
    p = oracle.Problem.from_domain(d)
    src = np.arange(d.n)
    G, m = p.kernels(src)
    assert np.max(np.abs(m - 1.0)) <= 1e-13
    assert G.min() >= 0.0
    imperm = np.flatnonzero(d.d_phase[d.label.ravel()] == 0.0)
    assert imperm.size > 0
    W = p.W
    e = np.zeros((W, W, W))
    e[3, 3, 3] = 1.0
    for s in imperm:
        assert np.array_equal(G[s], e)


def test_mass_at_config2_parameters():
    # r = 8, n = 200, D contrast 1e6: per-kernel mass to 1e-13
    d = synth.config2(seed=13, n=24)
    p = oracle.Problem.from_domain(d)
    G, m = p.kernels([0, 5000, 13824 - 1, 7000])
    assert np.max(np.abs(m - 1.0)) <= 1e-13
    assert G.min() >= 0.0


def test_support_matches_l1_ball_and_nonzero_pattern():
    r, n = 4, 3
    shape = (11, 11, 11)
    p = _uniform_problem(shape, r, n)
    s = _lin(shape, 5, 5, 5)
    sup = p.support(s)
    W = p.W
    zz, yy, xx = np.meshgrid(np.arange(W) - r, np.arange(W) - r, np.arange(W) - r, indexing="ij")
    assert np.array_equal(sup.astype(bool), (np.abs(zz) + np.abs(yy) + np.abs(xx)) <= n)
    G, _ = p.kernels([s])
    assert np.array_equal(G[0] > 0, sup.astype(bool))
    # porous mask with impermeable phase: nonzeros of G == BFS support
    d = synth.random_small((8, 9, 10), 2, r=3, n_sub=5, seed=8)
    q = oracle.Problem.from_domain(d)
    for s in (0, 77, 400, 719):
        G, _ = q.kernels([s])
        assert np.array_equal(G[0] > 0, q.support(s).astype(bool))


# ------------------------------------------------------------------ superposition, mass balance

def _tiny_covered(seed, shape, n_phase, n_sub):
    d = synth.random_small(shape, n_phase, r=max(shape) - 1, n_sub=n_sub, seed=seed)
    return d, oracle.Problem.from_domain(d)


@pytest.mark.parametrize("seed,shape", [(1, (3, 3, 3)), (2, (2, 4, 3)), (3, (4, 4, 4)), (4, (1, 3, 4))])
def test_covered_superposition_equals_matrix_power_and_global_fd(seed, shape):
    d, p = _tiny_covered(seed, shape, 3, 9)
    A = dense_operator(d.label, d.d_phase, p.dt, p.h)
    P = np.linalg.matrix_power(A, d.n_sub)
    G, _ = p.kernels(np.arange(d.n))
    # column j of P is the kernel of source j, placed in the grid
    for j in range(d.n):
        z, y, x = np.unravel_index(j, d.shape)
        r = p.r
        W = p.W
        col = G[j][r - z: r - z + shape[0], r - y: r - y + shape[1], r - x: r - x + shape[2]].ravel()
        assert np.max(np.abs(col - P[:, j])) <= 1e-13
    assert np.max(np.abs(P - P.T)) <= 1e-13                 # equal cell volumes: P symmetric
    c_new, _, _ = p.step(d.c0)
    assert np.max(np.abs(c_new.ravel() - P @ d.c0.ravel())) <= 1e-13
    assert np.max(np.abs(c_new - p.global_fd(d.c0))) <= 1e-13


def test_exact_rational_kernels_on_3cube():
    # D in {0, 1}, lambda = 3/20 exactly representable? (0.15 is not; use dt=0.125)
    label = synth.random_small((3, 3, 3), 2, r=2, n_sub=0, seed=31).label
    d_phase = np.array([1.0, 0.0])
    dt, n = 0.125, 8
    p = oracle.Problem(label, d_phase, r=2, n_sub=n, h=1.0, dt=dt)
    A = dense_operator(label, [Fraction(1), Fraction(0)], dt, 1.0, exact=True)
    P = matpow_exact(A, n)
    G, _ = p.kernels(np.arange(27))
    for j in range(27):
        z, y, x = np.unravel_index(j, (3, 3, 3))
        col = G[j][2 - z: 5 - z, 2 - y: 5 - y, 2 - x: 5 - x].ravel()
        for i in range(27):
            assert abs(Fraction(col[i]) - P[i][j]) <= Fraction(1, 10 ** 15)


def test_step_is_scatter_form_and_conserves_mass():
    # windows that do not cover the domain: the scatter (column) form keeps the
    # total mass, a gather form would not
    d = synth.random_small((10, 9, 12), 3, r=2, n_sub=25, seed=41)
    p = oracle.Problem.from_domain(d)
    c_new, used, (kmin, kmax) = p.step(d.c0)
    assert used == d.n
    assert abs(oracle.field_sum(c_new) - oracle.field_sum(d.c0)) <= 1e-12 * oracle.field_sum(d.c0)
    assert abs(kmin - 1.0) <= 1e-13 and abs(kmax - 1.0) <= 1e-13
    # one-hot: the output is the kernel, placed at its offset
    s = _lin(d.shape, 4, 0, 11)
    e = np.zeros(d.shape)
    e[4, 0, 11] = 1.0
    out, used, _ = p.step(e)
    assert used == 1
    G, _ = p.kernels([s])
    placed = np.zeros(d.shape)
    r = p.r
    for wz in range(p.W):
        for wy in range(p.W):
            for wx in range(p.W):
                Z, Y, X = 4 - r + wz, 0 - r + wy, 11 - r + wx
                if 0 <= Z < d.shape[0] and 0 <= Y < d.shape[1] and 0 <= X < d.shape[2]:
                    placed[Z, Y, X] = G[0][wz, wy, wx]
    assert np.array_equal(out, placed)


def test_step_is_linear():
    d = synth.random_small((7, 8, 9), 3, r=3, n_sub=15, seed=51)
    p = oracle.Problem.from_domain(d)
    a = d.c0
    b = synth.uniform(99, d.n).reshape(d.shape)
    ca, _, _ = p.step(a)
    cb, _, _ = p.step(b)
    cab, _, _ = p.step(2.0 * a + 3.0 * b)
    assert np.max(np.abs(cab - (2.0 * ca + 3.0 * cb))) <= 1e-13


def test_windowed_step_differs_from_global_fd_when_not_covered():
    # diagnostic, not a gate: reflecting windows change the result once the
    # spread reaches the window walls
    d = synth.config0()
    p = oracle.Problem.from_domain(d)
    c_new, _, _ = p.step(d.c0)
    gap = np.max(np.abs(c_new - p.global_fd(d.c0)))
    assert gap > 1e-6
    assert abs(oracle.field_sum(c_new) - oracle.field_sum(d.c0)) <= 1e-12 * oracle.field_sum(d.c0)


def test_compensated_sum():
    v = np.array([1.0, 1e100, 1.0, -1e100] * 1000)
    assert oracle.field_sum(v) == 2000.0
    assert oracle.field_sum(np.full(10 ** 6, 0.1)) == pytest.approx(1e5, rel=1e-15)
