"""Pins of the 16-bit-copy kernels (oracle/lowprec.py) on the CPU.

The rounding is checked against independent conversions (numpy's float16,
torch's bfloat16) and values worked out by hand; the scheme against the FP64
oracle (bitwise when the copies are exact), against exact dyadic arithmetic,
against the conservation its antisymmetric fluxes give, and against the
error bound that follows from the update being a convex combination."""
import numpy as np
import pytest

import oracle
import synth
from oracle import lowprec


def test_fp16_rounding_matches_numpy_float16():
    rng = np.random.default_rng(5)
    # magnitudes from the subnormal range (< 2^-14) to 1, both signs, and exact ties
    x = rng.uniform(-1.0, 1.0, 20000) * 10.0 ** rng.uniform(-9.0, 0.0, 20000)
    ties = (np.arange(1, 2049) + 0.5) * 2.0 ** -11            # halfway between FP16 numbers of [1/2, 1)
    sub_ties = (np.arange(0, 64) + 0.5) * 2.0 ** -24           # halfway between FP16 subnormals
    for v in (x, ties, sub_ties):
        assert np.array_equal(lowprec.round_to_format(v, lowprec.FP16), v.astype(np.float16).astype(np.float64))


def test_bf16_rounding_against_hand_values_and_torch():
    one = 1.0
    cases = {one + 2.0 ** -8: 1.0,                             # tie, 1 is even
             one + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,             # tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
             one + 2.0 ** -8 + 2.0 ** -30: 1.0 + 2.0 ** -7,    # just above the tie
             2.0 ** -127: 2.0 ** -127,                         # a subnormal that is representable
             2.0 ** -134: 0.0,                                 # half the smallest subnormal: tie to even (0)
             3 * 2.0 ** -134: 2.0 ** -132}                     # 1.5 steps: tie to 2 steps
    for v, want in cases.items():
        assert lowprec.round_to_format(np.array([v]), lowprec.BF16)[0] == want, v
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    x = (rng.uniform(-1.0, 1.0, 20000) * 10.0 ** rng.uniform(-30.0, 0.0, 20000)).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lowprec.round_to_format(x.astype(np.float64), lowprec.BF16), want)


@pytest.mark.parametrize("shape,r,n_sub,seed", [((7, 8, 9), 3, 12, 3), ((5, 4, 6), 4, 20, 4), ((9, 9, 9), 2, 7, 5)])
def test_exact_copies_reproduce_the_fp64_oracle_bitwise(shape, r, n_sub, seed):
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed)
    p = oracle.Problem.from_domain(d)
    src = np.arange(0, d.label.size, 7)
    G, m = p.kernels(src)
    Gl, ml = lowprec.kernels(p, src, lowprec.FP64)
    assert np.array_equal(G, Gl)
    assert np.max(np.abs(m - ml)) <= 1e-15


@pytest.mark.parametrize("fmt,n_sub", [(lowprec.FP16, 3), (lowprec.BF16, 2)])
def test_dyadic_steps_are_exact(fmt, n_sub):
    # lambda = 1/8 everywhere: after k sub-steps every value is an integer
    # over 8^k small enough for the format, so the copies round nothing
    label = np.zeros((7, 7, 7), dtype=np.uint8)
    p = oracle.Problem(label, np.array([1.0]), 3, n_sub, 1.0, 0.125)
    src = [171, 0, 48]
    G, _ = p.kernels(src)
    Gl, ml = lowprec.kernels(p, src, fmt)
    assert np.array_equal(G, Gl)
    assert np.all(ml == 1.0)
    # the same with lambda = 0.15 rounds (the copies are really taken)
    p2 = oracle.Problem(label, np.array([1.0]), 3, n_sub + 3, 1.0, 0.15)
    assert not np.array_equal(p2.kernels(src)[0], lowprec.kernels(p2, src, fmt)[0])


@pytest.mark.parametrize("fmt", [lowprec.FP16, lowprec.BF16])
def test_copies_conserve_mass_and_stay_inside_the_bound(fmt):
    # three random phases (diffusivities 1, 10^U[-4, 0] and 0): each face
    # exchanges equal and opposite amounts, so the mass stays 1
    d = synth.random_small((11, 10, 12), 3, r=4, n_sub=40, seed=9)
    p = oracle.Problem.from_domain(d)
    src = np.arange(3, d.label.size, 37)
    G, _ = p.kernels(src)
    Gl, ml = lowprec.kernels(p, src, fmt)
    assert np.max(np.abs(ml - 1.0)) <= 1e-13
    lam_max = max(p.lx.max(), p.ly.max(), p.lz.max())
    bound = lowprec.error_bound(p.n_sub, lam_max, fmt)
    err = np.max(np.abs(Gl - G))
    assert 0.0 < err <= bound
    assert Gl.min() >= 0.0 and Gl.max() <= 1.0


@pytest.mark.parametrize("fmt", [lowprec.FP16, lowprec.BF16])
def test_rounded_state_stays_in_the_format_and_inside_its_bound(fmt):
    d = synth.random_small((9, 10, 8), 3, r=3, n_sub=25, seed=12)
    p = oracle.Problem.from_domain(d)
    src = np.arange(2, d.label.size, 41)
    G, _ = p.kernels(src)
    Gs, _ = lowprec.kernels(p, src, fmt, state=True)
    # every value is a number of the format
    assert np.array_equal(lowprec.round_to_format(Gs, fmt), Gs)
    lam_max = max(p.lx.max(), p.ly.max(), p.lz.max())
    assert np.max(np.abs(Gs - G)) <= lowprec.error_bound(p.n_sub, lam_max, fmt, state=True)
    # with lambda = 1/8 the first sub-steps are exact here too
    label = np.zeros((7, 7, 7), dtype=np.uint8)
    q = oracle.Problem(label, np.array([1.0]), 3, 2, 1.0, 0.125)
    assert np.array_equal(q.kernels([171])[0], lowprec.kernels(q, [171], fmt, state=True)[0])
