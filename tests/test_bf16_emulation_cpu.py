"""CPU pins of the BF16-rounding emulation used to check the GPU network.

The rounding itself is pinned to exact BF16 values (8 significant bits,
round to nearest, ties to even); the emulated network is pinned to the FP64
oracle: with the rounding replaced by the identity it is the oracle up to
FP32 rounding of pre-activations and logits, and with the rounding it differs
from the oracle by the BF16 unit roundoff's order (neither 0 nor O(1))."""
import numpy as np
import pytest

import synth
from oracle import surrogate as su
import bf16_emulation as emu


def test_bf16_rounding_values():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -8 + 2.0 ** -20, -3.0 - 2.0 ** -7,
                  2.0 ** -130, 0.0, 65504.0, 1.0 / 3.0])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -3.0, 2.0 ** -130, 0.0, 65536.0,
                     0.333984375])
    assert np.array_equal(emu.bf16(x), want)
    # every result has at most 8 significant bits and is within half an ulp
    rng = np.random.default_rng(0)
    v = rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000)
    r = emu.bf16(v)
    m, e = np.frexp(r)
    assert np.all(m * 256 == np.round(m * 256))
    x32 = np.float32(v).astype(np.float64)
    assert np.all(np.abs(r - x32) <= 2.0 ** -8 * np.abs(x32))


@pytest.fixture(scope="module")
def case():
    d = synth.random_small((18, 18, 18), 3, r=8, n_sub=30, seed=4)
    prior = su.prior_log_uniform(8, 30)
    p = su.init_params(3)
    p[4] = (p[4][0] * 10.0, p[4][1])
    params = [(w.astype(np.float32).astype(np.float64), (b + 0.01).astype(np.float32).astype(np.float64))
              for w, b in p]
    return d, prior, params, [0, 2915, 5831]


def test_emulation_without_rounding_is_the_oracle(case, monkeypatch):
    d, prior, params, srcs = case
    monkeypatch.setattr(emu, "bf16", lambda x: np.asarray(x, dtype=np.float64))
    for s in srcs:
        f = su.window_features(d.label, d.d_phase, s, 8, prior)
        lo, (acts, _) = su.forward(params, f)
        le, _ = emu.forward(params, emu.features(d.label, d.d_phase, s, 8, prior), prior)
        assert np.max(np.abs(le - lo)) <= 1e-5 * np.abs(lo).max()


def test_emulation_rounding_moves_the_output_by_the_unit_roundoff(case):
    d, prior, params, srcs = case
    for s in srcs:
        f = su.window_features(d.label, d.d_phase, s, 8, prior)
        lo, cache = su.forward(params, f)
        le, ecache = emu.forward(params, emu.features(d.label, d.d_phase, s, 8, prior), prior)
        err = np.linalg.norm((le - prior) - (lo - prior)) / np.linalg.norm(lo - prior)
        assert 2.0 ** -14 < err < 2.0 ** -5, err
        # the hidden activations are BF16 values
        for h in ecache[0][1:5]:
            assert np.array_equal(h, emu.bf16(h))
        # gradients: same order of difference from the oracle's
        dl = np.random.default_rng(s).standard_normal(lo.shape) * 1e-3
        go = su.flatten(su.backward(params, cache, dl))
        ge = su.flatten(emu.backward(params, ecache, dl, 1.0))
        gerr = np.linalg.norm(ge - go) / np.linalg.norm(go)
        assert 2.0 ** -14 < gerr < 2.0 ** -5, gerr
