"""Pins of the FP64 surrogate oracle (conv3d / SiLU / masked softmax / loss and
their gradients) against impulse responses, exact identities and central
finite differences.  CPU only."""
import numpy as np
import pytest

import oracle
import synth
from oracle import surrogate as su


def _rng(seed):
    return np.random.default_rng(seed)


def test_conv_impulse_response_pins_tap_orientation():
    rng = _rng(1)
    w = rng.standard_normal((2, 1, 3, 3, 3))
    b = np.array([0.5, -1.0])
    x = np.zeros((1, 5, 5, 5))
    x[0, 2, 2, 2] = 1.0
    y = su.conv3(x, w, b)
    # y[co, z, y, x] = b + w[co, 0, dz, dy, dx] with z + dz - 1 = 2
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                assert y[:, 3 - dz, 3 - dy, 3 - dx] == pytest.approx(b + w[:, 0, dz, dy, dx], abs=1e-15)
    # far from the impulse only the bias
    assert np.allclose(y[:, 0, :, :], b[:, None, None])
    # zero padding: an impulse in a corner reaches only 8 outputs
    x2 = np.zeros((1, 5, 5, 5))
    x2[0, 0, 0, 0] = 1.0
    y2 = su.conv3(x2, w, np.zeros(2))
    assert np.count_nonzero(np.abs(y2) > 0) == 2 * 8


def test_conv_is_linear_and_sums_channels():
    rng = _rng(2)
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    x1, x2 = rng.standard_normal((2, 2, 4, 4, 4))
    a = su.conv3(2 * x1 + 3 * x2, w, b)
    c = 2 * su.conv3(x1, w, b) + 3 * su.conv3(x2, w, b) - 4 * b[:, None, None, None]
    assert np.max(np.abs(a - c)) <= 1e-12
    # two input channels = sum of single-channel convolutions
    y = su.conv3(x1, w, np.zeros(3))
    y0 = su.conv3(x1[:1], w[:, :1], np.zeros(3))
    y1 = su.conv3(x1[1:], w[:, 1:], np.zeros(3))
    assert np.max(np.abs(y - y0 - y1)) <= 1e-12


def test_silu_values():
    assert su.silu(np.array([0.0]))[0] == 0.0
    assert su.silu(np.array([1.0]))[0] == pytest.approx(1.0 / (1.0 + np.exp(-1.0)), rel=1e-15)
    x = np.linspace(-5, 5, 11)
    h = 1e-6
    assert np.allclose(su.silu_grad(x), (su.silu(x + h) - su.silu(x - h)) / (2 * h), atol=1e-8)


def test_masked_softmax_unit_mass_and_support():
    rng = _rng(3)
    z = rng.standard_normal((5, 5, 5)) * 3
    s = rng.random((5, 5, 5)) < 0.6
    g = su.masked_softmax(z, s)
    assert g.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.all(g[~s] == 0) and np.all(g[s] > 0)
    # shift invariance
    assert np.allclose(su.masked_softmax(z + 7.0, s), g, atol=1e-15)


def _small_problem(seed, W=5):
    rng = _rng(seed)
    params = su.init_params(seed)
    feat = rng.standard_normal((3, W, W, W)) * 0.5
    support = rng.random((W, W, W)) < 0.8
    q = su.masked_softmax(rng.standard_normal((W, W, W)), support)
    return params, feat, support, q


def _loss(params, feat, support, q):
    logits, _ = su.forward(params, feat)
    g = su.masked_softmax(logits, support)
    return su.loss_and_dlogits(g, q, support)[0]


def test_dlogits_matches_finite_differences():
    rng = _rng(4)
    W = 4
    z = rng.standard_normal((W, W, W))
    s = rng.random((W, W, W)) < 0.7
    q = su.masked_softmax(rng.standard_normal((W, W, W)), s)
    g = su.masked_softmax(z, s)
    _, dz = su.loss_and_dlogits(g, q, s)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 3), (3, 3, 3), (2, 1, 0)]:
        zp, zm = z.copy(), z.copy()
        zp[idx] += h
        zm[idx] -= h
        fp = su.loss_and_dlogits(su.masked_softmax(zp, s), q, s)[0]
        fm = su.loss_and_dlogits(su.masked_softmax(zm, s), q, s)[0]
        assert dz[idx] == pytest.approx((fp - fm) / (2 * h), abs=1e-7)
    assert np.all(dz[~s] == 0)
    assert abs(dz.sum()) <= 1e-12          # softmax shift invariance


@pytest.mark.parametrize("layer", [0, 2, 4])
def test_parameter_gradients_match_finite_differences(layer):
    params, feat, support, q = _small_problem(5 + layer)
    logits, cache = su.forward(params, feat)
    g = su.masked_softmax(logits, support)
    _, dz = su.loss_and_dlogits(g, q, support)
    grads = su.backward(params, cache, dz)
    rng = _rng(10 + layer)
    w, b = params[layer]
    h = 1e-4          # smooth loss: O(h^2) truncation ~1e-9 relative, rounding noise far below
    for _ in range(6):
        idx = tuple(int(rng.integers(0, n)) for n in w.shape)
        wp = [(ww.copy(), bb.copy()) for ww, bb in params]
        wm = [(ww.copy(), bb.copy()) for ww, bb in params]
        wp[layer][0][idx] += h
        wm[layer][0][idx] -= h
        num = (_loss(wp, feat, support, q) - _loss(wm, feat, support, q)) / (2 * h)
        assert grads[layer][0][idx] == pytest.approx(num, rel=1e-5, abs=1e-10)
    j = int(rng.integers(0, b.shape[0]))
    bp = [(ww.copy(), bb.copy()) for ww, bb in params]
    bm = [(ww.copy(), bb.copy()) for ww, bb in params]
    bp[layer][1][j] += h
    bm[layer][1][j] -= h
    num = (_loss(bp, feat, support, q) - _loss(bm, feat, support, q)) / (2 * h)
    assert grads[layer][1][j] == pytest.approx(num, rel=1e-5, abs=1e-10)


def test_flatten_round_trip_and_count():
    params = su.init_params(3)
    theta = su.flatten(params)
    assert theta.size == su.num_params() == 3 * 16 * 27 + 16 + 3 * (16 * 16 * 27 + 16) + 16 * 27 + 1
    back = su.unflatten(theta)
    for (w, b), (w2, b2) in zip(params, back):
        assert np.array_equal(w, w2) and np.array_equal(b, b2)


def test_features_and_prior():
    r, n = 2, 20
    logu = su.prior_log_uniform(r, n)
    assert np.exp(logu).sum() == pytest.approx(1.0, abs=1e-13)
    d = synth.random_small((6, 7, 8), 3, r=r, n_sub=n, seed=9)
    f = su.window_features(d.label, d.d_phase, 0, r, logu)
    # source 0 sits in a corner: cells with negative offsets are outside
    assert np.all(f[0, :r] == 0) and np.all(f[1, :r] == -1.0)
    D = d.d_phase[d.label[0, 0, 0]]
    assert f[0, r, r, r] == (1.0 if D > 0 else 0.0)
    assert f[1, r, r, r] == pytest.approx((max(np.log10(D), -12) if D > 0 else -12) / 6 + 1)
    assert np.allclose(f[2] * su.PRIOR_SCALE, logu)
