"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: integer/index work and single-contribution outputs bit-exact; FP64
fields L_inf <= 1e-12 and kernel mass to 1e-13; FP32 fields L_inf <= 1e-5;
reduced-precision modes relative L1 <= 1e-3 against the FP64 oracle with mass
conserved to 1e-6.  Every input is seeded (synth).
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import oracle_point, place, rel_l1, to_dev, to_host, window_sources

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2408_11376_amd as fd  # noqa: E402


def _dev_domain(d):
    return fd.Domain(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)


# ------------------------------------------------------------------ coefficients

@pytest.mark.parametrize("seed,shape,nph", [(1, (9, 7, 11), 4), (2, (1, 1, 5), 2), (3, (16, 16, 16), 3)])
def test_coefficients_bitexact(seed, shape, nph):
    d = synth.random_small(shape, nph, r=2, n_sub=5, seed=seed)
    lam, dt = fd.fdirw_coefficients(_dev_domain(d))
    lx, ly, lz, dto = oracle.coefficients(d.label, d.d_phase, d.h, d.dt)
    assert dt == dto
    got = to_host(lam)
    assert np.array_equal(got[0], lx) and np.array_equal(got[1], ly) and np.array_equal(got[2], lz)


def test_coefficients_config0_and_given_dt():
    d = synth.config0()
    lam, dt = fd.fdirw_coefficients(_dev_domain(d))
    lx, ly, lz, dto = oracle.coefficients(d.label, d.d_phase, d.h, 0.0)
    assert dt == dto == (0.9 * 1.0 * 1.0) / (6.0 * 1.0)
    assert np.array_equal(to_host(lam), np.stack([lx, ly, lz]))
    dom = fd.Domain(d.label, d.d_phase, 3, 40, 0.5, 0.02)
    lam, dt = fd.fdirw_coefficients(dom)
    lx, ly, lz, _ = oracle.coefficients(d.label, d.d_phase, 0.5, 0.02)
    assert dt == 0.02 and np.array_equal(to_host(lam), np.stack([lx, ly, lz]))


# ------------------------------------------------------------------ window kernels

@pytest.mark.parametrize("r,n_sub,shape,seed", [(0, 7, (4, 5, 6), 1), (1, 9, (5, 5, 5), 2), (2, 20, (7, 9, 8), 3),
                                                 (3, 40, (12, 10, 14), 4), (4, 33, (6, 13, 11), 5),
                                                 (8, 60, (19, 18, 20), 6), (5, 0, (6, 6, 6), 7)])
def test_kernels_fp64_match_oracle(r, n_sub, shape, seed):
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed)
    p = oracle.Problem.from_domain(d)
    rng = np.random.default_rng(seed)
    src = np.unique(np.concatenate([[0, d.n - 1], rng.integers(0, d.n, 40)])).astype(np.int64)
    G, m = fd.fdirw_kernels(_dev_domain(d), to_dev(src), prec=fd.FP64)
    Go, mo = p.kernels(src)
    assert np.max(np.abs(to_host(G) - Go)) <= 1e-13
    assert np.max(np.abs(to_host(m) - mo)) <= 1e-13
    # structural support (integer): nonzero pattern equals the oracle's
    assert np.array_equal(to_host(G) != 0, Go != 0)


def test_kernel_support_bitexact_vs_bfs():
    d = synth.random_small((10, 11, 12), 2, r=4, n_sub=6, seed=12)   # D in {1, 0}
    p = oracle.Problem.from_domain(d)
    src = np.array([0, 5, 100, 777, 1319], dtype=np.int64)
    G, _ = fd.fdirw_kernels(_dev_domain(d), to_dev(src), prec=fd.FP64)
    G = to_host(G)
    for k, s in enumerate(src):
        assert np.array_equal(G[k] != 0, p.support(int(s)).astype(bool))


@pytest.mark.parametrize("prec", [fd.FP32])
def test_kernels_fp32_match_oracle(prec):
    d = synth.config2(seed=13, n=24)
    p = oracle.Problem.from_domain(d)
    src = np.array([0, 17, 4000, 6912, 13823], dtype=np.int64)
    G, m = fd.fdirw_kernels(_dev_domain(d), to_dev(src), prec=prec)
    Go, mo = p.kernels(src)
    assert np.max(np.abs(to_host(G) - Go)) <= 1e-5
    assert np.max(np.abs(to_host(m) - 1.0)) <= 1e-5


# ------------------------------------------------------------------ superposition, mass balance

def test_step_fp64_config0_full():
    d = synth.config0()
    p = oracle.Problem.from_domain(d)
    ref, used, (kmin, kmax) = p.step(d.c0)
    out, st = fd.fdirw_step(_dev_domain(d), to_dev(d.c0), prec=fd.FP64, stats=True)
    got = to_host(out)
    assert np.max(np.abs(got - ref)) <= 1e-12
    assert st["n_sources"] == used
    assert abs(st["kmass_min"] - 1.0) <= 1e-13 and abs(st["kmass_max"] - 1.0) <= 1e-13
    assert abs(st["mass_in"] - oracle.field_sum(d.c0)) <= 1e-12 * st["mass_in"]
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-12 * st["mass_in"]


@pytest.mark.parametrize("prec,tol", [(fd.FP64, 1e-12), (fd.FP32, 1e-5)])
@pytest.mark.parametrize("shape,r,n_sub,seed", [((5, 7, 11), 2, 9, 21), ((1, 1, 1), 3, 5, 22), ((3, 4, 2), 8, 12, 23),
                                                 ((17, 3, 9), 4, 25, 24), ((6, 6, 6), 0, 10, 25),
                                                 ((8, 9, 10), 3, 0, 26)])
def test_step_small_and_ragged(prec, tol, shape, r, n_sub, seed):
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed)
    p = oracle.Problem.from_domain(d)
    ref, _, _ = p.step(d.c0)
    out = fd.fdirw_step(_dev_domain(d), to_dev(d.c0), prec=prec)
    assert np.max(np.abs(to_host(out) - ref)) <= tol


@pytest.mark.parametrize("tune", [1, 2, 5, 1000])
def test_step_segmenting_does_not_change_result(tune):
    d = synth.random_small((13, 6, 7), 3, r=3, n_sub=15, seed=31)
    p = oracle.Problem.from_domain(d)
    ref, _, _ = p.step(d.c0)
    out = fd.fdirw_step(_dev_domain(d), to_dev(d.c0), prec=fd.FP64, tune=tune)
    assert np.max(np.abs(to_host(out) - ref)) <= 1e-13


@pytest.mark.parametrize("prec", [fd.FP64, fd.FP32, fd.FP16X32, fd.BF16_BANK])
def test_one_hot_step_is_placed_kernel_bitwise(prec):
    d = synth.random_small((9, 10, 11), 3, r=3, n_sub=30, seed=41)
    dom = _dev_domain(d)
    for (z, y, x) in [(0, 0, 0), (4, 5, 6), (8, 9, 10), (2, 9, 1)]:
        s = (z * 10 + y) * 11 + x
        e = np.zeros(d.shape)
        e[z, y, x] = 1.0
        out = to_host(fd.fdirw_step(dom, to_dev(e), prec=prec))
        G, m = fd.fdirw_kernels(dom, to_dev(np.array([s], dtype=np.int64)), prec=prec)
        g = to_host(G)[0].astype(np.float64)
        if prec != fd.FP64:
            g = (1.0 / float(to_host(m)[0])) * g           # renormalising modes
        assert np.array_equal(out, place(d.shape, s, g))


def test_step_fp32_config1_subblock():
    d = synth.config1()
    m = synth.sub_block_sources(d.shape, 8)
    c0 = np.where(m, d.c0, 0.0)
    p = oracle.Problem.from_domain(d)
    ref, used, _ = p.step(c0)
    out, st = fd.fdirw_step(_dev_domain(d), to_dev(c0), prec=fd.FP32, stats=True)
    assert st["n_sources"] == used == 512
    assert np.max(np.abs(to_host(out) - ref)) <= 1e-5
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-9 * st["mass_in"]


def test_field_sum_matches_oracle():
    rng = np.random.default_rng(5)
    for n in (1, 255, 4097, 1000003):
        v = rng.standard_normal(n) * 10.0 ** rng.integers(-8, 8, n)
        got = fd.fdirw_field_sum(to_dev(v))
        ref = oracle.field_sum(v)
        assert abs(got - ref) <= 1e-15 * np.abs(v).sum()


def test_multi_domain_call_equals_single_calls():
    ds = [synth.random_small((7, 8, 9), 3, r=2, n_sub=10, seed=50 + i) for i in range(3)]
    doms = [_dev_domain(d) for d in ds]
    outs = fd.fdirw_step(doms, [to_dev(d.c0) for d in ds], prec=fd.FP64)
    for d, o in zip(ds, outs):
        ref, _, _ = oracle.Problem.from_domain(d).step(d.c0)
        assert np.max(np.abs(to_host(o) - ref)) <= 1e-13


# ------------------------------------------------------------------ kernel bank

@pytest.mark.parametrize("prec", [fd.FP64, fd.FP32, fd.FP16X32, fd.BF16_BANK])
def test_run_bank_equals_fused(prec):
    d = synth.random_small((12, 11, 10), 3, r=3, n_sub=20, seed=61)
    dom = _dev_domain(d)
    a = to_dev(d.c0)
    b = to_dev(d.c0)
    _, sa = fd.fdirw_run(dom, a, 3, prec=prec, stats=True)
    _, sb = fd.fdirw_run(dom, b, 3, prec=prec, stats=True, bank_budget_bytes=1 << 34)
    assert sa["bank_used"] == 0 and sb["bank_used"] == 1
    A, B = to_host(a), to_host(b)
    assert np.max(np.abs(A - B)) <= 1e-12 * np.abs(A).max()
    # three steps of the oracle
    p = oracle.Problem.from_domain(d)
    c = d.c0
    for _ in range(3):
        c, _, _ = p.step(c)
    tol = {fd.FP64: 1e-12, fd.FP32: 1e-5}.get(prec, None)
    if tol is not None:
        assert np.max(np.abs(A - c)) <= tol
    else:
        assert rel_l1(A, c) <= 1e-3
    assert abs(sb["mass_out"] - sb["mass_in"]) <= 1e-9 * sb["mass_in"]


@pytest.mark.parametrize("prec", [fd.FP32, fd.FP16_BANK, fd.FP64])
def test_run_bank_equals_fused_several_tiles(prec):
    # r = 8 on a grid that spans two x tiles of the apply (the second ragged),
    # a ragged last z tile and z groups, against the fused step (whose kernels
    # are the same values, superposed in another order)
    d = synth.random_small((37, 21, 70), 3, r=8, n_sub=12, seed=63)
    dom = _dev_domain(d)
    a = to_dev(d.c0)
    b = to_dev(d.c0)
    fd.fdirw_run(dom, a, 2, prec=prec)
    _, sb = fd.fdirw_run(dom, b, 2, prec=prec, stats=True, bank_budget_bytes=1 << 34)
    assert sb["bank_used"] == 1
    A, B = to_host(a), to_host(b)
    assert np.max(np.abs(A - B)) <= 1e-12 * np.abs(A).max()
    assert abs(sb["mass_out"] - sb["mass_in"]) <= 1e-12 * sb["mass_in"]


@pytest.mark.parametrize("prec", [fd.FP32, fd.FP16_BANK, fd.FP64])
@pytest.mark.parametrize("shape,r,n_sub", [((1, 1, 1), 0, 3), ((1, 1, 1), 2, 3), ((9, 2, 1), 1, 5),
                                           ((3, 1, 70), 2, 4), ((17, 5, 65), 4, 0)])
def test_run_bank_degenerate_shapes(prec, shape, r, n_sub):
    # single cells, windows larger than the domain, z shorter than one 16-byte
    # group, lines of one cell, n_sub = 0 (identity kernels): bank == fused
    d = synth.random_small(shape, 2, r=r, n_sub=n_sub, seed=64)
    dom = _dev_domain(d)
    a = to_dev(d.c0)
    b = to_dev(d.c0)
    fd.fdirw_run(dom, a, 2, prec=prec)
    _, sb = fd.fdirw_run(dom, b, 2, prec=prec, stats=True, bank_budget_bytes=1 << 34)
    assert sb["bank_used"] == 1
    A, B = to_host(a), to_host(b)
    assert np.max(np.abs(A - B)) <= 1e-12 * max(np.abs(A).max(), 1e-300)
    if n_sub == 0:
        assert np.array_equal(B, d.c0)


@pytest.mark.parametrize("shape,r,n_sub", [((12, 11, 10), 3, 20), ((48, 40, 40), 2, 4)])
def test_bank_kernel_mass_range_equals_fused(shape, r, n_sub):
    # the bank's statistics reduce one mass per source (the larger domain
    # takes the multi-block reduction); the fused step reduces per-workgroup
    # ranges of the same kernels
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=62)
    dom = _dev_domain(d)
    _, sa = fd.fdirw_run(dom, to_dev(d.c0), 1, prec=fd.FP32, stats=True)
    _, sb = fd.fdirw_run(dom, to_dev(d.c0), 1, prec=fd.FP32, stats=True, bank_budget_bytes=1 << 34)
    assert sb["bank_used"] == 1
    assert sb["kmass_min"] == pytest.approx(sa["kmass_min"], rel=1e-12)
    assert sb["kmass_max"] == pytest.approx(sa["kmass_max"], rel=1e-12)
    assert sb["kmass_min"] <= sb["kmass_max"]


def test_run_zero_and_odd_steps_keep_result_in_place():
    d = synth.random_small((6, 7, 8), 2, r=2, n_sub=4, seed=71)
    dom = _dev_domain(d)
    c = to_dev(d.c0)
    fd.fdirw_run(dom, c, 0, prec=fd.FP64)
    assert np.array_equal(to_host(c), d.c0)
    fd.fdirw_run(dom, c, 1, prec=fd.FP64)
    ref, _, _ = oracle.Problem.from_domain(d).step(d.c0)
    assert np.max(np.abs(to_host(c) - ref)) <= 1e-13


# ------------------------------------------------------------------ precision modes

@pytest.mark.parametrize("prec,kern_tol", [(fd.FP16X32, 1e-3), (fd.BF16X32, 3e-3), (fd.FP16_BANK, 1e-3),
                                           (fd.BF16_BANK, 4e-3), (fd.FP16_STATE, 2e-2), (fd.BF16_STATE, 1e-1)])
def test_reduced_precision_against_fp64_oracle(prec, kern_tol):
    d = synth.config2(seed=13, n=32)
    p = oracle.Problem.from_domain(d)
    m = synth.sub_block_sources(d.shape, 6)
    c0 = np.where(m, d.c0, 0.0)
    ref, _, _ = p.step(c0)
    out, st = fd.fdirw_step(_dev_domain(d), to_dev(c0), prec=prec, stats=True)
    got = to_host(out)
    # renormalised kernels: mass conserved to 1e-6 in every reduced mode
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-6 * st["mass_in"]
    err = rel_l1(got, ref)
    if prec in (fd.FP16X32, fd.FP16_BANK, fd.BF16X32, fd.BF16_BANK):
        assert err <= 1e-3, err
    # per-kernel L1 of a few kernels against the oracle
    src = np.array([d.n // 2 + 3, 100, 5000], dtype=np.int64)
    G, _ = fd.fdirw_kernels(_dev_domain(d), to_dev(src), prec=prec)
    Go, mo = p.kernels(src)
    Gh = to_host(G).astype(np.float64)
    for k in range(len(src)):
        ref_k = Go[k] / mo[k]
        got_k = Gh[k] / Gh[k].sum()
        assert np.abs(got_k - ref_k).sum() <= kern_tol


# ------------------------------------------------------------------ errors

def test_errors_are_reported_not_raised_in_library():
    d = synth.random_small((4, 4, 4), 2, r=1, n_sub=3, seed=81)
    bad = d.label.copy()
    bad[1, 2, 3] = 7
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_step(fd.Domain(bad, d.d_phase, 1, 3), to_dev(d.c0))
    assert e.value.status == fd.E_ARG
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_step(fd.Domain(d.label, d.d_phase, 1, 3, 1.0, 0.5), to_dev(d.c0))
    assert e.value.status == fd.E_UNSTABLE
    c = to_dev(d.c0)
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_step(_dev_domain(d), c, c)
    assert e.value.status == fd.E_ARG
    nan = d.c0.copy()
    nan[0, 0, 0] = np.nan
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_step(_dev_domain(d), to_dev(nan), stats=True)
    assert e.value.status == fd.E_NONFINITE
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_kernels(_dev_domain(d), to_dev(np.array([64], dtype=np.int64)))
    assert e.value.status == fd.E_ARG
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_step(fd.Domain(d.label, d.d_phase, 9, 3), to_dev(d.c0))
    assert e.value.status == fd.E_ARG
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_step(fd.Domain(d.label, np.array([1.0, -1.0]), 1, 3), to_dev(d.c0))
    assert e.value.status == fd.E_ARG
    assert "d_phase" in fd.fdirw_last_error()
    # the library still works after errors
    out = fd.fdirw_step(_dev_domain(d), to_dev(d.c0), prec=fd.FP64)
    ref, _, _ = oracle.Problem.from_domain(d).step(d.c0)
    assert np.max(np.abs(to_host(out) - ref)) <= 1e-13


# ------------------------------------------------------------------ full size

@pytest.mark.slow
def test_config2_full_size_sampled_points():
    """192^3, r = 8, 200 sub-steps, every cell a source: the launch the
    benchmark times.  Sampled outputs against the oracle (each needs the 4913
    kernels that reach it) and global properties at full size."""
    d = synth.config2()
    dom = _dev_domain(d)
    c0 = to_dev(d.c0)
    p = oracle.Problem.from_domain(d)
    rng = np.random.default_rng(7)
    pts = [(0, 0, 0), (191, 100, 7)] + [tuple(int(v) for v in rng.integers(0, 192, 3)) for _ in range(1)]
    ref = [oracle_point(p, d.c0, q) for q in pts]
    out32, st = fd.fdirw_step(dom, c0, prec=fd.FP32, stats=True)
    o32 = to_host(out32)
    assert st["n_sources"] == d.n
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-6 * st["mass_in"]
    for q, v in zip(pts, ref):
        assert abs(o32[q] - v) <= 1e-5
    for prec in (fd.FP16X32, fd.BF16X32):
        out, st = fd.fdirw_step(dom, c0, prec=prec, stats=True)
        o = to_host(out)
        assert rel_l1(o, o32) <= 1e-3
        assert abs(st["mass_out"] - st["mass_in"]) <= 1e-6 * st["mass_in"]
        for q, v in zip(pts, ref):
            assert abs(o[q] - v) <= 1e-3 * abs(v)


def test_evolving_geometry_regenerates_every_step():
    # the fused step regenerates every kernel from the labels it is given, so
    # a geometry that changes between big steps (e.g. a dissolving or growing
    # solid) needs nothing else: each step equals the oracle on its own labels
    a = synth.random_small((9, 8, 10), 3, r=3, n_sub=12, seed=81)
    b = synth.random_small((9, 8, 10), 3, r=3, n_sub=12, seed=82)
    c = to_dev(a.c0)
    ref = a.c0
    for d in (a, b, a):
        c = fd.fdirw_step(_dev_domain(d), c, prec=fd.FP64)
        ref, _, _ = oracle.Problem.from_domain(d).step(ref)
        assert np.max(np.abs(to_host(c) - ref)) <= 1e-12 * np.abs(ref).max()
