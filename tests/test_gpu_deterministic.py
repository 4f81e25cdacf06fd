"""GPU: the deterministic step (no floating-point atomics).

The contract (Eq. 8 marched in time): with deterministic = 1 the result of
fdirw_step / fdirw_run is a function of the inputs, so a repeated call, a
batched call (n_dom > 1) and single calls, and a run resumed from its
intermediate field all agree bitwise; every result still matches the FP64
oracle to the usual bars (L_inf 1e-12 in FP64, 1e-5 in FP32).  FP32 steps at
r = 4..8 store their partials from the flat-layout kernel (several lines per
workgroup at r = 4..6), the other cases from the segment-layout kernel."""
import numpy as np
import pytest

import oracle
import synth
from helpers import place, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2408_11376_amd as fd  # noqa: E402


def _dev(d):
    return fd.Domain(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)


@pytest.mark.parametrize("prec,tol", [(fd.FP64, 1e-12), (fd.FP32, 1e-5)])
@pytest.mark.parametrize("shape,r,n_sub,seed", [((5, 7, 11), 2, 9, 21), ((1, 1, 1), 3, 5, 22), ((3, 4, 2), 8, 12, 23),
                                                 ((17, 3, 9), 4, 25, 24), ((6, 6, 6), 0, 10, 25),
                                                 ((8, 9, 10), 3, 0, 26), ((19, 18, 20), 8, 40, 27),
                                                 ((10, 9, 11), 6, 23, 28), ((12, 7, 13), 5, 17, 29),
                                                 ((4, 1, 2), 4, 7, 30)])
def test_deterministic_step_matches_oracle_and_repeats_bitwise(prec, tol, shape, r, n_sub, seed):
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed)
    ref, used, _ = oracle.Problem.from_domain(d).step(d.c0)
    dom = _dev(d)
    a, st = fd.fdirw_step(dom, to_dev(d.c0), prec=prec, stats=True, deterministic=True)
    b = fd.fdirw_step(dom, to_dev(d.c0), prec=prec, deterministic=True)
    A = to_host(a)
    assert np.max(np.abs(A - ref)) <= tol
    assert np.array_equal(A, to_host(b))
    assert st["n_sources"] == used
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-9 * max(st["mass_in"], 1e-300)
    # the atomic form differs from it by summation order only
    c = to_host(fd.fdirw_step(dom, to_dev(d.c0), prec=prec))
    assert np.max(np.abs(A - c)) <= 1e-13 * max(np.abs(A).max(), 1e-300)


@pytest.mark.parametrize("slab", [1, 2, 3, 7, 1000])
def test_deterministic_slabs_match_oracle(slab):
    # slabs of source planes thinner than the window (r = 3): the planes a
    # slab shares with its neighbours are reduced in slab order
    d = synth.random_small((13, 6, 17), 3, r=3, n_sub=15, seed=31)
    ref, _, (kmin, kmax) = oracle.Problem.from_domain(d).step(d.c0)
    dom = _dev(d)
    out, st = fd.fdirw_step(dom, to_dev(d.c0), prec=fd.FP64, tune=slab, stats=True, deterministic=True)
    again = fd.fdirw_step(dom, to_dev(d.c0), prec=fd.FP64, tune=slab, deterministic=True)
    assert np.max(np.abs(to_host(out) - ref)) <= 1e-13
    assert np.array_equal(to_host(out), to_host(again))
    assert st["tuned_config_id"] == min(slab, d.shape[0])      # planes along z (nz = 13)
    assert st["kmass_min"] == pytest.approx(kmin, abs=1e-13) and st["kmass_max"] == pytest.approx(kmax, abs=1e-13)


@pytest.mark.parametrize("slab", [1, 3, 1000])
def test_deterministic_flat_layout_slabs(slab):
    # FP32 at r = 5 (two lines per workgroup of the flat kernel) in slabs of
    # source planes, the thinnest far below the window
    d = synth.random_small((14, 9, 7), 3, r=5, n_sub=21, seed=32)
    ref, used, _ = oracle.Problem.from_domain(d).step(d.c0)
    dom = _dev(d)
    out, st = fd.fdirw_step(dom, to_dev(d.c0), prec=fd.FP32, tune=slab, stats=True, deterministic=True)
    again = fd.fdirw_step(dom, to_dev(d.c0), prec=fd.FP32, tune=slab, deterministic=True)
    A = to_host(out)
    assert np.max(np.abs(A - ref)) <= 1e-5
    assert np.array_equal(A, to_host(again))
    assert st["n_sources"] == used and st["tuned_config_id"] == min(slab, d.shape[0])
    atomic = to_host(fd.fdirw_step(dom, to_dev(d.c0), prec=fd.FP32))
    assert np.max(np.abs(A - atomic)) <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("prec", [fd.FP64, fd.FP32, fd.FP16X32])
def test_deterministic_one_hot_is_placed_kernel_bitwise(prec):
    d = synth.random_small((9, 10, 11), 3, r=3, n_sub=30, seed=41)
    dom = _dev(d)
    for (z, y, x) in [(0, 0, 0), (4, 5, 6), (8, 9, 10)]:
        s = (z * 10 + y) * 11 + x
        e = np.zeros(d.shape)
        e[z, y, x] = 1.0
        out = to_host(fd.fdirw_step(dom, to_dev(e), prec=prec, deterministic=True, tune=2))
        G, m = fd.fdirw_kernels(dom, to_dev(np.array([s], dtype=np.int64)), prec=prec)
        g = to_host(G)[0].astype(np.float64)
        if prec != fd.FP64:
            g = (1.0 / float(to_host(m)[0])) * g
        assert np.array_equal(out, place(d.shape, s, g))


@pytest.mark.parametrize("prec", [fd.FP64, fd.FP32])
def test_deterministic_batched_equals_single_bitwise(prec):
    ds = [synth.random_small(shape, 3, r=r, n_sub=n, seed=50 + i)
          for i, (shape, r, n) in enumerate([((7, 8, 9), 2, 10), ((12, 5, 14), 8, 30), ((6, 6, 6), 0, 3),
                                             ((20, 19, 11), 4, 33)])]
    doms = [_dev(d) for d in ds]
    outs, sts = fd.fdirw_step(doms, [to_dev(d.c0) for d in ds], prec=prec, stats=True, deterministic=True)
    for d, dom, o, st in zip(ds, doms, outs, sts):
        one = fd.fdirw_step(dom, to_dev(d.c0), prec=prec, deterministic=True)
        assert np.array_equal(to_host(o), to_host(one))
        ref, used, _ = oracle.Problem.from_domain(d).step(d.c0)
        assert np.max(np.abs(to_host(o) - ref)) <= (1e-12 if prec == fd.FP64 else 1e-5)
        assert st["n_sources"] == used
    # fdirw_run over the batch: each domain bitwise its own single run
    cs = [to_dev(d.c0) for d in ds]
    fd.fdirw_run(doms, cs, 2, prec=prec, deterministic=True)
    for d, dom, c in zip(ds, doms, cs):
        one = to_dev(d.c0)
        fd.fdirw_run(dom, one, 2, prec=prec, deterministic=True)
        assert np.array_equal(to_host(c), to_host(one))


@pytest.mark.parametrize("bank,r", [(0, 3), (1 << 34, 3), (0, 6)])
def test_deterministic_run_resumes_bitwise(bank, r):
    d = synth.random_small((12, 11, 10), 3, r=r, n_sub=20, seed=61)
    dom = _dev(d)
    full = to_dev(d.c0)
    _, st = fd.fdirw_run(dom, full, 3, prec=fd.FP32, stats=True, bank_budget_bytes=bank, deterministic=True)
    assert st["bank_used"] == (1 if bank else 0)
    part = to_dev(d.c0)
    fd.fdirw_run(dom, part, 1, prec=fd.FP32, bank_budget_bytes=bank, deterministic=True)
    fd.fdirw_run(dom, part, 2, prec=fd.FP32, bank_budget_bytes=bank, deterministic=True)
    assert np.array_equal(to_host(full), to_host(part))
    c = d.c0
    p = oracle.Problem.from_domain(d)
    for _ in range(3):
        c, _, _ = p.step(c)
    assert np.max(np.abs(to_host(full) - c)) <= 1e-5


def test_deterministic_argument_errors():
    d = synth.random_small((6, 6, 6), 2, r=2, n_sub=4, seed=71)
    dom = _dev(d)
    c = to_dev(d.c0)
    o = fd.make_opts(fd.FP32, deterministic=2)
    import ctypes
    ds = dom.c_struct()
    out = torch.empty_like(c)
    st = fd.load_library().fdirw_step(ctypes.byref(ds), 1, ctypes.byref(o), fd._ptr_array([c]), fd._ptr_array([out]),
                                      None)
    assert st == fd.E_ARG
    nn = fd.Surrogate(4, seed=0)
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_step(fd.Domain(d.label, d.d_phase, 8, 4), c, nn=nn, deterministic=True)
    assert e.value.status == fd.E_UNSUPPORTED


@pytest.mark.slow
def test_deterministic_config1_full_grid_repeats_bitwise():
    """96^3 Voronoi three-phase grid, r = 8, 200 sub-steps, every cell a
    source: two deterministic steps are bitwise equal and differ from the
    atomic step by summation order only."""
    d = synth.config1()
    dom = _dev(d)
    c0 = to_dev(d.c0)
    a = to_host(fd.fdirw_step(dom, c0, prec=fd.FP32, deterministic=True))
    b = to_host(fd.fdirw_step(dom, c0, prec=fd.FP32, deterministic=True))
    c = to_host(fd.fdirw_step(dom, c0, prec=fd.FP32))
    assert np.array_equal(a, b)
    assert np.max(np.abs(a - c)) <= 1e-12 * np.abs(a).max()
