"""GPU: fdirw_step_noalloc, the fused step for callers that cannot allocate.

Its output is compared with fdirw_step's on the same inputs (the same kernels
and arithmetic; the FP64 atomics of the superposition may add in another
order): FP64 within 1e-12 and FP32 within 1e-5 of the step (L_inf), the
16-bit-copy modes within 1e-12 relative, and FP64 / FP32 also against the
oracle.  Two calls in a row, the second on a smaller grid, exercise the
shared scratch array (flags, counters, table and partials keep the previous
call's contents until rewritten)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from helpers import to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2408_11376_amd as fd  # noqa: E402


def _dev(d):
    return fd.Domain(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)


def _check_pair(d, prec):
    dom = _dev(d)
    c0 = to_dev(d.c0)
    print(f"[noalloc] prec={prec} shape={d.shape} r={d.r} n_sub={d.n_sub}", flush=True)
    ref_gpu, st_ref = fd.fdirw_step(dom, c0, prec=prec, stats=True)
    out, st = fd.fdirw_step_noalloc(dom, c0, torch.full_like(c0, np.nan), prec=prec, stats=True)
    A, B = to_host(out), to_host(ref_gpu)
    scale = max(np.abs(B).max(), 1e-300)
    if prec == fd.FP64:
        assert np.max(np.abs(A - B)) <= 1e-12
    elif prec == fd.FP32:
        assert np.max(np.abs(A - B)) <= 1e-5
    else:
        assert np.max(np.abs(A - B)) <= 1e-12 * scale
    assert st["n_sources"] == st_ref["n_sources"]
    assert st["mass_in"] == st_ref["mass_in"]
    assert st["kmass_min"] == st_ref["kmass_min"] and st["kmass_max"] == st_ref["kmass_max"]
    assert abs(st["mass_out"] - st_ref["mass_out"]) <= 1e-12 * abs(st_ref["mass_out"])
    if prec in (fd.FP64, fd.FP32):
        ref, used, _ = oracle.Problem.from_domain(d).step(d.c0)
        assert np.max(np.abs(A - ref)) <= (1e-12 if prec == fd.FP64 else 1e-5)
        assert st["n_sources"] == used
    # without statistics (no kernel-mass partials)
    again = to_host(fd.fdirw_step_noalloc(dom, c0, torch.empty_like(c0), prec=prec))
    assert np.max(np.abs(again - B)) <= (1e-12 if prec == fd.FP64 else 1e-5) * (1.0 if prec in (fd.FP64, fd.FP32)
                                                                                else scale)


@pytest.mark.parametrize("prec", [fd.FP64, fd.FP32, fd.FP16X32, fd.BF16X32])
def test_noalloc_matches_step_two_calls_second_smaller(prec):
    big = synth.random_small((14, 13, 15), 3, r=4, n_sub=30, seed=801)
    small = synth.random_small((5, 7, 6), 2, r=3, n_sub=12, seed=802)
    _check_pair(big, prec)
    _check_pair(small, prec)


def test_noalloc_window_radius_8_grf():
    # the benchmark's radius and sub-step count on a small porous grid,
    # several source lines per CU and windows clipped on every side
    d = synth.config2(seed=803, n=24)
    _check_pair(d, fd.FP32)


def test_noalloc_fp32_line_groups():
    # FP32 at r = 5 and 6 runs two source lines per workgroup: 45 and 35 lines
    # leave the last workgroup's second line empty
    for shape, r, n_sub, seed in [((7, 5, 9), 5, 14, 814), ((9, 7, 5), 6, 11, 815)]:
        _check_pair(synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed), fd.FP32)


def test_noalloc_edge_cases():
    # one cell; r = 0; no sub-steps
    for shape, r, n_sub, seed in [((1, 1, 1), 3, 5, 811), ((4, 5, 6), 0, 7, 812), ((6, 5, 4), 2, 0, 813)]:
        _check_pair(synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed), fd.FP64)


def test_noalloc_rejections():
    d = synth.random_small((6, 6, 6), 3, r=2, n_sub=4, seed=821)
    dom = _dev(d)
    c = to_dev(d.c0)
    out = torch.empty_like(c)
    lib = fd.load_library()
    ds = dom.c_struct()
    for kw, code in [({"prec": fd.FP16_STATE}, fd.E_UNSUPPORTED), ({"prec": fd.FP16_BANK}, fd.E_UNSUPPORTED),
                     ({"deterministic": 1}, fd.E_UNSUPPORTED)]:
        o = fd.make_opts(**kw)
        assert lib.fdirw_step_noalloc(ctypes.byref(ds), ctypes.byref(o), ctypes.c_void_p(c.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), None) == code
    o = fd.make_opts(fd.FP32)
    assert lib.fdirw_step_noalloc(ctypes.byref(ds), ctypes.byref(o), ctypes.c_void_p(c.data_ptr()),
                                  ctypes.c_void_p(c.data_ptr()), None) == fd.E_ARG
    nn = fd.Surrogate(4, seed=0)
    o = fd.make_opts(fd.FP32, gen=fd.GEN_NN, nn=nn)
    assert lib.fdirw_step_noalloc(ctypes.byref(ds), ctypes.byref(o), ctypes.c_void_p(c.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), None) == fd.E_UNSUPPORTED
    # statistics need one kernel-mass slot per workgroup: a grid with more
    # source lines than the scratch holds is refused with stats, runs without
    wide = synth.random_small((1, 250, 280), 2, r=1, n_sub=3, seed=822)
    wdom = _dev(wide)
    wc = to_dev(wide.c0)
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_step_noalloc(wdom, wc, torch.empty_like(wc), prec=fd.FP64, stats=True)
    assert e.value.status == fd.E_ARG
    got = to_host(fd.fdirw_step_noalloc(wdom, wc, torch.empty_like(wc), prec=fd.FP64))
    ref = to_host(fd.fdirw_step(wdom, wc, prec=fd.FP64))
    assert np.max(np.abs(got - ref)) <= 1e-12
