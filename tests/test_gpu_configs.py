"""GPU parity at the benchmark grid sizes, on sources the oracle can check.

* 192^3 GRF porous grid (solid fraction 0.35, correlation length 6, D 1 /
  1e-6, r = 8, 200 sub-steps): c0 is kept on a 16^3 sub-block of sources
  (4,096 kernels) and zeroed elsewhere, and the full 192^3 output of every
  precision mode is compared with the FP64 oracle (Sec. 4.2 compares every
  precision against FP64): FP64 L_inf <= 1e-12, FP32 L_inf <= 1e-5, the
  FP16 / BF16 copy and bank modes relative L1 <= 1e-3 with the mass
  conserved to 1e-6 (their kernels are renormalised).  The *_STATE controls
  (16-bit state every sub-step) are held to the looser bars their rounding
  allows.
* 96^3 Voronoi three-phase grid (200 seeds, boundary width 2, log-uniform D
  per phase, r = 8, 200 sub-steps): a 16^3 source sub-block in FP32 against
  the oracle, and ten big steps of the full field, regenerated every step
  (fused) against the stored kernel bank (the same kernels, superposed in
  another order: 1e-12 relative).
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import rel_l1, to_dev, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2408_11376_amd as fd  # noqa: E402


def _dev(d):
    return fd.Domain(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)


@pytest.fixture(scope="module")
def grf192():
    d = synth.config2()
    m = synth.sub_block_sources(d.shape, 16)
    c0 = np.where(m, d.c0, 0.0)
    print(f"[configs] oracle: 192^3 GRF, 16^3 = {int(m.sum())} sources", flush=True)
    ref, used, _ = oracle.Problem.from_domain(d).step(c0)
    return d, c0, ref, used


@pytest.mark.parametrize("prec,bar", [(fd.FP64, ("linf", 1e-12)), (fd.FP32, ("linf", 1e-5)),
                                      (fd.FP16X32, ("rel_l1", 1e-3)), (fd.BF16X32, ("rel_l1", 1e-3)),
                                      (fd.FP16_BANK, ("rel_l1", 1e-3)), (fd.BF16_BANK, ("rel_l1", 1e-3)),
                                      (fd.FP16_STATE, ("rel_l1", 2e-2)), (fd.BF16_STATE, ("rel_l1", 1e-1))])
def test_grf192_subblock_every_mode_vs_fp64_oracle(grf192, prec, bar):
    d, c0, ref, used = grf192
    out, st = fd.fdirw_step(_dev(d), to_dev(c0), prec=prec, stats=True)
    got = to_host(out)
    assert st["n_sources"] == used == 4096
    kind, tol = bar
    err = np.max(np.abs(got - ref)) if kind == "linf" else rel_l1(got, ref)
    print(f"[configs] 192^3 sub-block prec={prec}: {kind} {err:.3e}", flush=True)
    assert err <= tol, err
    drift = abs(st["mass_out"] - st["mass_in"]) / st["mass_in"]
    assert drift <= (1e-12 if prec in (fd.FP64, fd.FP32) else 1e-6), drift
    # every output cell lies in the union of the block's windows
    assert np.all(got[ref == 0.0] == 0.0)


@pytest.fixture(scope="module")
def voronoi96():
    return synth.config1()


def test_voronoi96_subblock16_fp32_vs_oracle(voronoi96):
    d = voronoi96
    m = synth.sub_block_sources(d.shape, 16)
    c0 = np.where(m, d.c0, 0.0)
    print("[configs] oracle: 96^3 Voronoi, 16^3 sources", flush=True)
    ref, used, _ = oracle.Problem.from_domain(d).step(c0)
    out, st = fd.fdirw_step(_dev(d), to_dev(c0), prec=fd.FP32, stats=True)
    assert st["n_sources"] == used == 4096
    assert np.max(np.abs(to_host(out) - ref)) <= 1e-5
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-12 * st["mass_in"]


def test_voronoi96_ten_steps_fused_equals_bank(voronoi96):
    d = voronoi96
    dom = _dev(d)
    a = to_dev(d.c0)
    b = to_dev(d.c0)
    print("[configs] 96^3 Voronoi: 10 fused big steps", flush=True)
    _, sa = fd.fdirw_run(dom, a, 10, prec=fd.FP32, stats=True)
    W3 = (2 * d.r + 1) ** 3
    budget = d.n * W3 * 4 + 2 * d.n * 8 + (1 << 30)
    print("[configs] 96^3 Voronoi: 10 big steps from the kernel bank", flush=True)
    _, sb = fd.fdirw_run(dom, b, 10, prec=fd.FP32, stats=True, bank_budget_bytes=budget)
    assert sa["bank_used"] == 0 and sb["bank_used"] == 1
    A, B = to_host(a), to_host(b)
    assert np.max(np.abs(A - B)) <= 1e-12 * np.abs(A).max()
    m0 = oracle.field_sum(d.c0)
    for s in (sa, sb):
        assert abs(s["mass_out"] - m0) <= 1e-12 * m0
