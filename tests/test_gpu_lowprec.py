"""GPU: the reduced-precision kernel modes against the 16-bit-copy oracle.

FP16X32 and BF16X32 keep the state in FP32 and publish it to the neighbours
as copies rounded to FP16 / BF16 (ties to even) every sub-step; FP16_STATE /
BF16_STATE round the state itself every sub-step.  oracle/lowprec.py does the
same with an FP64 state (and an FP64 accumulation).  Two checks per mode:
  * the kernels lie within twice the oracle's bound for the copies, 12 n
    lambda_max 2^-bits (the device's kernel and the oracle's are each that
    close to the exact one), plus the FP32 state's own rounding (per
    sub-step at most seven FMA roundings of values <= 1 and the FP32
    coefficients: 8 n 2^-24);
  * the kernels are closer to the oracle's copy kernels than to the exact
    FP64 kernels (summed |difference| over all kernels, at most half of it):
    the device really rounds the copies, and rounds them the oracle's way.  A
    device that kept FP32 copies would sit next to the exact kernels instead.
    (Summed over the sources: a source in a slow phase barely spreads, and its
    copy effect can be as small as the FP32 state's own rounding.)"""
import numpy as np
import pytest

import oracle
import synth
from helpers import to_dev, to_host
from oracle import lowprec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2408_11376_amd as fd  # noqa: E402


@pytest.mark.parametrize("prec,fmt,state", [(fd.FP16X32, lowprec.FP16, False), (fd.BF16X32, lowprec.BF16, False),
                                            (fd.FP16_STATE, lowprec.FP16, True), (fd.BF16_STATE, lowprec.BF16, True)])
@pytest.mark.parametrize("shape,r,n_sub,seed", [((11, 10, 12), 4, 30, 91), ((9, 13, 8), 3, 45, 92),
                                                 ((12, 12, 12), 6, 60, 93)])
def test_copy_modes_follow_the_copy_oracle(prec, fmt, state, shape, r, n_sub, seed):
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed)
    dom = fd.Domain(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)
    p = oracle.Problem.from_domain(d)
    src = np.arange(seed % 7, d.label.size, 29)
    print(f"[lowprec] prec={prec} shape={shape} r={r} n_sub={n_sub} sources={src.size}", flush=True)
    G, m = fd.fdirw_kernels(dom, to_dev(src), prec=prec)
    Gd = to_host(G).astype(np.float64).reshape(src.size, -1)
    Gc, _ = lowprec.kernels(p, src, fmt, state)
    Ge, _ = p.kernels(src)
    Gc = Gc.reshape(src.size, -1)
    Ge = Ge.reshape(src.size, -1)
    lam_max = max(p.lx.max(), p.ly.max(), p.lz.max())
    bound = 2.0 * lowprec.error_bound(n_sub, lam_max, fmt, state) + 8.0 * n_sub * 2.0 ** -24
    assert np.max(np.abs(Gd - Gc)) <= bound
    to_copy = np.abs(Gd - Gc).sum()
    to_exact = np.abs(Gd - Ge).sum()
    print(f"[lowprec] L1 to the copy oracle {to_copy:.3e}, to the exact kernels {to_exact:.3e}", flush=True)
    assert to_copy <= 0.5 * to_exact
