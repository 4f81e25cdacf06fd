"""GPU: the flat-layout fused kernel (FP32 steps with r = 4..8).

It generates the same window kernels as the segment-layout kernels (same
terms in the same order per cell) and superposes them through a register
shift ring, so its step must equal
  * the FP64 oracle within the FP32 bar (L_inf 1e-5),
  * the deterministic step (segment-layout kernels, fixed-order sums) up to
    the summation order of the superposition and of the kernel masses
    (1e-13 relative),
  * for a one-hot field, the kernel of fdirw_kernels divided by its mass,
    placed at the source (same nonzero pattern, values within 1e-14
    relative: the masses are summed in another grouping).
Cases cover every radius of the kernel, domains smaller than the window,
lines cut into several segments, odd and zero sub-step counts, zero sources
between nonzero ones (the ring still shifts past them), and line counts that
leave the last workgroup's group of lines short (r = 4 runs four lines per
workgroup, r = 5 and 6 two: 110 and 9 lines at r = 4, 91 at r = 5, 99 at
r = 6)."""
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


CASES = [((9, 10, 11), 4, 21, 901), ((12, 7, 13), 5, 30, 902), ((6, 15, 8), 6, 17, 903),
         ((16, 16, 16), 7, 40, 904), ((19, 18, 20), 8, 45, 905), ((5, 6, 7), 8, 33, 906),
         ((1, 1, 1), 8, 5, 907), ((3, 20, 2), 8, 0, 908), ((25, 4, 9), 4, 1, 909),
         ((10, 9, 11), 6, 23, 910), ((8, 3, 3), 4, 12, 912), ((11, 5, 7), 7, 19, 913),
         # one line at r = 4 (three of the workgroup's four line groups empty), three at r = 6
         ((6, 1, 1), 4, 9, 914), ((5, 1, 3), 6, 8, 915)]


@pytest.mark.parametrize("shape,r,n_sub,seed", CASES)
def test_flat_step_matches_oracle_and_segment_kernels(shape, r, n_sub, seed):
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed)
    c0 = d.c0.copy()
    c0.reshape(-1)[::3] = 0.0                        # zero sources between nonzero ones
    print(f"[flat] shape={shape} r={r} n_sub={n_sub}", flush=True)
    dom = _dev(d)
    out, st = fd.fdirw_step(dom, to_dev(c0), prec=fd.FP32, stats=True)
    A = to_host(out)
    ref, used, (kmin, kmax) = oracle.Problem.from_domain(d).step(c0)
    assert np.max(np.abs(A - ref)) <= 1e-5
    assert st["n_sources"] == used
    det, sd = fd.fdirw_step(dom, to_dev(c0), prec=fd.FP32, stats=True, deterministic=True)
    B = to_host(det)
    assert np.max(np.abs(A - B)) <= 1e-13 * max(np.abs(B).max(), 1e-300)
    if used:
        assert st["kmass_min"] == pytest.approx(sd["kmass_min"], rel=1e-14)
        assert st["kmass_max"] == pytest.approx(sd["kmass_max"], rel=1e-14)
        # FP32 kernels lose or gain ~1e-5 of their mass over the sub-steps (1 - sum lambda
        # rounded); the FP64 oracle keeps it to 1e-13
        assert st["kmass_min"] == pytest.approx(kmin, abs=5e-5) and st["kmass_max"] == pytest.approx(kmax, abs=5e-5)


@pytest.mark.parametrize("tune", [2, 3, 7])
def test_flat_step_lines_in_segments(tune):
    d = synth.random_small((23, 9, 8), 3, r=8, n_sub=25, seed=911)
    dom = _dev(d)
    out, st = fd.fdirw_step(dom, to_dev(d.c0), prec=fd.FP32, tune=tune, stats=True)
    ref, used, _ = oracle.Problem.from_domain(d).step(d.c0)
    seg_len = -(-23 // tune)                        # the library's split of nz = 23 into `tune` segments
    assert st["tuned_config_id"] == -(-23 // seg_len)
    assert np.max(np.abs(to_host(out) - ref)) <= 1e-5
    whole = to_host(fd.fdirw_step(dom, to_dev(d.c0), prec=fd.FP32, tune=1))
    assert np.max(np.abs(to_host(out) - whole)) <= 1e-13 * np.abs(whole).max()


@pytest.mark.parametrize("r", [4, 5, 6, 8])
def test_flat_one_hot_is_placed_kernel(r):
    d = synth.random_small((14, 13, 15), 3, r=r, n_sub=37, seed=921 + r)
    dom = _dev(d)
    nz, ny, nx = d.shape
    for (z, y, x) in [(0, 0, 0), (7, 6, 7), (13, 12, 14), (2, 12, 1), (13, 0, 7)]:
        s = (z * ny + y) * nx + x
        e = np.zeros(d.shape)
        e[z, y, x] = 1.0
        out = to_host(fd.fdirw_step(dom, to_dev(e), prec=fd.FP32))
        G, m = fd.fdirw_kernels(dom, to_dev(np.array([s], dtype=np.int64)), prec=fd.FP32)
        g = (1.0 / float(to_host(m)[0])) * to_host(G)[0].astype(np.float64)
        want = place(d.shape, s, g)
        assert np.array_equal(out != 0, want != 0)
        assert np.max(np.abs(out - want)) <= 1e-14 * np.abs(want).max()


def test_flat_grf_radius8_200_substeps_subblock():
    # the benchmark's geometry kind, radius and sub-step count on a 40^3 grid,
    # a 10^3 block of sources
    d = synth.config2(seed=931, n=40)
    m = synth.sub_block_sources(d.shape, 10)
    c0 = np.where(m, d.c0, 0.0)
    out, st = fd.fdirw_step(_dev(d), to_dev(c0), prec=fd.FP32, stats=True)
    ref, used, _ = oracle.Problem.from_domain(d).step(c0)
    assert st["n_sources"] == used == 1000
    assert np.max(np.abs(to_host(out) - ref)) <= 1e-5
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-9 * st["mass_in"]
