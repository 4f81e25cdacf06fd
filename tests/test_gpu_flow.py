"""GPU parity of the steady-flow window kernels (upwind advection added to the
explicit diffusion, the flow extension of P in Sec. 5) and of the coarse
operator built from them, through the C ABI, against the oracle (pinned in
test_oracle_flow.py and test_oracle_coarse.py).

Bars: FP64 kernels to 1e-13 (mass to 1e-13), FP32 kernels to 1e-6 relative,
coarse P / P_BC to 1e-13 and the coarse step to 1e-12 in FP64."""
import numpy as np
import pytest

import oracle
import synth
from helpers import to_dev, to_host
from oracle import coarse

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2408_11376_amd as fd  # noqa: E402


def _flow_case(shape, r, n_sub, seed, umax=0.5, dt=0.1):
    # lambda <= 0.1 per face (D <= 1), Courant numbers <= 0.05 per face: the
    # explicit scheme stays stable
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed)
    u = (synth.uniform(seed + 1000, 3 * d.label.size).reshape((3,) + d.label.shape) * 2.0 - 1.0) * umax
    return d, u, dt


@pytest.mark.parametrize("shape,r,n_sub,seed", [((7, 8, 9), 2, 10, 41), ((12, 11, 10), 4, 25, 42),
                                                ((3, 2, 30), 3, 12, 43)])
def test_flow_kernels_fp64_match_oracle(shape, r, n_sub, seed):
    d, u, dt = _flow_case(shape, r, n_sub, seed)
    p = oracle.Problem(d.label, d.d_phase, r, n_sub, d.h, dt, velocity=u)
    src = np.arange(0, d.label.size, 3)
    Gw, mw = p.kernels(src)
    dom = fd.Domain(d.label, d.d_phase, r, n_sub, d.h, dt)
    G, mass = fd.fdirw_kernels_flow(dom, to_dev(u), to_dev(src), prec=fd.FP64)
    assert np.max(np.abs(to_host(G) - Gw)) <= 1e-13
    assert np.max(np.abs(to_host(mass) - mw)) <= 1e-13
    assert np.max(np.abs(to_host(mass) - 1.0)) <= 1e-13         # no sinks: the window conserves mass


def test_flow_kernels_fp32_and_zero_flow():
    d, u, dt = _flow_case((9, 10, 8), 3, 20, 44)
    dom = fd.Domain(d.label, d.d_phase, 3, 20, d.h, dt)
    src = to_dev(np.arange(d.label.size))
    p = oracle.Problem(d.label, d.d_phase, 3, 20, d.h, dt, velocity=u)
    Gw, _ = p.kernels(np.arange(d.label.size))
    G32, _ = fd.fdirw_kernels_flow(dom, to_dev(u), src, prec=fd.FP32)
    assert np.max(np.abs(to_host(G32) - Gw)) <= 1e-6
    # no flow: the plain kernels
    G0, _ = fd.fdirw_kernels_flow(dom, to_dev(np.zeros_like(u)), src, prec=fd.FP64)
    Gp, _ = fd.fdirw_kernels(dom, src, prec=fd.FP64)
    assert np.max(np.abs(to_host(G0) - to_host(Gp))) <= 1e-14


@pytest.mark.parametrize("shape,r,n_sub,seed", [((10, 9, 11), 4, 16, 47), ((12, 13, 14), 8, 12, 48),
                                                 ((9, 7, 8), 5, 14, 51), ((8, 9, 7), 6, 11, 52)])
def test_flow_kernels_fp32_flat_layout(shape, r, n_sub, seed):
    """r = 4..8 in FP32 runs the flat-layout flow kernel: against the FP64
    oracle to 1e-6 (window edges, domain walls, the source near a corner),
    unit mass without sinks.  r = 4 runs four sources per workgroup, r = 5
    and 6 two; 198 and 101 sources leave the last workgroup short."""
    d, u, dt = _flow_case(shape, r, n_sub, seed)
    dom = fd.Domain(d.label, d.d_phase, r, n_sub, d.h, dt)
    src = np.arange(0, d.label.size, 5)
    p = oracle.Problem(d.label, d.d_phase, r, n_sub, d.h, dt, velocity=u)
    Gw, _ = p.kernels(src)
    G32, m32 = fd.fdirw_kernels_flow(dom, to_dev(u), to_dev(src), prec=fd.FP32)
    print(f"[flow fp32 flat] r={r} max |gpu - oracle| = {np.max(np.abs(to_host(G32) - Gw)):.2e}", flush=True)
    assert np.max(np.abs(to_host(G32) - Gw)) <= 1e-6
    assert np.max(np.abs(to_host(m32) - 1.0)) <= 1e-5


def test_coarse_with_flow_fp32_flat_layout_far_field():
    """The coarse build with a flow at r = 4 (flat-layout kernels with
    far-field sinks): P and P_BC against the oracle at FP32 accuracy."""
    d, u, dt = _flow_case((9, 8, 10), 4, 10, 49)
    label = d.label.copy()
    dph = np.array(list(d.d_phase) + [1.0])
    label[:, :, 0] = len(dph) - 1
    res = [0] * (len(dph) - 1) + [1]
    p = oracle.Problem(label, dph, 4, 10, d.h, dt, velocity=u)
    P = coarse.coarse_matrix(p, 3, reservoir=res)
    cg = fd.Coarse(fd.Domain(label, dph, 4, 10, d.h, dt), 3, fd.FP32, reservoir=res, velocity=to_dev(u))
    kw = 2 * cg.K + 1
    got = cg.matrix()
    ncz, ncy, ncx = cg.coarse_shape
    ref = np.zeros_like(got)
    for I in range(P.shape[0]):
        bz, rem = divmod(I, ncy * ncx)
        by, bx = divmod(rem, ncx)
        for o in range(kw ** 3):
            oz, rem2 = divmod(o, kw * kw)
            oy, ox = divmod(rem2, kw)
            jz, jy, jx = bz - (oz - cg.K), by - (oy - cg.K), bx - (ox - cg.K)
            if 0 <= jz < ncz and 0 <= jy < ncy and 0 <= jx < ncx:
                ref[o, I] = P[I, (jz * ncy + jy) * ncx + jx]
    assert np.max(np.abs(got - ref)) <= 2e-6 * np.abs(ref).max()
    cg.close()


def test_flow_instability_and_errors():
    d, u, dt = _flow_case((5, 5, 5), 2, 4, 45)
    dom = fd.Domain(d.label, d.d_phase, 2, 4, d.h, dt)
    src = to_dev(np.arange(10))
    with pytest.raises(fd.FdirwError):
        fd.fdirw_kernels_flow(dom, to_dev(u * 20.0), src, prec=fd.FP64)      # Courant sum > 1
    with pytest.raises(fd.FdirwError):
        fd.fdirw_kernels_flow(dom, to_dev(u), src, prec=fd.FP16X32)          # FP64 / FP32 only


@pytest.mark.parametrize("B,far", [(2, False), (3, True), (1, True)])
def test_coarse_with_flow_matches_oracle(B, far):
    d, u, dt = _flow_case((6, 7, 8), 2, 9, 46)
    label = d.label.copy()
    dph = np.array(list(d.d_phase) + [1.0])
    res = None
    if far:
        label[:, :, 0] = len(dph) - 1
        label[:, :, -1] = len(dph) - 1
        res = [0] * (len(dph) - 1) + [1]
    p = oracle.Problem(label, dph, 2, 9, d.h, dt, velocity=u)
    P = coarse.coarse_matrix(p, B, reservoir=res)
    cg = fd.Coarse(fd.Domain(label, dph, 2, 9, d.h, dt), B, fd.FP64, reservoir=res, velocity=to_dev(u))
    kw = 2 * cg.K + 1
    got = cg.matrix()
    ncz, ncy, ncx = cg.coarse_shape
    ref = np.zeros_like(got)
    for I in range(P.shape[0]):
        bz, rem = divmod(I, ncy * ncx)
        by, bx = divmod(rem, ncx)
        for o in range(kw ** 3):
            oz, rem2 = divmod(o, kw * kw)
            oy, ox = divmod(rem2, kw)
            jz, jy, jx = bz - (oz - cg.K), by - (oy - cg.K), bx - (ox - cg.K)
            if 0 <= jz < ncz and 0 <= jy < ncy and 0 <= jx < ncx:
                ref[o, I] = P[I, (jz * ncy + jy) * ncx + jx]
    assert np.max(np.abs(got - ref)) <= 1e-13
    if far:
        pbc = coarse.p_bc(p, B, reservoir=res)
        assert np.max(np.abs(cg.p_bc() - pbc)) <= 1e-13
        fixed = coarse.reservoir_mask(label, res)
        c = np.where(fixed, 0.2, d.c0)
        m_total = c[~fixed].sum() + 0.2 * 9.0
        want, cff_w = coarse.step_far_field(p, P, pbc, c, 0.2, m_total, 9.0, B, reservoir=res)
        out, cff = cg.step_far_field(to_dev(c), 0.2, m_total, 9.0)
        assert np.max(np.abs(to_host(out) - want)) <= 1e-12 * np.abs(want).max()
        assert abs(cff - cff_w) <= 1e-12
    else:
        want = coarse.step(p, P, d.c0, B)
        out = cg.step(to_dev(d.c0))
        assert np.max(np.abs(to_host(out) - want)) <= 1e-12 * np.abs(want).max()
    cg.close()
