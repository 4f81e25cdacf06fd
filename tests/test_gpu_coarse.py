"""GPU parity of the coarse-mesh FDiRW (Sec. 3.1, Eqs. 10-15) through the C ABI
against the coarse oracle (oracle/coarse.py, pinned in test_oracle_coarse.py).

Bars: P and the step in FP64 to 1e-13 / 1e-12 (atomic summation order only);
FP32 P to 1e-6 of the field maximum (1e-5 per entry at 192^3); FP16 / BF16 P:
relative L1 of the step <= 1e-3 / 5e-3; immobile cells bit-exact; mass to
1e-12 with FP64 P."""
import numpy as np
import pytest

import oracle
import synth
from helpers import rel_l1, to_dev, to_host
from oracle import coarse

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2408_11376_amd as fd  # noqa: E402


def _dev_domain(d):
    return fd.Domain(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)


def _offset_form(P, cshape, K):
    """Dense oracle P[I, J] -> [o, I] with o = (oz, oy, ox) = I - J + K."""
    ncz, ncy, ncx = cshape
    kw = 2 * K + 1
    out = np.zeros((kw ** 3, P.shape[0]))
    for I in range(P.shape[0]):
        bz, rem = divmod(I, ncy * ncx)
        by, bx = divmod(rem, ncx)
        for o in range(kw ** 3):
            oz, rem2 = divmod(o, kw * kw)
            oy, ox = divmod(rem2, kw)
            jz, jy, jx = bz - (oz - K), by - (oy - K), bx - (ox - K)
            if 0 <= jz < ncz and 0 <= jy < ncy and 0 <= jx < ncx:
                out[o, I] = P[I, (jz * ncy + jy) * ncx + jx]
    return out


# K = ceil(r / B) from 1 to 5: K >= 5 runs the product with one lane per chunk
# of P's layout and a second, ordered summing launch (ragged z chunks here)
CASES = [((6, 7, 5), 2, 6, 2, 11), ((9, 8, 10), 3, 10, 3, 12), ((5, 4, 6), 2, 5, 8, 13), ((7, 6, 8), 2, 8, 1, 14),
         ((3, 1, 70), 2, 4, 5, 15), ((7, 6, 5), 4, 6, 1, 21), ((9, 5, 6), 5, 7, 1, 22), ((11, 5, 6), 8, 6, 2, 23)]


@pytest.mark.parametrize("shape,r,n_sub,B,seed", CASES)
def test_matrix_and_step_fp64_match_oracle(shape, r, n_sub, B, seed):
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed)
    p = oracle.Problem.from_domain(d)
    P = coarse.coarse_matrix(p, B)
    cg = fd.Coarse(_dev_domain(d), B, fd.FP64)
    assert cg.coarse_shape == coarse.coarse_dims(shape, B)
    assert cg.K == -(-r // B)
    got = cg.matrix()
    ref = _offset_form(P, cg.coarse_shape, cg.K)
    assert np.max(np.abs(got - ref)) <= 1e-13
    out, st = cg.step(to_dev(d.c0), stats=True)
    want = coarse.step(p, P, d.c0, B)
    assert np.max(np.abs(to_host(out) - want)) <= 1e-12 * max(np.abs(want).max(), 1e-300)
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-12 * st["mass_in"]
    _, mobile, _ = coarse.groups(d.label, d.d_phase, B)
    assert np.array_equal(to_host(out)[~mobile], d.c0[~mobile])
    cg.close()


@pytest.mark.parametrize("B,r", [(3, 3), (1, 5)])
@pytest.mark.parametrize("prec,kind,tol", [(fd.FP32, "max", 1e-6), (fd.FP16_BANK, "l1", 1e-3),
                                           (fd.BF16_BANK, "l1", 5e-3)])
def test_reduced_precision_p(prec, kind, tol, B, r):
    d = synth.random_small((12, 11, 13), 3, r=r, n_sub=12, seed=16)
    p = oracle.Problem.from_domain(d)
    P = coarse.coarse_matrix(p, B)
    want = coarse.step(p, P, d.c0, B)
    cg = fd.Coarse(_dev_domain(d), B, prec)
    assert cg.K == -(-r // B)
    out, st = cg.step(to_dev(d.c0), stats=True)
    got = to_host(out)
    if kind == "max":
        assert np.max(np.abs(got - want)) <= tol * np.abs(want).max()
    else:
        assert rel_l1(got, want) <= tol
    # every column of the FP64 P conserves mass (sum_I N_I P[I][J] = N_J);
    # rounding each entry to the storage type moves a column's mass by at
    # most the unit roundoff u (relative), plus, for FP16, the absolute
    # rounding of subnormal entries (<= 2^-25 each, at most (2K+1)^3 of them
    # per column, weighted by N_I / N_J <= B^3); with c >= 0 the field's mass
    # moves by at most that share
    u = {fd.FP32: 2.0 ** -24, fd.FP16_BANK: 2.0 ** -11, fd.BF16_BANK: 2.0 ** -8}[prec]
    sub = (2 * cg.K + 1) ** 3 * B ** 3 * 2.0 ** -25 if prec == fd.FP16_BANK else 0.0
    assert abs(st["mass_out"] - st["mass_in"]) <= (u + sub + 1e-12) * st["mass_in"]
    cg.close()


@pytest.mark.parametrize("B,r", [(2, 3), (4, 3), (1, 5)])
def test_liquid_only_grouping_matches_oracle(B, r):
    # only phase 0 grouped (the other phases keep their values); kernels are
    # renormalised over the grouped cells.  B = 1, r = 5 (K = 5): many chunks
    # of P's layout hold no grouped node and are not stored
    d = synth.random_small((9, 10, 11), 3, r=r, n_sub=9, seed=19, d_zero_phase=False)
    grouped = [1, 0, 0]
    p = oracle.Problem.from_domain(d)
    P = coarse.coarse_matrix(p, B, grouped)
    cg = fd.Coarse(_dev_domain(d), B, fd.FP64, grouped=grouped)
    assert np.max(np.abs(cg.matrix() - _offset_form(P, cg.coarse_shape, cg.K))) <= 1e-13
    out, st = cg.step(to_dev(d.c0), stats=True)
    want = coarse.step(p, P, d.c0, B, grouped)
    assert np.max(np.abs(to_host(out) - want)) <= 1e-12 * np.abs(want).max()
    assert abs(st["mass_out"] - st["mass_in"]) <= 1e-12 * st["mass_in"]
    assert np.array_equal(to_host(out)[d.label != 0], d.c0[d.label != 0])
    cg.close()


def test_block_one_equals_the_fine_step():
    d = synth.random_small((10, 9, 11), 3, r=3, n_sub=15, seed=17)
    dom = _dev_domain(d)
    fine = to_host(fd.fdirw_step(dom, to_dev(d.c0), prec=fd.FP64))
    cg = fd.Coarse(dom, 1, fd.FP64)
    got = to_host(cg.step(to_dev(d.c0)))
    assert np.max(np.abs(got - fine)) <= 1e-12 * np.abs(fine).max()
    cg.close()


def test_two_steps_and_errors():
    d = synth.random_small((8, 9, 7), 2, r=2, n_sub=6, seed=18)
    dom = _dev_domain(d)
    cg = fd.Coarse(dom, 2, fd.FP64)
    p = oracle.Problem.from_domain(d)
    P = coarse.coarse_matrix(p, 2)
    a = cg.step(to_dev(d.c0))
    b = cg.step(a)
    want = coarse.step(p, P, coarse.step(p, P, d.c0, 2), 2)
    assert np.max(np.abs(to_host(b) - want)) <= 1e-12 * np.abs(want).max()
    with pytest.raises(fd.FdirwError):
        cg.step(a, a)
    with pytest.raises(fd.FdirwError):
        fd.Coarse(dom, 0, fd.FP64)
    with pytest.raises(fd.FdirwError):
        fd.Coarse(dom, 2, fd.FP16X32)
    cg.close()


@pytest.mark.parametrize("B,r,prec", [(3, 3, "FP16_BANK"), (1, 5, "FP16_BANK"), (1, 5, "FP64"), (2, 9, "FP32")])
def test_step_is_deterministic(B, r, prec):
    # the product sums every node in one fixed order (no atomics in the step):
    # the same handle gives bit-identical fields for the same input, in both
    # product shapes (K = 1: one lane per node; K = 5: one lane per chunk and
    # the ordered summing launch) and with a far field
    d = synth.random_small((11, 10, 13), 3, r=r, n_sub=8, seed=24)
    cg = fd.Coarse(_dev_domain(d), B, getattr(fd, prec))
    assert cg.K == -(-r // B)
    c = to_dev(d.c0)
    a = to_host(cg.step(c))
    b = to_host(cg.step(c))
    assert np.array_equal(a, b)
    cg.close()
    label, dph, c0 = _far_field_domain(20)
    res = [0, 0, 1]
    cg = fd.Coarse(fd.Domain(label, dph, r, 9, 1.0, 0.0), B, getattr(fd, prec), reservoir=res)
    c = to_dev(np.where(coarse.reservoir_mask(label, res), 0.4, c0))
    m_total = float(to_host(c).sum()) + 0.4 * 30.0
    o1, f1 = cg.step_far_field(c, 0.4, m_total, 30.0)
    o2, f2 = cg.step_far_field(c, 0.4, m_total, 30.0)
    assert np.array_equal(to_host(o1), to_host(o2)) and f1 == f2
    cg.close()


@pytest.mark.slow
def test_full_size_sampled_columns():
    """The 192^3 workload (GRF, D 1 / 1e-6, r = 8, n = 200) with 5^3 blocks and
    FP32 P: sampled columns J of P against the oracle's kernels of the
    sources of group J."""
    d = synth.config2()
    B = 5
    cg = fd.Coarse(_dev_domain(d), B, fd.FP32)
    K = cg.K
    kw = 2 * K + 1
    got = cg.matrix()
    ncz, ncy, ncx = cg.coarse_shape
    p = oracle.Problem.from_domain(d)
    block, mobile, count = coarse.groups(d.label, d.d_phase, B)
    for (jz, jy, jx) in [(0, 0, 0), (19, 20, 7), (38, 38, 38)]:
        J = (jz * ncy + jy) * ncx + jx
        src = np.flatnonzero(mobile.ravel() & (block.ravel() == J))
        S = np.zeros(count.size)
        G, mass = p.kernels(src)
        W, r = p.W, p.r
        rel = np.arange(W) - r
        for q, s in enumerate(src):
            sz, sy, sx = np.unravel_index(s, d.label.shape)
            Z, Y, X = sz + rel, sy + rel, sx + rel
            kz, ky, kx = (Z >= 0) & (Z < 192), (Y >= 0) & (Y < 192), (X >= 0) & (X < 192)
            np.add.at(S, block[np.ix_(Z[kz], Y[ky], X[kx])].ravel(), (G[q][np.ix_(kz, ky, kx)] / mass[q]).ravel())
        for o in range(kw ** 3):
            oz, rem = divmod(o, kw * kw)
            oy, ox = divmod(rem, kw)
            iz, iy, ix = jz + oz - K, jy + oy - K, jx + ox - K
            if not (0 <= iz < ncz and 0 <= iy < ncy and 0 <= ix < ncx):
                continue
            I = (iz * ncy + iy) * ncx + ix
            want = S[I] / count[I] if count[I] > 0 else 0.0
            assert abs(got[o, I] - want) <= 1e-5 * max(abs(want), 1e-3), (J, o)
    cg.close()


# ------------------------------------------------------------------ far field

def _far_field_domain(seed, shape=(5, 6, 7)):
    # x walls of reservoir phase 2 (the far-field boundary); liquid 0 and a
    # slow phase 1 inside
    d = synth.random_small(shape, 2, r=3, n_sub=9, seed=seed, d_zero_phase=False)
    label = d.label.copy()
    label[:, :, 0] = 2
    label[:, :, -1] = 2
    return label, np.array([1.0, 0.05, 1.0]), d.c0


@pytest.mark.parametrize("B,prec,tol", [(1, fd.FP64, 1e-12), (3, fd.FP64, 1e-12), (2, fd.FP32, 1e-5)])
def test_far_field_matches_oracle(B, prec, tol):
    label, dph, c0 = _far_field_domain(20)
    res = [0, 0, 1]
    p = oracle.Problem(label, dph, 3, 9, 1.0, 0.0)
    P = coarse.coarse_matrix(p, B, reservoir=res)
    pbc = coarse.p_bc(p, B, reservoir=res)
    cg = fd.Coarse(fd.Domain(label, dph, 3, 9, 1.0, 0.0), B, prec, reservoir=res)
    assert np.max(np.abs(cg.matrix() - _offset_form(P, cg.coarse_shape, cg.K))) <= tol * 0.1
    assert np.max(np.abs(cg.p_bc() - pbc)) <= tol * 0.1
    fixed = coarse.reservoir_mask(label, res)
    c_ff, v_ff = 0.4, 30.0
    c = np.where(fixed, c_ff, c0)
    m_total = c[~fixed].sum() + c_ff * v_ff
    want, cff_want = coarse.step_far_field(p, P, pbc, c, c_ff, m_total, v_ff, B, reservoir=res)
    out, cff, st = cg.step_far_field(to_dev(c), c_ff, m_total, v_ff, stats=True)
    got = to_host(out)
    assert np.max(np.abs(got - want)) <= tol * np.abs(want).max()
    assert abs(cff - cff_want) <= tol * max(abs(cff_want), 1.0)
    assert np.all(got[fixed] == cff)
    assert abs(st["mass_out"] - m_total) <= 1e-12 * m_total
    # a second step from the first
    want2, cff_want2 = coarse.step_far_field(p, P, pbc, want, cff_want, m_total, v_ff, B, reservoir=res)
    out2, cff2 = cg.step_far_field(out, cff, m_total, v_ff)
    assert np.max(np.abs(to_host(out2) - want2)) <= tol * np.abs(want2).max()
    assert abs(cff2 - cff_want2) <= tol * max(abs(cff_want2), 1.0)
    cg.close()


def test_far_field_uniform_state_is_stationary():
    # windows covering the domain: the uniform state with c_ff = c stays put
    label, dph, _ = _far_field_domain(21)
    res = [0, 0, 1]
    dom = fd.Domain(label, dph, 8, 9, 1.0, 0.0)
    cg = fd.Coarse(dom, 2, fd.FP64, reservoir=res)
    near = ~coarse.reservoir_mask(label, res)
    c = np.full(label.shape, 0.7)
    out, cff = cg.step_far_field(to_dev(c), 0.7, 0.7 * (near.sum() + 12.0), 12.0)
    assert np.max(np.abs(to_host(out) - 0.7)) <= 1e-13
    assert abs(cff - 0.7) <= 1e-13
    cg.close()


def test_far_field_errors():
    label, dph, c0 = _far_field_domain(22)
    dom = fd.Domain(label, dph, 2, 4, 1.0, 0.0)
    cf = fd.Coarse(dom, 2, fd.FP64, reservoir=[0, 0, 1])
    c = to_dev(c0)
    with pytest.raises(fd.FdirwError):
        cf.step(c)                                   # a far-field handle needs c_ff
    with pytest.raises(fd.FdirwError):
        cf.step_far_field(c, 0.1, 1.0, 0.0)          # v_ff must be > 0
    cn = fd.Coarse(dom, 2, fd.FP64)
    with pytest.raises(fd.FdirwError):
        cn.step_far_field(c, 0.1, 1.0, 1.0)          # no far field on this handle
    cf.close()
    cn.close()


@pytest.mark.parametrize("B,r,far,prec,tol", [(2, 9, False, fd.FP64, 1e-13), (3, 11, True, fd.FP64, 1e-13),
                                             (2, 16, False, fd.FP64, 1e-13), (2, 12, True, fd.FP32, 1e-6)])
def test_node_windows_match_oracle(B, r, far, prec, tol):
    # radius above the per-source kernels: P from node windows (FD of a whole
    # group on its block and the K blocks around it)
    d = synth.random_small((13, 9, 26), 3, r=r, n_sub=10, seed=60 + r)
    label = d.label.copy()
    dph = np.array(list(d.d_phase) + [1.0])
    res = None
    if far:
        label[:, :, -1] = len(dph) - 1
        res = [0] * (len(dph) - 1) + [1]
    p = oracle.Problem(label, dph, r, 10, d.h, 0.1)
    P = coarse.coarse_matrix(p, B, reservoir=res)
    cg = fd.Coarse(fd.Domain(label, dph, r, 10, d.h, 0.1), B, prec, reservoir=res)
    assert np.max(np.abs(cg.matrix() - _offset_form(P, cg.coarse_shape, cg.K))) <= tol
    if far:
        fixed = coarse.reservoir_mask(label, res)
        c = np.where(fixed, 0.3, d.c0)
        m_total = c[~fixed].sum() + 0.3 * 50.0
        want, cff_w = coarse.step_far_field(p, P, coarse.p_bc(p, B, reservoir=res), c, 0.3, m_total, 50.0, B,
                                            reservoir=res)
        out, cff = cg.step_far_field(to_dev(c), 0.3, m_total, 50.0)
        assert abs(cff - cff_w) <= 10 * tol * abs(cff_w)
    else:
        want = coarse.step(p, P, d.c0, B)
        out = cg.step(to_dev(d.c0))
    assert np.max(np.abs(to_host(out) - want)) <= 10 * tol * np.abs(want).max()
    cg.close()


def test_node_window_limits():
    d = synth.random_small((8, 8, 8), 2, r=20, n_sub=3, seed=70)
    with pytest.raises(fd.FdirwError):                            # K = ceil(20 / 2) = 10 > 8
        fd.Coarse(fd.Domain(d.label, d.d_phase, 20, 3, d.h, 0.1), 2, fd.FP64)
    u = to_dev(np.zeros((3,) + d.label.shape))
    with pytest.raises(fd.FdirwError):                            # flow kernels stop at r = 8
        fd.Coarse(fd.Domain(d.label, d.d_phase, 10, 3, d.h, 0.1), 2, fd.FP64, velocity=u)


@pytest.mark.slow
def test_full_size_node_window_columns():
    # the particle case with Table 1's big step: r = 40, 1000 fast sub-steps,
    # 5^3 blocks, FP32 build, liquid walled off from the solid, far field;
    # three sampled node columns against the oracle's node windows
    dom_s, t = synth.particle_case(192, 50.0, r=40, n_sub=1000)
    a_rt = np.array([t["A_L_RT"], t["A_S_RT"], t["A_L_RT"]])
    d_liq = dom_s.d_phase * a_rt * np.array([1.0, 0.0, 1.0])
    res = [0, 0, 1]
    grouped = [1, 0, 0]
    cg = fd.Coarse(fd.Domain(dom_s.label, d_liq, 40, 1000, dom_s.h, dom_s.dt), 5, fd.FP32, grouped=grouped,
                   reservoir=res)
    assert cg.K == 8
    got = cg.matrix()
    p = oracle.Problem(dom_s.label, d_liq, 40, 1000, dom_s.h, dom_s.dt)
    _, _, count = coarse.groups(dom_s.label, d_liq, 5, grouped, res)
    ncz, ncy, ncx = cg.coarse_shape
    used = np.flatnonzero(count > 0)
    kw = 2 * cg.K + 1
    for J in used[[0, len(used) // 2, len(used) - 1]]:
        col = coarse.node_window_column(p, 5, int(J), grouped, res)
        jz, rem = divmod(int(J), ncy * ncx)
        jy, jx = divmod(rem, ncx)
        for I in np.flatnonzero(col):
            iz, rem = divmod(int(I), ncy * ncx)
            iy, ix = divmod(rem, ncx)
            o = ((iz - jz + cg.K) * kw + (iy - jy + cg.K)) * kw + (ix - jx + cg.K)
            want = col[I] / count[I]
            assert abs(got[o, I] - want) <= 1e-5 * max(abs(want), 1e-4), (J, I)
    cg.close()


# ---------------------------------------------------------------- arithmetic of the product (Sec. 3.3, Table 2)

ARITH_PREC = {"fp64": fd.FP64, "fp32": fd.FP32, "mixed": fd.FP16_BANK, "fp16": fd.FP16_BANK}


def _block_constant(d, B, seed):
    """A field constant over every B^3 block, with values k / 64 (k < 1024):
    exact in FP16, so every group mean is the same number on both sides."""
    ncz, ncy, ncx = coarse.coarse_dims(d.shape, B)
    v = np.floor(synth.uniform(seed, ncz * ncy * ncx) * 1024.0) / 64.0
    z, y, x = np.meshgrid(*[np.arange(n) for n in d.shape], indexing="ij")
    return v[((z // B) * ncy + (y // B)) * ncx + (x // B)]


# K < 5 (one lane per node) and K >= 5 (one lane per chunk, ordered range sum)
ARITH_CASES = [((10, 9, 11), 4, 4, 2, 41), ((9, 10, 8), 5, 3, 1, 42), ((6, 7, 5), 2, 6, 2, 43)]


@pytest.mark.parametrize("arith", ["fp64", "fp32", "mixed", "fp16"])
@pytest.mark.parametrize("shape,r,n_sub,B,seed", ARITH_CASES)
def test_arith_step_matches_oracle_within_the_accumulation_bound(arith, shape, r, n_sub, B, seed):
    """Every product formed as the precision forms it (same rounded operands
    and FP16 products on both sides); only the order of the accumulation
    differs, so |GPU - oracle| <= gamma_n(u) sum |terms| per node.  The P of
    both sides must be the same number before its storage rounding, so the
    geometry is dyadic: D in {1, 0} and dt = 1/8 (lambda = 1/8), whose FD
    kernels over a few sub-steps are exact in FP32 (the reduced-precision
    handles build P from FP32 kernels, the oracle from FP64 ones)."""
    d = synth.random_small(shape, 2, r=r, n_sub=n_sub, seed=seed, dt=0.125)
    p = oracle.Problem.from_domain(d)
    P = coarse.coarse_matrix(p, B)
    cg = fd.Coarse(_dev_domain(d), B, ARITH_PREC[arith])
    cg.set_arith(arith)
    for c0 in (_block_constant(d, B, seed + 100), d.c0):
        ref, bnd = coarse.step_arith(p, P, c0, B, arith)
        got = to_host(cg.step(to_dev(c0)))
        slack = 1e-14 * np.abs(ref).max()
        if c0 is d.c0 and arith != "fp64":
            # group means of a noise field are rounded to the C type on both
            # sides from FP64 means summed in different orders: they agree
            # except at a rounding tie (probability ~1e-13 per node)
            slack += 4.0 * 2.0 ** -53 * np.abs(ref).max()
        print(f"[coarse arith] {arith} K={cg.K} max |gpu - oracle| / bound = "
              f"{np.max(np.abs(got - ref) / (bnd + slack)):.3f}", flush=True)
        assert np.all(np.abs(got - ref) <= bnd + slack)
    cg.close()


def test_arith_rejects_a_mismatched_p_storage():
    d = synth.random_small((6, 6, 6), 2, r=2, n_sub=4, seed=44)
    dom = _dev_domain(d)
    for prec, bad in ((fd.FP64, ("fp32", "mixed", "fp16")), (fd.FP32, ("mixed", "fp16")), (fd.FP16_BANK, ("fp32",))):
        cg = fd.Coarse(dom, 2, prec)
        for a in bad:
            with pytest.raises(fd.FdirwError) as e:
                cg.set_arith(a)
            assert e.value.status == fd.E_ARG
        with pytest.raises(fd.FdirwError):
            cg.set_arith(7)
        cg.set_arith("fp64")
        cg.close()


def test_arith_back_and_forth_and_far_field():
    """Switching the arithmetic of one handle back to FP64 gives the FP64
    step again bitwise; with a far field the mixed step keeps the Eq. 7
    balance (c_ff takes what the near field loses)."""
    d = synth.random_small((8, 9, 10), 3, r=3, n_sub=10, seed=45, d_zero_phase=False)
    dom = _dev_domain(d)
    cg = fd.Coarse(dom, 2, fd.FP16_BANK)
    c0 = to_dev(d.c0)
    a = to_host(cg.step(c0))
    cg.set_arith("mixed")
    m = to_host(cg.step(c0))
    cg.set_arith("fp64")
    b = to_host(cg.step(c0))
    assert np.array_equal(a, b) and not np.array_equal(a, m)
    cg.close()
    res = [0, 0, 1]
    cf = fd.Coarse(dom, 2, fd.FP16_BANK, grouped=[1, 1, 0], reservoir=res)
    cf.set_arith("mixed")
    far = d.label == 2
    v_ff = float(far.sum())
    m_total = float(d.c0[~far].sum()) + 0.3 * v_ff
    out, c_ff = cf.step_far_field(c0, 0.3, m_total, v_ff)
    o = to_host(out)
    assert abs(o[~far].sum() + c_ff * v_ff - m_total) <= 1e-12 * m_total
    cf.close()


# ---------------------------------------------------------------- ensemble product (Eq. 14, several right-hand sides)

def _ensemble_fields(n_ens, n_nodes, seed):
    """Members of different magnitudes (1e-12 .. 1e6: below FP16's normal
    range and above its largest number before the scaling), seeded."""
    v = synth.uniform(seed, n_ens * n_nodes).reshape(n_ens, n_nodes)
    scale = 10.0 ** (3 * (np.arange(n_ens) % 7) - 12)
    return v * scale[:, None]


# K = 1, 2, 3, 4; ragged 4 x 4 tiles; member counts below, at and above the
# 16-member column tile and the 128 members of one wave
ENSEMBLE_CASES = [((7, 9, 6), 2, 6, 2, 1, 70), ((10, 11, 9), 3, 8, 2, 17, 71), ((13, 9, 12), 3, 5, 1, 5, 72),
                  ((14, 12, 13), 8, 8, 2, 130, 73), ((20, 18, 22), 8, 8, 4, 16, 74),
                  # 128 or more members at K <= 2: the plane-walking form (ragged z-chunks of 8 planes)
                  ((12, 9, 21), 3, 6, 2, 130, 79), ((9, 13, 19), 2, 6, 2, 140, 80),
                  # 125 nodes: member rows of odd length (every other one starts off a 16-byte boundary)
                  ((9, 9, 9), 3, 6, 2, 9, 81)]


@pytest.mark.parametrize("shape,r,n_sub,B,n_ens,seed", ENSEMBLE_CASES)
def test_ensemble_product_matches_oracle(shape, r, n_sub, B, n_ens, seed):
    """Every member's product within the FP32 accumulation bound of the
    oracle's exact products of the same FP16 operands (dyadic geometry: P is
    the same number on both sides before its FP16 rounding)."""
    d = synth.random_small(shape, 2, r=r, n_sub=n_sub, seed=seed, dt=0.125)
    p = oracle.Problem.from_domain(d)
    P = coarse.coarse_matrix(p, B)
    cg = fd.Coarse(_dev_domain(d), B, fd.FP16_BANK)
    C = _ensemble_fields(n_ens, cg.n_nodes, seed)
    print(f"[ensemble] shape={shape} r={r} B={B} K={cg.K} n_ens={n_ens}", flush=True)
    got = to_host(cg.apply_ensemble(to_dev(C)))
    ref, bnd = coarse.ensemble_product(P, C)
    ratio = np.max(np.abs(got - ref) / (bnd + 1e-300))
    print(f"[ensemble] max |gpu - oracle| / bound = {ratio:.3f}", flush=True)
    assert np.all(np.abs(got - ref) <= bnd)
    cg.close()


def test_ensemble_input_off_16_byte_boundary():
    """Member fields that start 8 bytes past a 16-byte boundary (a view one
    double into its allocation) give the same products bitwise."""
    d = synth.random_small((9, 9, 9), 2, r=3, n_sub=6, seed=82, dt=0.125)
    cg = fd.Coarse(_dev_domain(d), 2, fd.FP16_BANK)
    C = _ensemble_fields(6, cg.n_nodes, 82)
    whole = to_dev(np.concatenate([[7.0], C.ravel()]))
    view = whole[1:].view(C.shape)
    assert view.data_ptr() % 16 == 8
    a = to_host(cg.apply_ensemble(view))
    b = to_host(cg.apply_ensemble(to_dev(C)))
    assert np.array_equal(a, b)
    cg.close()


def test_ensemble_second_call_with_fewer_members():
    """Grids kept from a larger call do not leak into a smaller one; the
    same members give the same results bitwise."""
    d = synth.random_small((11, 10, 12), 2, r=3, n_sub=6, seed=75, dt=0.125)
    p = oracle.Problem.from_domain(d)
    P = coarse.coarse_matrix(p, 2)
    cg = fd.Coarse(_dev_domain(d), 2, fd.FP16_BANK)
    C = _ensemble_fields(40, cg.n_nodes, 75)
    big = to_host(cg.apply_ensemble(to_dev(C)))
    small = to_host(cg.apply_ensemble(to_dev(C[3:10].copy())))
    assert np.array_equal(small, big[3:10])
    ref, bnd = coarse.ensemble_product(P, C[3:10])
    assert np.all(np.abs(small - ref) <= bnd)
    cg.close()


def test_ensemble_grf_blocks_of_five():
    """The benchmark's coarse shape (r = 8, 5^3 blocks, K = 2) on a 40^3 GRF
    geometry: each member's product within the bound of the oracle's terms
    formed from the library's own FP16 P (the oracle's P differs from it by
    FP32 kernel rounding on this non-dyadic geometry), and members equal to
    single-member calls bitwise."""
    d = synth.config2(seed=76, n=40)
    cg = fd.Coarse(_dev_domain(d), 5, fd.FP16_BANK)
    Pm = cg.matrix()                                    # [o, I], the stored FP16 values widened
    K, kw = cg.K, 2 * cg.K + 1
    ncz, ncy, ncx = cg.coarse_shape
    n = cg.n_nodes
    P = np.zeros((n, n))
    for I in range(n):
        bz, rem = divmod(I, ncy * ncx)
        by, bx = divmod(rem, ncx)
        for o in range(kw ** 3):
            oz, rem2 = divmod(o, kw * kw)
            oy, ox = divmod(rem2, kw)
            jz, jy, jx = bz - (oz - K), by - (oy - K), bx - (ox - K)
            if 0 <= jz < ncz and 0 <= jy < ncy and 0 <= jx < ncx:
                P[I, (jz * ncy + jy) * ncx + jx] = Pm[o, I]
    C = _ensemble_fields(24, n, 76)
    got = to_host(cg.apply_ensemble(to_dev(C)))
    ref, bnd = coarse.ensemble_product(P, C)
    assert np.all(np.abs(got - ref) <= bnd)
    one = to_host(cg.apply_ensemble(to_dev(C[5:6].copy())))
    assert np.array_equal(one[0], got[5])
    cg.close()


def test_ensemble_rejections():
    d = synth.random_small((8, 8, 8), 2, r=3, n_sub=4, seed=77)
    dom = _dev_domain(d)
    c32 = fd.Coarse(dom, 2, fd.FP32)
    C = to_dev(np.ones((2, c32.n_nodes)))
    with pytest.raises(fd.FdirwError) as e:
        c32.apply_ensemble(C)
    assert e.value.status == fd.E_ARG
    c32.close()
    c16 = fd.Coarse(dom, 2, fd.FP16_BANK)
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_coarse_apply_ensemble(c16.handle, C, C, 2)            # in place
    assert e.value.status == fd.E_ARG
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_coarse_apply_ensemble(c16.handle, C, torch.empty_like(C), 0)
    assert e.value.status == fd.E_ARG
    c16.close()
    k5 = fd.Coarse(_dev_domain(synth.random_small((7, 7, 7), 2, r=5, n_sub=4, seed=78)), 1, fd.FP16_BANK)
    with pytest.raises(fd.FdirwError) as e:
        k5.apply_ensemble(to_dev(np.ones((1, k5.n_nodes))))
    assert e.value.status == fd.E_UNSUPPORTED
    k5.close()


def test_ensemble_forms_agree_bitwise():
    """128 members go through the plane-walking form, 16 through the
    per-tile form: the same fragments summed in the same order, so the
    members they share agree bitwise."""
    d = synth.random_small((15, 14, 19), 2, r=3, n_sub=6, seed=81, dt=0.125)
    cg = fd.Coarse(_dev_domain(d), 2, fd.FP16_BANK)
    C = _ensemble_fields(128, cg.n_nodes, 81)
    many = to_host(cg.apply_ensemble(to_dev(C)))
    few = to_host(cg.apply_ensemble(to_dev(C[:16].copy())))
    assert np.array_equal(few, many[:16])
    cg.close()


def test_ensemble_without_diffusion_is_the_identity_band():
    """r = 0 (K = 0): P is diagonal (every group keeps its mass), so each
    member's product is the member itself in the mixed precision: the
    FP32-then-FP16 rounding of its scaled values, bitwise."""
    d = synth.random_small((9, 10, 11), 2, r=0, n_sub=3, seed=82, dt=0.125)
    p = oracle.Problem.from_domain(d)
    P = coarse.coarse_matrix(p, 2)
    cg = fd.Coarse(_dev_domain(d), 2, fd.FP16_BANK)
    assert cg.K == 0
    C = _ensemble_fields(20, cg.n_nodes, 82)
    got = to_host(cg.apply_ensemble(to_dev(C)))
    ref, bnd = coarse.ensemble_product(P, C)
    assert np.array_equal(got, ref)
    cg.close()


def test_ensemble_member_count_limit():
    d = synth.random_small((6, 6, 6), 2, r=2, n_sub=3, seed=83)
    cg = fd.Coarse(_dev_domain(d), 2, fd.FP16_BANK)
    C = torch.zeros((4097, cg.n_nodes), dtype=torch.float64, device="cuda")
    with pytest.raises(fd.FdirwError) as e:
        fd.fdirw_coarse_apply_ensemble(cg.handle, C, torch.empty_like(C), 4097)
    assert e.value.status == fd.E_ARG
    cg.close()
