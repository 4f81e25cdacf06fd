"""Pins of the coarse-mesh oracle (Sec. 3.1, Eqs. 10-15) against results that
it does not compute itself: the fine oracle step (B = 1), the whole-domain
average (one block), dense powers of the whole-domain operator aggregated by
blocks, and mass conservation.  CPU only."""
import numpy as np
import pytest

import oracle
import synth
from closed_forms import dense_operator
from oracle import coarse


def _problem(d):
    return oracle.Problem(d.label, d.d_phase, d.r, d.n_sub, d.h, d.dt)


@pytest.mark.parametrize("shape,r,n_sub,seed", [((6, 7, 5), 2, 6, 1), ((4, 5, 9), 1, 3, 2)])
def test_block_one_is_the_fine_step(shape, r, n_sub, seed):
    d = synth.random_small(shape, 3, r=r, n_sub=n_sub, seed=seed)
    p = _problem(d)
    P = coarse.coarse_matrix(p, 1)
    got = coarse.step(p, P, d.c0, 1)
    ref, _, _ = p.step(d.c0)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.abs(ref).max()


def test_one_block_is_the_domain_average():
    d = synth.random_small((5, 4, 6), 2, r=2, n_sub=5, seed=3, d_zero_phase=False)
    p = _problem(d)
    P = coarse.coarse_matrix(p, 8)
    assert P.shape == (1, 1)
    assert abs(P[0, 0] - 1.0) <= 1e-13
    got = coarse.step(p, P, d.c0, 8)
    assert np.max(np.abs(got - d.c0.mean())) <= 1e-13


@pytest.mark.parametrize("B", [2, 3])
def test_matrix_equals_aggregated_whole_domain_operator(B):
    # windows larger than the domain: every fine kernel is a column of the
    # n-th power of the whole-domain one-sub-step operator, so
    # S = A M^n A^T with A the block membership of the mobile cells
    d = synth.random_small((3, 4, 5), 3, r=5, n_sub=4, seed=4)
    p = _problem(d)
    M = np.linalg.matrix_power(dense_operator(d.label, d.d_phase, p.dt, p.h), d.n_sub)
    block, mobile, count = coarse.groups(d.label, d.d_phase, B)
    A = np.zeros((count.size, d.label.size))
    A[block.ravel()[mobile.ravel()], np.flatnonzero(mobile.ravel())] = 1.0
    S = A @ M @ A.T
    ref = np.zeros_like(S)
    ref[count > 0] = S[count > 0] / count[count > 0, None]
    got = coarse.coarse_matrix(p, B)
    assert np.max(np.abs(got - ref)) <= 1e-13


@pytest.mark.parametrize("B", [2, 3, 5])
def test_mass_conserved_and_immobile_cells_kept(B):
    d = synth.random_small((7, 6, 8), 3, r=2, n_sub=8, seed=5)
    p = _problem(d)
    P = coarse.coarse_matrix(p, B)
    _, mobile, count = coarse.groups(d.label, d.d_phase, B)
    # column sums of the mass form N_I P[I, J] / N_J are one
    has = count > 0
    colsum = (count[:, None] * P)[:, has].sum(axis=0) / count[has]
    assert np.max(np.abs(colsum - 1.0)) <= 1e-13
    got = coarse.step(p, P, d.c0, B)
    assert abs(got.sum() - d.c0.sum()) <= 1e-12 * d.c0.sum()
    assert np.array_equal(got[~mobile], d.c0[~mobile])
    # remapping makes every group uniform
    block, _, _ = coarse.groups(d.label, d.d_phase, B)
    for I in np.flatnonzero(has)[:10]:
        vals = got[mobile & (block == I)]
        assert np.all(vals == vals[0])


def test_liquid_only_grouping_conserves_mass():
    # only phase 0 grouped: the kernels are renormalised over the grouped
    # cells, the other phases keep their values, mass is conserved
    d = synth.random_small((8, 7, 9), 3, r=2, n_sub=10, seed=6, d_zero_phase=False)
    p = _problem(d)
    grouped = [1, 0, 0]
    P = coarse.coarse_matrix(p, 3, grouped)
    block, mobile, count = coarse.groups(d.label, d.d_phase, 3, grouped)
    assert np.array_equal(mobile, d.label == 0)
    has = count > 0
    colsum = (count[:, None] * P)[:, has].sum(axis=0) / count[has]
    assert np.max(np.abs(colsum - 1.0)) <= 1e-13
    got = coarse.step(p, P, d.c0, 3, grouped)
    assert np.array_equal(got[~mobile], d.c0[~mobile])
    assert abs(got[mobile].sum() - d.c0[mobile].sum()) <= 1e-12 * d.c0.sum()
    # the default grouping of this domain (every D > 0) is every cell
    _, all_mobile, _ = coarse.groups(d.label, d.d_phase, 3)
    assert all_mobile.all()


# ------------------------------------------------------------------ far field

def test_far_field_two_cell_closed_form():
    # one liquid cell next to one reservoir cell (same D): the kernel decays
    # as (1 - lam)^n and the unit-boundary response is 1 - (1 - lam)^n
    label = np.array([[[0, 1]]], dtype=np.uint8)
    p = oracle.Problem(label, np.array([1.0, 1.0]), 1, 7, 1.0, 0.15)
    res = [0, 1]
    P = coarse.coarse_matrix(p, 1, reservoir=res)
    pbc = coarse.p_bc(p, 1, reservoir=res)
    q = (1.0 - 0.15) ** 7
    assert abs(P[0, 0] - q) <= 1e-15
    assert abs(pbc[0] - (1.0 - q)) <= 1e-15
    assert P[1, 1] == 0.0 and pbc[1] == 0.0          # the reservoir block has no node


def _far_field_domain(seed):
    # x walls of reservoir phase 2; liquid 0 and a slow phase 1 inside
    d = synth.random_small((5, 6, 7), 2, r=8, n_sub=9, seed=seed, d_zero_phase=False)
    label = d.label.copy()
    label[:, :, 0] = 2
    label[:, :, -1] = 2
    return label, np.array([1.0, 0.05, 1.0]), d.c0


def test_far_field_uniform_state_is_stationary():
    label, dph, _ = _far_field_domain(7)
    p = oracle.Problem(label, dph, 8, 9, 1.0, 0.0)
    res = [0, 0, 1]
    for B in (1, 3):
        P = coarse.coarse_matrix(p, B, reservoir=res)
        pbc = coarse.p_bc(p, B, reservoir=res)
        near = ~coarse.reservoir_mask(label, res)
        v_ff = 40.0
        c = np.ones(label.shape)
        out, c_ff = coarse.step_far_field(p, P, pbc, c, 1.0, near.sum() + v_ff, v_ff, B, reservoir=res)
        assert np.max(np.abs(out - 1.0)) <= 1e-13
        assert abs(c_ff - 1.0) <= 1e-13


def test_far_field_block_one_is_the_dirichlet_fd():
    # windows covering the domain: Eq. 8 with P_BC equals the whole-domain FD
    # with the reservoir cells held at c_ff, and Eq. 7 conserves the total
    label, dph, c0 = _far_field_domain(8)
    p = oracle.Problem(label, dph, 8, 9, 1.0, 0.0)
    res = [0, 0, 1]
    fixed = coarse.reservoir_mask(label, res)
    P = coarse.coarse_matrix(p, 1, reservoir=res)
    pbc = coarse.p_bc(p, 1, reservoir=res)
    c_ff, v_ff = 0.3, 25.0
    c = np.where(fixed, c_ff, c0)
    m_total = c[~fixed].sum() + c_ff * v_ff
    out, c_ff_new = coarse.step_far_field(p, P, pbc, c, c_ff, m_total, v_ff, 1, reservoir=res)
    ref = p.global_fd(c, fixed=fixed, fval=c_ff)
    assert np.max(np.abs(out[~fixed] - ref[~fixed])) <= 1e-13
    assert np.all(out[fixed] == c_ff_new)
    assert abs(out[~fixed].sum() + c_ff_new * v_ff - m_total) <= 1e-12 * m_total


def test_node_windows_with_block_one_are_the_source_windows():
    # B = 1: the window of node J is the point-source window of radius r, so
    # both constructions give the same P (r = 10 > 8: windows shorter than the
    # domain along z)
    d = synth.random_small((24, 4, 5), 3, r=10, n_sub=7, seed=41)
    p = _problem(d)
    got = coarse.coarse_matrix_node_windows(p, 1)
    want = coarse.coarse_matrix_source_windows(p, 1)
    assert np.max(np.abs(got - want)) <= 1e-13
    assert np.max(np.abs(coarse.coarse_matrix(p, 1) - got)) == 0.0    # r > 8 takes the node windows


@pytest.mark.parametrize("B", [2, 3])
def test_node_windows_covering_equal_aggregated_operator(B):
    # windows larger than the domain: the node column is A M^n of the
    # indicator of group J, so S = A M^n A^T as for the source windows
    d = synth.random_small((3, 4, 5), 3, r=9, n_sub=4, seed=42)
    p = _problem(d)
    M = np.linalg.matrix_power(dense_operator(d.label, d.d_phase, p.dt, p.h), d.n_sub)
    block, mobile, count = coarse.groups(d.label, d.d_phase, B)
    A = np.zeros((count.size, d.label.size))
    A[block.ravel()[mobile.ravel()], np.flatnonzero(mobile.ravel())] = 1.0
    S = A @ M @ A.T
    ref = np.zeros_like(S)
    ref[count > 0] = S[count > 0] / count[count > 0, None]
    assert np.max(np.abs(coarse.coarse_matrix_node_windows(p, B) - ref)) <= 1e-13


def test_node_windows_far_field_covering_equal_source_windows():
    # with absorbing far-field cells and covering windows both constructions
    # are sums of the same absorbed kernels
    d = synth.random_small((6, 5, 7), 3, r=9, n_sub=5, seed=43)
    label = d.label.copy()
    label[:, :, 0] = 2
    dph = np.array([1.0, 0.3, 1.0])
    p = oracle.Problem(label, dph, 9, 5, 1.0, 0.1)
    res = [0, 0, 1]
    got = coarse.coarse_matrix_node_windows(p, 2, reservoir=res)
    want = coarse.coarse_matrix_source_windows(p, 2, reservoir=res)
    assert np.max(np.abs(got - want)) <= 1e-13
    # mass only leaves, through the far field: N_I P[I, J] summed over I is at
    # most N_J, and below it for groups next to the far-field cells
    _, _, count = coarse.groups(label, dph, 2, reservoir=res)
    has = count > 0
    out = (count[:, None] * got).sum(axis=0)[has] / count[has]
    assert np.all(out <= 1.0 + 1e-13) and np.any(out < 0.999)


# ---------------------------------------------------------------- reduced-precision arithmetic (Sec. 3.3, Table 2)

def test_arith_fp64_is_the_plain_product():
    rng = np.random.default_rng(3)
    P = rng.random((30, 40))
    C = rng.random(40)
    out, bnd = coarse.arith_product(P, C, "fp64")
    assert np.max(np.abs(out - P @ C)) <= 1e-14 * np.abs(P @ C).max()
    assert np.all(bnd < 1e-12 * np.abs(P @ C))


def test_arith_exactly_representable_operands_agree():
    # P entries k / 64 and C small integers: every product is a multiple of
    # 1/64 below 16 (exact in FP16) and every row sum is exact in FP32, so the
    # fp32 and mixed steps equal fp64 exactly; FP16 accumulation does not
    rng = np.random.default_rng(4)
    P = rng.integers(0, 65, (25, 125)) / 64.0
    C = rng.integers(0, 17, 125).astype(np.float64)
    ref, _ = coarse.arith_product(P, C, "fp64")
    for a in ("fp32", "mixed"):
        out, _ = coarse.arith_product(P, C, a)
        assert np.array_equal(out, ref), a
    out16, bnd16 = coarse.arith_product(P, C, "fp16")
    assert not np.array_equal(out16, ref)
    assert np.all(np.abs(out16 - ref) <= bnd16)


def test_arith_mixed_rounds_each_product_to_fp16():
    # 1/3 rounds to 0.333251953125 in FP16; times 3 that is 1 - 2^-12, exactly
    # half way between the FP16 neighbours 1 - 2^-11 and 1: round to even -> 1
    out, _ = coarse.arith_product(np.array([[1.0 / 3.0]]), np.array([3.0]), "mixed")
    assert out[0] == 1.0
    out, _ = coarse.arith_product(np.array([[1.0 / 3.0]]), np.array([3.0]), "fp32")
    assert out[0] == np.float64(np.float32(1.0 / 3.0)) * 3.0 != 1.0


def test_arith_fp16_accumulation_stalls():
    # Sec. 3.3: adding small terms to a large sum needs digits FP16 lacks:
    # 4096 unit terms accumulate to 2048 in FP16 (2048 + 1 rounds back to
    # 2048) and to 4096 with FP32 accumulation
    P = np.ones((1, 4096))
    C = np.ones(4096)
    assert coarse.arith_product(P, C, "fp16")[0][0] == 2048.0
    assert coarse.arith_product(P, C, "mixed")[0][0] == 4096.0


@pytest.mark.parametrize("arith", ["fp32", "mixed"])
def test_arith_bound_covers_other_orders(arith):
    # the per-node bound holds for FP32 accumulation in another order
    # (reversed, sequential FP32 additions of the same terms)
    rng = np.random.default_rng(5)
    P = rng.random((50, 125)) * 10.0 ** rng.integers(-6, 0, (50, 125))
    C = rng.random(125)
    out, bnd = coarse.arith_product(P, C, arith)
    t = coarse.arith_terms(P, C, arith).astype(np.float32)
    acc = np.zeros(50, dtype=np.float32)
    for j in range(124, -1, -1):
        acc = (acc + t[:, j]).astype(np.float32)
    assert np.all(np.abs(acc.astype(np.float64) - out) <= bnd)


def test_arith_step_on_a_grid_conserves_mass_to_the_precision():
    d = synth.random_small((10, 10, 10), 2, r=3, n_sub=20, seed=7)
    p = oracle.Problem.from_domain(d)
    P = coarse.coarse_matrix(p, 5)
    ref = coarse.step(p, P, d.c0, 5)
    for a, tol in (("fp64", 1e-14), ("fp32", 1e-6), ("mixed", 2e-3), ("fp16", 5e-2)):
        out, bnd = coarse.step_arith(p, P, d.c0, 5, a)
        assert abs(out.sum() - ref.sum()) <= tol * ref.sum(), a


# ---------------------------------------------------------------- ensemble product (Eq. 14, several right-hand sides)

def test_ensemble_representable_operands_are_exact():
    # P entries k / 64 and C small integers are FP16 numbers, every product
    # and every row sum is exact: the ensemble product is the plain product
    rng = np.random.default_rng(11)
    P = rng.integers(0, 65, (20, 125)) / 64.0
    C = rng.integers(0, 33, (6, 125)).astype(np.float64)
    out, bnd = coarse.ensemble_product(P, C)
    assert np.array_equal(out, C @ P.T)
    assert np.all(bnd >= 0.0)


def test_ensemble_rounds_c_through_fp32():
    # 1 + 2^-11 + 2^-40 is 1 + 2^-11 in FP32, exactly half way between the
    # FP16 neighbours 1 and 1 + 2^-10: round to even gives 1 (rounded
    # directly to FP16 it would be 1 + 2^-10)
    c = 1.0 + 2.0 ** -11 + 2.0 ** -40
    assert np.float64(np.float16(c)) == 1.0 + 2.0 ** -10
    out, _ = coarse.ensemble_product(np.array([[1.0]]), np.array([[c]]))
    assert out[0, 0] == 1.0


def test_ensemble_products_are_exact():
    # 1/3 in FP16 is 0.333251953125; times 3 that is 0.999755859375 = 1 - 2^-12,
    # kept as it is (the mixed VALU form rounds that product to 1)
    out, _ = coarse.ensemble_product(np.array([[1.0 / 3.0]]), np.array([[3.0]]))
    assert out[0, 0] == 1.0 - 2.0 ** -12
    assert coarse.arith_product(np.array([[1.0 / 3.0]]), np.array([3.0]), "mixed")[0][0] == 1.0


def test_ensemble_bound_covers_fp32_orders():
    # sequential FP32 sums of the exact products, in reverse and in a random
    # order, stay within the bound
    rng = np.random.default_rng(12)
    P = rng.random((40, 125)) * 10.0 ** rng.integers(-5, 0, (40, 125))
    C = rng.random((3, 125)) * 10.0 ** rng.integers(-2, 2, (3, 125))
    out, bnd = coarse.ensemble_product(P, C)
    Ps, Cs, sp, tc = coarse.ensemble_operands(P, C)
    for e in range(3):
        back = 2.0 ** -(sp + int(tc[e]))
        t = (Ps * Cs[e][None, :]).astype(np.float32)
        assert np.array_equal(t.astype(np.float64), Ps * Cs[e][None, :])       # products exact in FP32
        for order in (np.arange(124, -1, -1), rng.permutation(125)):
            acc = np.zeros(40, dtype=np.float32)
            for j in order:
                acc = (acc + t[:, j]).astype(np.float32)
            assert np.all(np.abs(acc.astype(np.float64) * back - out[e]) <= bnd[e])


def test_ensemble_members_are_independent():
    # each member's result is that member's product alone, in any order of
    # the members
    rng = np.random.default_rng(13)
    P = rng.random((15, 30))
    C = rng.random((5, 30))
    out, bnd = coarse.ensemble_product(P, C)
    perm = np.array([3, 0, 4, 1, 2])
    out_p, _ = coarse.ensemble_product(P, C[perm])
    assert np.array_equal(out_p, out[perm])
    one, _ = coarse.ensemble_product(P, C[2])
    assert np.array_equal(one[0], out[2])


def test_ensemble_power_of_two_scaling_is_exact():
    # a member scaled by 2^k (into what would be FP16's subnormal range or far
    # above its largest number) gives the same result scaled by 2^k, bitwise
    rng = np.random.default_rng(14)
    P = 0.01 + rng.random((30, 50)) * 0.3                   # FP16-normal, also times 8
    C = rng.random((2, 50))
    out, bnd = coarse.ensemble_product(P, C)
    for k in (-40, -20, 9, 30):
        o2, b2 = coarse.ensemble_product(P, C * 2.0 ** k)
        assert np.array_equal(o2, out * 2.0 ** k) and np.array_equal(b2, bnd * 2.0 ** k), k
    o3, _ = coarse.ensemble_product(P * 8.0, C)
    assert np.array_equal(o3, out * 8.0)


def test_ensemble_keeps_operands_normal():
    # largest |C| = 1 scales by 2^14: a value 2^-27 becomes 2^-13 (normal,
    # kept), 2^-29 becomes 2^-15 (below the smallest normal FP16, taken as 0)
    P = np.array([[0.5, 0.25, 0.125]])
    kept, _ = coarse.ensemble_product(P, np.array([[1.0, 2.0 ** -27, 0.0]]))
    assert kept[0, 0] == 0.5 + 0.25 * 2.0 ** -27
    gone, _ = coarse.ensemble_product(P, np.array([[1.0, 2.0 ** -29, 0.0]]))
    assert gone[0, 0] == 0.5
    assert coarse.pow2_scale(1.0) == 14 and coarse.pow2_scale(2.0 ** 15 - 1) == 0 and coarse.pow2_scale(0.0) == 0
