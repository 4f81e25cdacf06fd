"""FP64 CPU oracle of the coarse-mesh FDiRW step (arXiv 2408.11376, Sec. 3.1,
Eqs. 10-15), test infrastructure only: the tests and the benchmark's CPU leg
may use it, the product library never does.

Definition (built on the fine oracle's window kernels, ``Problem.kernels``):

Nodes.  The grid is cut into blocks of B x B x B cells (ragged at the far
edges).  A cell is grouped if its phase is one of the fast (liquid) phases:
by default every phase with D > 0, or the phases the caller flags.  The
grouped cells of block I form group I with N_I cells and the representative
node I (blocks without a grouped cell have no node).  Other cells take no part
and keep their value (the paper maps only the liquid nodes; the solid phase
and the liquid-solid exchange belong to other parts of its solver).

P (Eq. 10, coarse counterpart of p, Eq. 9).  The mass of group J, spread
uniformly over its cells, moves in one big step as the sum of the fine kernels
of its cells; the share that lands in group I, as a concentration ratio, is
    S[I, J] = sum over grouped j in J, cells i in I of G_j(i) / m_j
    P[I, J] = S[I, J] / N_I
(G_j the fine kernel of source j, m_j its mass over the grouped cells;
normalising every kernel that way makes the columns of N_I P[I, J] / N_J sum
to one, so the coarse step conserves mass exactly.  With the default grouping
m_j is the whole kernel mass, since cells with D = 0 never receive any).

Step (Eqs. 13-15):
    mapping     C_J = mean of c over the cells of group J               (Eq. 13)
    FDiRW       C'_I = sum_J P[I, J] C_J                                 (Eq. 14)
    remapping   c'(i) = C'_I for every cell i of group I; c'(i) = c(i)  (Eq. 15)
                for the cells outside every group

Node windows (radius r > 8).  The per-source windows stop at r = 8; beyond
it the column of group J is the FD of unit mass on all of J's grouped cells at
once, on the window made of J's block and K = ceil(r / B) blocks around it
(coarse_matrix_node_windows).  With B = 1 that is the per-source window of
radius r.

Without a far field the term P_BC c_far-field of Eq. 14 is zero (no-flux
domain walls, as in the fine step).  With B = 1 every group is one cell and the
step is the fine step with renormalised kernels.

Far field (Eqs. 7, 8, 10, 14).  Cells of the reservoir phases are the
far-field boundary: Dirichlet cells that hold the uniform far-field
concentration c_ff.  Then
    G_j          the window kernel with the reservoir cells held at 0 (they
                 absorb), not renormalised: the mass it loses is what leaves
                 for the far field
    S, P         as above from these kernels (over the grouped cells)
    p_bc(i)      the whole-domain FD of n sub-steps from 0 with the reservoir
                 cells held at 1 (the response to a unit boundary
                 concentration); P_BC[I] = mean of p_bc over group I
    step         C' = P C + P_BC c_ff, remapping as above, and then Eq. 7:
                 c_ff' = (M_total - sum of c' over the non-reservoir cells)
                 / V_ff, written into the reservoir cells.
"""
from __future__ import annotations

import numpy as np

from . import Problem


def coarse_dims(shape, B: int):
    nz, ny, nx = shape
    return ((nz + B - 1) // B, (ny + B - 1) // B, (nx + B - 1) // B)


def groups(label, d_phase, B: int, grouped=None, reservoir=None):
    """(block index of every cell [nz, ny, nx] int64, grouped-cell mask, N per
    node [n_nodes]) with nodes numbered (bz * ncy + by) * ncx + bx.
    grouped: per-phase flags of the fast phases, or None for D > 0;
    reservoir: per-phase flags of the far-field boundary (never grouped)."""
    label = np.asarray(label)
    d_phase = np.asarray(d_phase, dtype=np.float64)
    nz, ny, nx = label.shape
    ncz, ncy, ncx = coarse_dims(label.shape, B)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    block = ((z // B) * ncy + (y // B)) * ncx + (x // B)
    flags = d_phase > 0 if grouped is None else np.asarray(grouped, dtype=bool)
    if reservoir is not None:
        flags = flags & ~np.asarray(reservoir, dtype=bool)
    mobile = flags[label]
    count = np.bincount(block[mobile].ravel(), minlength=ncz * ncy * ncx).astype(np.float64)
    return block, mobile, count


def reservoir_mask(label, reservoir):
    return np.asarray(reservoir, dtype=bool)[np.asarray(label)]


# Largest window radius of the per-source kernels; beyond it P comes from node
# windows (coarse_matrix_node_windows).
MAX_SOURCE_WINDOW_RADIUS = 8


def coarse_matrix(problem, B: int, grouped=None, reservoir=None) -> np.ndarray:
    """Dense P [n_nodes, n_nodes] (rows = destination I, columns = source J):
    from the per-source window kernels for r <= 8, from node windows beyond."""
    if problem.r > MAX_SOURCE_WINDOW_RADIUS:
        return coarse_matrix_node_windows(problem, B, grouped, reservoir)
    return coarse_matrix_source_windows(problem, B, grouped, reservoir)


def coarse_matrix_node_windows(problem, B: int, grouped=None, reservoir=None) -> np.ndarray:
    """P from node windows: the column of group J is one whole-window FD of
    unit mass on every grouped cell of J, on the window made of J's block and
    the K = ceil(r / B) blocks around it on every side (clipped at the domain;
    its faces are walls), binned over the groups it reaches.  Without a far
    field the column is scaled to N_J over the grouped cells (the sum of N_J
    unit kernels renormalised over the grouped cells); with one, the far-field
    cells absorb (held at 0) and nothing is rescaled.  By linearity the column
    is the sum of the point-source kernels of J's cells on that shared window."""
    label = problem.label
    block, mobile, count = groups(label, problem.d_phase, B, grouped, reservoir)
    S = np.zeros((count.size, count.size))
    for J in np.flatnonzero(count > 0):
        S[:, J] = node_window_column(problem, B, int(J), grouped, reservoir)
    P = np.zeros_like(S)
    has = count > 0
    P[has] = S[has] / count[has, None]
    return P


def node_window_column(problem, B: int, J: int, grouped=None, reservoir=None) -> np.ndarray:
    """Column J of S (before the division by N_I) from the node window of
    group J: dense over the n_nodes destinations."""
    label = problem.label
    block, mobile, count = groups(label, problem.d_phase, B, grouped, reservoir)
    nz, ny, nx = label.shape
    ncz, ncy, ncx = coarse_dims(label.shape, B)
    K = -(-problem.r // B)
    fixed = None if reservoir is None else reservoir_mask(label, reservoir)
    bz, rem = divmod(int(J), ncy * ncx)
    by, bx = divmod(rem, ncx)
    win = (slice(max(0, (bz - K) * B), min(nz, (bz + K + 1) * B)),
           slice(max(0, (by - K) * B), min(ny, (by + K + 1) * B)),
           slice(max(0, (bx - K) * B), min(nx, (bx + K + 1) * B)))
    sub = Problem(label[win], problem.d_phase, 0, problem.n_sub, problem.h, problem.dt)
    keep = mobile[win]
    c = ((block[win] == J) & keep).astype(np.float64)
    G = sub.global_fd(c, fixed=None if fixed is None else fixed[win], fval=0.0)
    g = G[keep]
    if fixed is None:
        g = g * (count[J] / g.sum())
    col = np.zeros(count.size)
    np.add.at(col, block[win][keep], g)
    return col


def coarse_matrix_source_windows(problem, B: int, grouped=None, reservoir=None) -> np.ndarray:
    """P from the per-source window kernels of every grouped cell."""
    label = problem.label
    block, mobile, count = groups(label, problem.d_phase, B, grouped, reservoir)
    n_nodes = count.size
    shape = label.shape
    nz, ny, nx = shape
    r, W = problem.r, problem.W
    S = np.zeros((n_nodes, n_nodes))
    src = np.flatnonzero(mobile.ravel())
    fixed = None if reservoir is None else reservoir_mask(label, reservoir)
    G, mass = problem.kernels(src, fixed)
    rel = np.arange(W) - r
    for q, s in enumerate(src):
        sz, sy, sx = np.unravel_index(s, shape)
        Z, Y, X = sz + rel, sy + rel, sx + rel
        kz, ky, kx = (Z >= 0) & (Z < nz), (Y >= 0) & (Y < ny), (X >= 0) & (X < nx)
        inside = np.ix_(Z[kz], Y[ky], X[kx])
        keep = mobile[inside]
        g = G[q][np.ix_(kz, ky, kx)][keep]
        np.add.at(S[:, block.flat[s]], block[inside][keep], g / g.sum() if fixed is None else g)
    P = np.zeros_like(S)
    has = count > 0
    P[has] = S[has] / count[has, None]
    return P


def mapping(c, label, d_phase, B: int, grouped=None, reservoir=None) -> np.ndarray:
    """Eq. 13: the mean of c over each group (0 for blocks without a node)."""
    block, mobile, count = groups(label, d_phase, B, grouped, reservoir)
    tot = np.bincount(block[mobile].ravel(), weights=np.asarray(c)[mobile].ravel(), minlength=count.size)
    C = np.zeros_like(tot)
    C[count > 0] = tot[count > 0] / count[count > 0]
    return C


def remapping(C, c_old, label, d_phase, B: int, grouped=None, reservoir=None) -> np.ndarray:
    """Eq. 15: every grouped cell takes its node's value; other cells keep c_old."""
    block, mobile, _ = groups(label, d_phase, B, grouped, reservoir)
    out = np.array(c_old, dtype=np.float64, copy=True)
    out[mobile] = np.asarray(C)[block[mobile]]
    return out


def step(problem, P, c, B: int, grouped=None) -> np.ndarray:
    """One coarse big step (Eqs. 13-15) with the matrix from coarse_matrix."""
    C = mapping(c, problem.label, problem.d_phase, B, grouped)
    return remapping(P @ C, c, problem.label, problem.d_phase, B, grouped)


def p_bc(problem, B: int, grouped=None, reservoir=None) -> np.ndarray:
    """P_BC [n_nodes]: group means of the whole-domain response to a unit
    concentration held on the reservoir cells (0 elsewhere at the start)."""
    fixed = reservoir_mask(problem.label, reservoir)
    field = problem.global_fd(np.zeros(problem.label.shape), fixed=fixed, fval=1.0)
    return mapping(field, problem.label, problem.d_phase, B, grouped, reservoir)


def step_far_field(problem, P, pbc, c, c_ff: float, m_total: float, v_ff: float, B: int, grouped=None,
                   reservoir=None):
    """One coarse big step with the far field (Eqs. 14, 15, 7); returns
    (c_new, c_ff_new)."""
    C = mapping(c, problem.label, problem.d_phase, B, grouped, reservoir)
    out = remapping(P @ C + pbc * c_ff, c, problem.label, problem.d_phase, B, grouped, reservoir)
    res = reservoir_mask(problem.label, reservoir)
    out[res] = 0.0
    c_ff_new = (m_total - out.sum()) / v_ff
    out[res] = c_ff_new
    return out, c_ff_new


# --------------------------------------------------------------------------
# Reduced-precision arithmetic of the coarse step (Sec. 3.3, Fig. 3, Table 2).
#
# The paper compares four precisions of the FDiRW superposition:
#   fp64   P, C, products and sums in FP64
#   fp32   P and C in FP32, products and sums in FP32
#   mixed  (its FP32/FP16 scheme) C computed in FP32 and converted to FP16,
#          P stored in FP16, each product P[I, J] C_J taken in FP16, the
#          products accumulated in FP32, the result widened for the remapping
#   fp16   as mixed, but the products also accumulated in FP16
# The far-field term P_BC c_ff is formed the same way as one more product.
# Reading: the mapping (Eq. 13) is the FP64 group mean rounded to the C
# precision (the paper maps in FP32; the mean is the same to FP32 rounding and
# the mapping is memory-bound either way).
#
# ARITH_TERMS gives the terms exactly as the precision forms them; the sum is
# then written out per node: for fp64 / fp32 / mixed the exact FP64 sum of the
# terms (any FP32 accumulation order differs from it by at most
# gamma_n(2^-24) times the sum of |terms|), for fp16 the sequential FP16 sum
# over J in increasing order (the paper's example of why FP16 accumulation
# fails: a large partial sum absorbs small terms).

ARITH = ("fp64", "fp32", "mixed", "fp16")
UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "mixed": 2.0 ** -24, "fp16": 2.0 ** -11}


def arith_operands(P, C, arith: str):
    """(P, C) rounded to the storage precision of ``arith``, as FP64 arrays
    (mixed / fp16: C through FP32, as the scheme forms it)."""
    P = np.asarray(P, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    if arith == "fp64":
        return P, C
    if arith == "fp32":
        return P.astype(np.float32).astype(np.float64), C.astype(np.float32).astype(np.float64)
    if arith in ("mixed", "fp16"):
        # C is formed in FP32 and then converted to FP16 (Sec. 3.3); P is
        # stored in FP16 from its FP64 values
        return P.astype(np.float16).astype(np.float64), C.astype(np.float32).astype(np.float16).astype(np.float64)
    raise ValueError(f"unknown arithmetic {arith!r}")


def arith_terms(P, C, arith: str) -> np.ndarray:
    """terms[I, J] = the product P[I, J] C_J as the precision forms it: exact
    for fp64 / fp32 (a product of two FP32 numbers is exact in FP64; FP32
    accumulates it with a fused multiply-add), rounded to FP16 for mixed and
    fp16 (an FP16 multiply of the FP16 operands)."""
    Pr, Cr = arith_operands(P, C, arith)
    t = Pr * Cr[None, :]
    if arith in ("mixed", "fp16"):
        t = (Pr.astype(np.float16) * Cr.astype(np.float16)[None, :]).astype(np.float64)
    return t


def arith_sum(terms: np.ndarray, arith: str) -> np.ndarray:
    """Row sums of ``terms`` in the accumulation precision (see above)."""
    terms = np.asarray(terms, dtype=np.float64)
    if arith != "fp16":
        return terms.sum(axis=1)
    out = np.zeros(terms.shape[0], dtype=np.float16)
    t16 = terms.astype(np.float16)
    for j in range(terms.shape[1]):
        out = (out + t16[:, j]).astype(np.float16)
    return out.astype(np.float64)


def arith_product(P, C, arith: str, pbc=None, c_ff: float = 0.0):
    """(C', bound): Eq. 14 in the precision ``arith`` and, per node, the
    bound gamma_n(u) * sum |terms| (n = number of nonzero terms + 1) within
    which any summation order of the same terms agrees with C'."""
    t = arith_terms(P, C, arith)
    if pbc is not None:
        t = np.concatenate([t, arith_terms(np.asarray(pbc, dtype=np.float64)[:, None], np.array([c_ff]), arith)],
                           axis=1)
    out = arith_sum(t, arith)
    n = (t != 0).sum(axis=1) + 1
    u = UNIT_ROUNDOFF[arith]
    nu = n * u
    gam = np.where(nu < 1.0, nu / np.maximum(1.0 - nu, 1e-300), np.inf)
    return out, gam * np.abs(t).sum(axis=1)


def step_arith(problem, P, c, B: int, arith: str, grouped=None):
    """One coarse big step (Eqs. 13-15) in the precision ``arith``; returns
    (c_new, per-cell bound of the accumulation order, 0 outside the groups)."""
    C = mapping(c, problem.label, problem.d_phase, B, grouped)
    Cn, bnd = arith_product(P, C, arith)
    out = remapping(Cn, c, problem.label, problem.d_phase, B, grouped)
    bcell = remapping(bnd, np.zeros_like(np.asarray(c, dtype=np.float64)), problem.label, problem.d_phase, B,
                      grouped)
    return out, bcell


# --------------------------------------------------------------------------
# Ensemble product (Eq. 14 with several right-hand sides, Sec. 3.3).
#
# With E coarse fields C_e over the same geometry the E products P C_e are one
# matrix product P [C_1 ... C_E], which the matrix cores take in the mixed
# FP32/FP16 precision: C_e computed in FP32 and converted to FP16, P stored in
# FP16, every product of two FP16 operands formed exactly (11 x 11 significant
# bits fit in FP32) and the products summed in FP32.
# Readings:
#   * FP16 operands are kept in the normal range: P (as stored in FP16) and
#     each member C_e are scaled by powers of two, 2^s and 2^t_e, that bring
#     their largest magnitude into [2^14, 2^15); operands still below the
#     smallest normal FP16 number (2^-14) after the scaling are taken as 0
#     (they are below 2^-28 of the largest one); the sums are scaled back by
#     2^-(s + t_e), exactly.  (A matrix unit may sum products of subnormal
#     operands less accurately than FP32; with the scaling none occur, and the
#     scaling changes no normal FP16 value's rounding.)
#   * The unit's order and rounding of the FP32 sum are not specified, so the
#     result is written out as the FP64 sum of the exact products (its own
#     rounding is below 2^-40 relative here) and the bound allows one FP32 ulp
#     (2^-23 relative) per addition:
#         |C'_e[I] - sum_J terms| <= gamma_n(2^-23) * sum_J |terms|
#     (n = number of nonzero terms + 1).
# Without a far field (the term P_BC c_ff of Eq. 14 is zero).
ENSEMBLE_UNIT = 2.0 ** -23
F16_MIN_NORMAL = 2.0 ** -14


def pow2_scale(m: float) -> int:
    """t such that m 2^t lies in [2^14, 2^15) (0 for m = 0)."""
    if m == 0.0:
        return 0
    return 15 - int(np.frexp(m)[1])


def _f16_normal(x):
    """FP32 values rounded to FP16, results below the smallest normal FP16
    number flushed to 0 (as FP64)."""
    y = np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)
    return np.where(np.abs(y) < F16_MIN_NORMAL, 0.0, y)


def ensemble_operands(P, C):
    """(P, C, s, t) as the ensemble product takes them: P16 = P rounded to
    FP16 (its storage), then scaled by 2^s; every member of C (shape (E, n))
    rounded to FP32, scaled by 2^t_e and rounded to FP16; operands below
    2^-14 after the scaling set to 0.  FP64 arrays of the scaled values, s and
    the vector t."""
    P = np.asarray(P, dtype=np.float64)
    C = np.atleast_2d(np.asarray(C, dtype=np.float64))
    P16 = P.astype(np.float16).astype(np.float64)
    s = pow2_scale(float(np.abs(P16).max()) if P16.size else 0.0)
    Ps = _f16_normal(P16 * 2.0 ** s)
    C32 = C.astype(np.float32)
    t = np.array([pow2_scale(float(np.abs(C32[e]).max()) if C32.shape[1] else 0.0) for e in range(C32.shape[0])])
    Cs = np.stack([_f16_normal(C32[e].astype(np.float64) * 2.0 ** int(t[e])) for e in range(C32.shape[0])])
    return Ps, Cs, s, t


def ensemble_product(P, C):
    """(C', bound) for the ensemble C (shape (E, n), one coarse field per
    row): C'[e] = P C[e] with the operands of ensemble_operands, the exact
    products summed in FP64 and scaled back; bound[e, I] as above."""
    Ps, Cs, s, t = ensemble_operands(P, C)
    E = Cs.shape[0]
    out = np.empty((E, Ps.shape[0]))
    bnd = np.empty_like(out)
    nz = Ps != 0.0
    for e in range(E):
        back = 2.0 ** -(s + int(t[e]))
        tm = Ps * Cs[e][None, :]                 # exact: FP16 x FP16 fits FP64
        out[e] = tm.sum(axis=1) * back
        n = (nz & (Cs[e][None, :] != 0.0)).sum(axis=1) + 1
        nu = n * ENSEMBLE_UNIT
        gam = np.where(nu < 1.0, nu / np.maximum(1.0 - nu, 1e-300), np.inf)
        bnd[e] = gam * np.abs(tm).sum(axis=1) * back
    return out, bnd
