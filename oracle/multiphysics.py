"""FP64 CPU oracle of the integrated near-field solver of arXiv 2408.11376
(Sec. 2, Eqs. 1-7, and the flowchart of Sec. 3.4): fast diffusion in the
near-field liquid by the coarse-mesh FDiRW step, absorption at the particle
surface, slow diffusion in the solid, and the far-field concentration from
conservation.  TEST INFRASTRUCTURE: only the tests and the benchmark's CPU leg
may use it; the product library never does.

Phases play one of three roles: near-field liquid (fast), solid (slow) or
far-field liquid (the uniform reservoir of Eq. 7, held in its cells as
Dirichlet boundary).  One field c holds c_L in liquid cells and c_S in solid
cells.

Diffusion (Eqs. 1-3).  Inside one phase A_m and c_m^eq are constant, so the
gradient of mu_m / RT is A_m / RT times the gradient of c_m: each phase
diffuses with the FD coefficient D_m A_m / RT (harmonic mean across faces of
one role, as in the fast step).  The two media exchange mass only through the
interface reaction, so for the liquid step the solid is a wall, and for the
solid step the liquid is.  With the Table 1 values this gives lambda = 0.1 for
the liquid per fast sub-step dt_fd and for the solid per big step dt.

One big step dt = n_sub dt_fd, in the order of the flowchart:
  1. fast diffusion   coarse FDiRW step of the near-field liquid with the
                      far-field term P_BC c_ff (Eqs. 13-15, 14); solid cells
                      keep their value; far-field cells read 0 until step 4
  2. absorption       for every face between a near-field liquid cell and a
                      solid cell, the pseudo-second-order law (Eqs. 4-6)
                          d c_S / dt = k f_L f_S = - d c_L / dt
                      integrated exactly over dt for the pair alone; the faces
                      are taken in six groups in which no cell appears twice:
                      x faces between cells 2i and 2i+1, then 2i+1 and 2i+2,
                      then the same along y and along z
  3. slow diffusion   n_sub_solid explicit sub-steps of dt / n_sub_solid in
                      the solid
  4. far field        Eq. 7: c_ff = (M_total - Q_L - Q_S) / V_ff with Q_L the
                      near-field liquid sum and Q_S the solid sum, written
                      into the far-field cells

Exact pair integration.  Moving x from the liquid cell (value cl) to the solid
cell (value cs), with a = cl - c_L^eq, b = c_S^eq - cs and kappa = k /
(c_L^eq c_S^eq), the law reads dx/dt = kappa (a - x)(b - x) while the liquid
stays above equilibrium.  Partial fractions give, with d = (b - a) kappa dt,
    x = a b (e^d - 1) / (b e^d - a)        (x = a^2 kappa dt / (1 + a kappa dt) if a = b)
which tends to the nearer root and never crosses c_L^eq, so one big step of
the Table 1 case (where an explicit update over dt would overshoot the liquid
value) stays positive.  If a <= 0, f_L = 0 and nothing moves.
"""
from __future__ import annotations

import numpy as np

from . import Problem
from . import coarse

ROLE_LIQUID, ROLE_SOLID, ROLE_FAR = 0, 1, 2


def fd_coefficient(d_phase, a_over_rt):
    """Per-phase coefficient of the Laplacian of c in Eq. 1 with Eqs. 2-3."""
    return np.asarray(d_phase, dtype=np.float64) * np.asarray(a_over_rt, dtype=np.float64)


def masks(label, role):
    role = np.asarray(role)[np.asarray(label)]
    return role == ROLE_LIQUID, role == ROLE_SOLID, role == ROLE_FAR


def pso_transfer(a, b, kappa_dt):
    """Amount moved from liquid to solid over one step for one face: the exact
    solution of dx/dt = kappa (a - x)(b - x), x(0) = 0, at t = dt (0 if a <= 0)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    out = np.zeros(np.broadcast(a, b).shape)
    act = np.broadcast_to(a > 0.0, out.shape)
    a, b = np.broadcast_to(a, out.shape)[act], np.broadcast_to(b, out.shape)[act]
    d = (b - a) * kappa_dt
    x = np.empty_like(a)
    pos = d > 0.0
    # d > 0: divide through by e^d so nothing overflows
    m = -np.expm1(-d[pos])
    x[pos] = a[pos] * b[pos] * m / ((b[pos] - a[pos]) + a[pos] * m)
    neg = d < 0.0
    m = np.expm1(d[neg])
    x[neg] = a[neg] * b[neg] * m / (b[neg] * m + (b[neg] - a[neg]))
    eq = d == 0.0
    x[eq] = a[eq] * b[eq] * kappa_dt / (1.0 + a[eq] * kappa_dt)
    out[act] = x
    return out


def react(c, label, role, k, c_eq_l, c_eq_s, dt):
    """Step 2: interface absorption over dt, the six face groups in order."""
    c = np.array(c, dtype=np.float64, copy=True)
    liq, sol, _ = masks(label, role)
    kappa_dt = k / (c_eq_l * c_eq_s) * dt
    for axis in (2, 1, 0):                      # x, y, z of [z, y, x] arrays
        n = c.shape[axis]
        for parity in (0, 1):
            lo = np.arange(parity, n - 1, 2)
            if lo.size == 0:
                continue
            il = [slice(None)] * 3
            ih = [slice(None)] * 3
            il[axis], ih[axis] = lo, lo + 1
            il, ih = tuple(il), tuple(ih)
            cl, ch = c[il], c[ih]
            l_lo = liq[il] & sol[ih]            # liquid below, solid above
            l_hi = sol[il] & liq[ih]
            cliq = np.where(l_lo, cl, ch)
            csol = np.where(l_lo, ch, cl)
            pair = l_lo | l_hi
            x = np.zeros(cl.shape)
            x[pair] = pso_transfer(cliq[pair] - c_eq_l, c_eq_s - csol[pair], kappa_dt)
            c[il] = cl - np.where(l_lo, x, 0.0) + np.where(l_hi, x, 0.0)
            c[ih] = ch + np.where(l_lo, x, 0.0) - np.where(l_hi, x, 0.0)
    return c


def solid_problem(label, d_phase, a_over_rt, role, h, dt, n_sub_solid):
    """The solid step as an FD problem: coefficient D A / RT in solid phases, 0
    (walls) elsewhere, sub-step dt / n_sub_solid."""
    d = fd_coefficient(d_phase, a_over_rt)
    d = np.where(np.asarray(role) == ROLE_SOLID, d, 0.0)
    return Problem(label, d, 0, n_sub_solid, h, dt / n_sub_solid)


def liquid_problem(label, d_phase, a_over_rt, role, r, n_sub, h, dt_fd):
    """The fast step's FD problem: coefficient D A / RT in liquid phases (near
    and far field), 0 in the solid."""
    d = fd_coefficient(d_phase, a_over_rt)
    d = np.where(np.asarray(role) == ROLE_SOLID, 0.0, d)
    return Problem(label, d, r, n_sub, h, dt_fd)


def far_field(c, label, role, m_total, v_ff):
    """Step 4 (Eq. 7): returns (c with the far-field cells at c_ff, c_ff, Q_L, Q_S)."""
    liq, sol, far = masks(label, role)
    q_l = float(np.sum(c[liq]))
    q_s = float(np.sum(c[sol]))
    c_ff = (m_total - q_l - q_s) / v_ff
    out = np.array(c, dtype=np.float64, copy=True)
    out[far] = c_ff
    return out, c_ff, q_l, q_s


class Model:
    """The integrated solver of one geometry.

    d_phase, a_over_rt: per phase D and A / RT; role: per phase ROLE_*;
    r, n_sub, dt_fd: window radius and fast sub-steps of the liquid kernels
    (big step dt = n_sub dt_fd); B: coarse block edge; k, c_eq_l, c_eq_s: the
    interface law; n_sub_solid: solid sub-steps per big step; v_ff: far-field
    volume in cells.  P and P_BC come from the coarse oracle (dense)."""

    def __init__(self, label, d_phase, a_over_rt, role, r, n_sub, h, dt_fd, B, k, c_eq_l, c_eq_s,
                 n_sub_solid, v_ff, P=None, pbc=None):
        self.label = np.asarray(label)
        self.role = np.asarray(role)
        self.B = int(B)
        self.k, self.c_eq_l, self.c_eq_s = float(k), float(c_eq_l), float(c_eq_s)
        self.v_ff = float(v_ff)
        self.dt = n_sub * float(dt_fd)
        self.liquid = liquid_problem(label, d_phase, a_over_rt, role, r, n_sub, h, dt_fd)
        self.solid = solid_problem(label, d_phase, a_over_rt, role, h, self.dt, n_sub_solid)
        self.grouped = self.role == ROLE_LIQUID
        self.reservoir = self.role == ROLE_FAR
        self.P = coarse.coarse_matrix(self.liquid, self.B, self.grouped, self.reservoir) if P is None else P
        self.pbc = coarse.p_bc(self.liquid, self.B, self.grouped, self.reservoir) if pbc is None else pbc

    def fast(self, c, c_ff):
        """Step 1: C' = P C + P_BC c_ff on the near-field groups (Eqs. 13-15);
        far-field cells set to 0."""
        C = coarse.mapping(c, self.label, self.liquid.d_phase, self.B, self.grouped, self.reservoir)
        out = coarse.remapping(self.P @ C + self.pbc * c_ff, c, self.label, self.liquid.d_phase, self.B,
                               self.grouped, self.reservoir)
        out[coarse.reservoir_mask(self.label, self.reservoir)] = 0.0
        return out

    def step(self, c, c_ff, m_total):
        """One big step; returns (c', c_ff', Q_L, Q_S)."""
        c1 = self.fast(c, c_ff)
        c2 = react(c1, self.label, self.role, self.k, self.c_eq_l, self.c_eq_s, self.dt)
        c3 = self.solid.global_fd(c2)
        return far_field(c3, self.label, self.role, m_total, self.v_ff)

    def run(self, c, c_ff, m_total, n_steps):
        """n_steps big steps; returns (c, c_ff, history [n_steps, 3] of Q_L, Q_S, c_ff)."""
        hist = np.zeros((n_steps, 3))
        for s in range(n_steps):
            c, c_ff, q_l, q_s = self.step(c, c_ff, m_total)
            hist[s] = (q_l, q_s, c_ff)
        return c, c_ff, hist
