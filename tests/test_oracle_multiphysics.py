"""Pins of the oracle's integrated near-field solver (Sec. 2, Eqs. 1-7; the
flowchart of Sec. 3.4) against results it does not compute itself: a
fourth-order Runge-Kutta integration of the interface law of Eqs. 4-6, the
explicit update of that law for small rates, the decay of a cosine mode in a
solid box, the whole-domain FD formulation of the fast step, the equilibrium
state as a fixed point, and conservation.  CPU only."""
import numpy as np
import pytest

import oracle
import synth
from oracle import coarse
from oracle import multiphysics as mp

LIQ, SOL, FAR = mp.ROLE_LIQUID, mp.ROLE_SOLID, mp.ROLE_FAR


def _rk4_transfer(cl, cs, k, e_l, e_s, dt, steps=40000):
    """Integrate d cs/dt = k f_L f_S, d cl/dt = -k f_L f_S (Eqs. 4-6, f_L = 0
    at or below equilibrium) with classical RK4; vectorised over cases."""
    cl = np.array(cl, dtype=np.float64)
    cs = np.array(cs, dtype=np.float64)
    cs0 = cs.copy()
    h = dt / steps

    def rate(l, s):
        f_l = np.where(l > e_l, (l - e_l) / e_l, 0.0)
        f_s = (e_s - s) / e_s
        return k * f_l * f_s

    for _ in range(steps):
        r1 = rate(cl, cs)
        r2 = rate(cl - 0.5 * h * r1, cs + 0.5 * h * r1)
        r3 = rate(cl - 0.5 * h * r2, cs + 0.5 * h * r2)
        r4 = rate(cl - h * r3, cs + h * r3)
        inc = h * (r1 + 2 * r2 + 2 * r3 + r4) / 6.0
        cl = cl - inc
        cs = cs + inc
    return cs - cs0


def test_pso_transfer_matches_runge_kutta():
    t = synth.TABLE1
    # (cl, cs, k, e_l, e_s, dt): Table 1 first step; liquid-limited; solid-
    # limited; a = b; supersaturated solid (mass goes back); liquid at or below
    # equilibrium (nothing moves); a slow rate
    cases = [
        (t["c0_L"], t["c0_S"], t["k"], t["c_eq_L"], t["c_eq_S"], t["dt"]),
        (1.3, 0.2, 0.8, 1.0, 2.0, 3.0),
        (4.0, 1.7, 0.5, 1.0, 2.0, 2.0),
        (1.4, 1.6, 0.9, 1.0, 2.0, 1.5),
        (2.5, 2.6, 0.7, 1.0, 2.0, 1.0),
        (0.9, 0.3, 1.0, 1.0, 2.0, 1.0),
        (1.0, 0.3, 1.0, 1.0, 2.0, 1.0),
        (3.0, 0.1, 1e-4, 1.0, 2.0, 0.5),
    ]
    for cl, cs, k, e_l, e_s, dt in cases:
        want = _rk4_transfer([cl], [cs], k, e_l, e_s, dt)[0]
        got = float(mp.pso_transfer(cl - e_l, e_s - cs, k / (e_l * e_s) * dt))
        assert abs(got - want) <= 1e-10 * max(abs(want), 1e-300) + 1e-18, (cl, cs, got, want)


def _roles_case(shape, seed, p_solid=0.4, p_far=0.1):
    u = synth.uniform(seed, int(np.prod(shape))).reshape(shape)
    label = np.where(u < p_solid, 1, np.where(u < p_solid + p_far, 2, 0)).astype(np.uint8)
    role = np.array([LIQ, SOL, FAR])
    c = 1.0 + synth.uniform(seed + 1, label.size).reshape(shape)          # liquid above c_eq = 1
    c[label == 1] = 2.0 * synth.uniform(seed + 2, label.size).reshape(shape)[label == 1]
    return label, role, c


def test_react_is_the_explicit_update_for_small_rates():
    label, role, c = _roles_case((6, 7, 8), 61)
    k, e_l, e_s, dt = 1e-8, 1.0, 2.5, 1.0
    got = mp.react(c, label, role, k, e_l, e_s, dt)
    # every liquid/solid face moves k dt f_L f_S from the old values
    want = c.copy()
    liq, sol = label == 0, label == 1
    nz, ny, nx = label.shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for dz, dy, dx in ((0, 0, 1), (0, 1, 0), (1, 0, 0)):
                    z2, y2, x2 = z + dz, y + dy, x + dx
                    if z2 >= nz or y2 >= ny or x2 >= nx:
                        continue
                    a, b = (z, y, x), (z2, y2, x2)
                    if liq[a] and sol[b]:
                        l_, s_ = a, b
                    elif sol[a] and liq[b]:
                        l_, s_ = b, a
                    else:
                        continue
                    f_l = max((c[l_] - e_l) / e_l, 0.0)
                    f_s = (e_s - c[s_]) / e_s
                    want[l_] -= k * dt * f_l * f_s
                    want[s_] += k * dt * f_l * f_s
    inc_got, inc_want = got - c, want - c
    assert np.count_nonzero(inc_want) > 50
    assert np.max(np.abs(inc_got - inc_want)) <= 1e-6 * np.max(np.abs(inc_want))


def test_react_conserves_and_never_crosses_equilibrium():
    label, role, c = _roles_case((9, 8, 7), 62)
    e_l, e_s = 1.0, 2.5
    got = mp.react(c, label, role, 40.0, e_l, e_s, 3.0)           # a large rate
    assert abs(got.sum() - c.sum()) <= 1e-13 * c.sum()
    liq = label == 0
    assert np.all(got[liq] >= e_l * (1 - 1e-15))
    # cells with no liquid/solid face keep their value, far-field cells too
    sol = label == 1
    touch = np.zeros(label.shape, dtype=bool)
    for ax in range(3):
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[ax], b[ax] = slice(0, -1), slice(1, None)
        pair = (liq[tuple(a)] & sol[tuple(b)]) | (sol[tuple(a)] & liq[tuple(b)])
        touch[tuple(a)] |= pair
        touch[tuple(b)] |= pair
    assert np.array_equal(got[~touch], c[~touch])
    # every solid value starts below c_S^eq and every liquid value above c_L^eq:
    # mass only moves from liquid to solid
    assert np.all(got[sol] >= c[sol]) and np.all(got[liq] <= c[liq])
    assert np.count_nonzero(got != c) > 0


def test_solid_diffusion_cosine_mode_in_a_box_walled_by_liquid():
    # a 6 x 5 x 7 solid box inside liquid: the liquid is a no-flux wall for the
    # solid step, so cos(pi k (x + 1/2) / L) decays by 1 - 2 lam (1 - cos(pi k / L))
    # per sub-step, lam = D A / RT * (dt / n) / h^2
    label = np.zeros((9, 8, 11), dtype=np.uint8)
    z0, y0, x0, Lz, Ly, Lx = 1, 2, 3, 6, 5, 7
    label[z0:z0 + Lz, y0:y0 + Ly, x0:x0 + Lx] = 1
    role = np.array([LIQ, SOL])
    d_phase, a_rt = np.array([3.0, 0.02]), np.array([1.0, 5.0])       # solid coefficient 0.1
    h, dt, n = 0.5, 0.4, 3
    lam = 0.1 * (dt / n) / (h * h)
    c = 7.0 + synth.uniform(71, label.size).reshape(label.shape)
    kx, ky, kz = 2, 1, 3
    zz, yy, xx = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    mode = (np.cos(np.pi * kx * (xx + 0.5) / Lx) * np.cos(np.pi * ky * (yy + 0.5) / Ly)
            * np.cos(np.pi * kz * (zz + 0.5) / Lz))
    c[z0:z0 + Lz, y0:y0 + Ly, x0:x0 + Lx] = mode
    got = mp.solid_problem(label, d_phase, a_rt, role, h, dt, n).global_fd(c)
    f = 1.0
    for k_, L in ((kx, Lx), (ky, Ly), (kz, Lz)):
        f -= 2.0 * lam * (1.0 - np.cos(np.pi * k_ / L))
    want = c.copy()
    want[z0:z0 + Lz, y0:y0 + Ly, x0:x0 + Lx] = mode * f ** n
    assert np.max(np.abs(got - want)) <= 1e-14


def _particle_model(n=10, r_p=3.0, r=3, n_sub=6, B=2, k=0.3, seed=81, **kw):
    label = synth.particle(n, r_p, shell=2.0, porosity=0.3, corr_len=1.5, seed=seed)
    d_phase = np.array([1.0, 0.02, 1.0])
    a_rt = np.array([0.15, 0.5, 0.15])
    role = np.array([LIQ, SOL, FAR])
    args = dict(label=label, d_phase=d_phase, a_over_rt=a_rt, role=role, r=r, n_sub=n_sub, h=1.0, dt_fd=0.5,
                B=B, k=k, c_eq_l=0.01, c_eq_s=1.0, n_sub_solid=2, v_ff=500.0)
    args.update(kw)
    return mp.Model(**args)


def test_fast_step_is_the_whole_domain_fd_with_the_far_field_held():
    # B = 1 and a window covering the domain: P C + P_BC c_ff is the explicit
    # FD of the liquid with the far-field cells held at c_ff
    m = _particle_model(n=8, r_p=2.5, r=7, n_sub=5, B=1)
    liq, sol, far = mp.masks(m.label, m.role)
    c = 0.01 + 0.05 * synth.uniform(82, m.label.size).reshape(m.label.shape)
    c[sol] = 0.3 * synth.uniform(83, m.label.size).reshape(m.label.shape)[sol]
    c_ff = 0.04
    c[far] = c_ff
    want = m.liquid.global_fd(c, fixed=far, fval=c_ff)
    want[far] = 0.0
    got = m.fast(c, c_ff)
    assert np.max(np.abs(got - want)) <= 1e-15
    assert np.array_equal(got[sol], c[sol])


def test_equilibrium_is_a_fixed_point():
    m = _particle_model(n=8, r_p=2.5, r=7, n_sub=5, B=1)
    liq, sol, far = mp.masks(m.label, m.role)
    c = np.full(m.label.shape, m.c_eq_l)
    c[sol] = 0.37
    m_total = c[liq].sum() + c[sol].sum() + m.v_ff * m.c_eq_l
    out, c_ff, hist = m.run(c, m.c_eq_l, m_total, 3)
    want = c.copy()
    want[far] = m.c_eq_l
    assert np.max(np.abs(out - want)) <= 1e-15
    assert abs(c_ff - m.c_eq_l) <= 1e-15


def test_without_reaction_and_solid_diffusion_the_step_is_the_far_field_step():
    m = _particle_model(k=0.0, d_phase=np.array([1.0, 0.0, 1.0]))
    liq, sol, far = mp.masks(m.label, m.role)
    c = 0.02 + 0.05 * synth.uniform(84, m.label.size).reshape(m.label.shape)
    c[sol] = 0.5
    m_total = c[~far].sum() + m.v_ff * 0.03
    got, cff, q_l, q_s = m.step(c, 0.03, m_total)
    want, cff_w = coarse.step_far_field(m.liquid, m.P, m.pbc, c, 0.03, m_total, m.v_ff, m.B, m.grouped,
                                        m.reservoir)
    assert np.max(np.abs(got - want)) <= 1e-15
    assert abs(cff - cff_w) <= 1e-15


def test_absorption_kinetics_conserve_and_fill_the_solid():
    m = _particle_model(k=0.05)
    liq, sol, far = mp.masks(m.label, m.role)
    c = np.where(sol, 1e-4, 0.2)
    c_ff = 0.2
    m_total = c[~far].sum() + m.v_ff * c_ff
    out, c_ff2, hist = m.run(c, c_ff, m_total, 8)
    # Eq. 7 closes the balance after every step
    assert np.max(np.abs(hist[:, 0] + hist[:, 1] + m.v_ff * hist[:, 2] - m_total)) <= 1e-12 * m_total
    # the solid absorbs, the far field empties, nothing crosses equilibrium
    assert np.all(np.diff(hist[:, 1]) > 0) and np.all(np.diff(hist[:, 2]) < 0)
    assert np.all(out[liq] >= m.c_eq_l * (1 - 1e-14))
    assert np.all(out[sol] <= m.c_eq_s)


def test_zero_radius_windows_give_the_identity_operator():
    # r = 0: every kernel is the unit point (no neighbour inside the window),
    # also with absorbing far-field cells, so P = I for B = 1
    m = _particle_model(n=7, r_p=2.0, r=0, n_sub=4, B=1)
    assert np.array_equal(m.P, np.diag(np.diag(m.P)))
    liq = mp.masks(m.label, m.role)[0].ravel()
    assert np.array_equal(np.diag(m.P)[liq], np.ones(liq.sum()))
