"""Seeded synthetic inputs for the FDiRW fast-diffusion step.

This module only *generates data*: phase-label grids, per-phase diffusivity
tables, initial concentration fields and the (r, n_sub) pairs of each workload.
It contains none of the method's arithmetic (no face coefficients, no time
step, no stencil, no superposition), so both the CPU oracle and the GPU path
can consume its arrays without sharing any computation.

The paper's own geometries (phase-field wasteform particles R25/R50/R75,
Figs. 1 and 13) are not available; the generators below stand in for them with
synthetic porous media of the same grid sizes and of the same kind of strongly
inhomogeneous diffusivity (liquid/pore vs solid contrast of 1e2..1e6).

Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) in its counter form: the i-th
output of stream ``seed`` is ``mix(seed + (i + 1) * GAMMA)``.  Uniforms in
[0, 1) take the top 53 bits; normals use the Box-Muller transform.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` raw 64-bit outputs of SplitMix64 stream ``seed`` starting at
    output index ``offset`` (counter form, vectorised)."""
    idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1): top 53 bits times 2**-53."""
    return (splitmix64(seed, count, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normals by Box-Muller on consecutive uniform pairs."""
    m = (count + 1) // 2
    u = uniform(seed, 2 * m)
    u1 = 1.0 - u[0::2]          # (0, 1]: log is finite
    u2 = u[1::2]
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([rad * np.cos(2.0 * np.pi * u2), rad * np.sin(2.0 * np.pi * u2)])
    out = np.empty(2 * m)
    out[0::2] = z[:m]
    out[1::2] = z[m:]
    return out[:count]


@dataclass
class Domain:
    """One synthetic workload.

    label   uint8 [nz, ny, nx] phase labels (x fastest)
    d_phase float64 [n_phase] diffusivity per label
    c0      float64 [nz, ny, nx] initial concentration
    r       window radius (window edge W = 2r + 1)
    n_sub   explicit sub-steps per big step
    dt      sub-step length; 0 means "derive from the stability limit"
    h       grid spacing
    """
    label: np.ndarray
    d_phase: np.ndarray
    c0: np.ndarray
    r: int
    n_sub: int
    dt: float = 0.0
    h: float = 1.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.label.shape

    @property
    def n(self):
        return int(self.label.size)


# ---------------------------------------------------------------- geometries

def spheres(n: int, count: int, rmin: float, rmax: float, seed: int, max_tries: int = 100000):
    """Binary mask of ``count`` non-overlapping solid spheres in an n^3 box.

    Radius ~ U[rmin, rmax], centre ~ U[0, n)^3, rejection until every pair is
    separated (|c_i - c_j| > rho_i + rho_j).  A cell is solid when its centre
    (x + 0.5) lies within a sphere.  Returns uint8 [n, n, n], 1 = solid."""
    centres, radii = [], []
    draw = 0
    u = uniform(seed, 4 * max_tries)
    while len(centres) < count:
        if draw >= max_tries:
            raise RuntimeError("sphere packing did not converge")
        rho = rmin + (rmax - rmin) * u[4 * draw]
        c = n * u[4 * draw + 1: 4 * draw + 4]
        draw += 1
        if all(np.linalg.norm(c - cj) > rho + rj for cj, rj in zip(centres, radii)):
            centres.append(c)
            radii.append(rho)
    g = np.arange(n) + 0.5
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    solid = np.zeros((n, n, n), dtype=bool)
    for c, rho in zip(centres, radii):
        # c = (cx, cy, cz)
        d2 = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2
        solid |= d2 <= rho * rho
    return solid.astype(np.uint8), np.array(centres), np.array(radii)


def voronoi3(n: int, n_seeds: int, gb_width: float, p_pore: float, seed: int):
    """Three-phase Voronoi microstructure in an n^3 box.

    Seeds ~ U[0, n)^3; each cell belongs to its nearest seed (ties to the lower
    seed index); a seed's grain is pore with probability ``p_pore``, else solid
    grain; cells whose second-nearest seed is closer than ``gb_width`` beyond
    the nearest form the grain boundary.  Labels: 0 pore, 1 grain, 2 grain
    boundary."""
    u = uniform(seed, 3 * n_seeds + n_seeds)
    pts = n * u[: 3 * n_seeds].reshape(n_seeds, 3)          # (x, y, z)
    is_pore = u[3 * n_seeds:] < p_pore
    g = np.arange(n, dtype=np.float64) + 0.5
    label = np.empty((n, n, n), dtype=np.uint8)
    yy, xx = np.meshgrid(g, g, indexing="ij")
    for z in range(n):
        d2 = ((xx[..., None] - pts[:, 0]) ** 2 + (yy[..., None] - pts[:, 1]) ** 2
              + (g[z] - pts[:, 2]) ** 2)                       # [n, n, seeds]
        order = np.argsort(d2, axis=-1, kind="stable")          # stable: ties -> lower index
        first = order[..., 0]
        d1 = np.sqrt(np.take_along_axis(d2, order[..., :1], -1)[..., 0])
        d2nd = np.sqrt(np.take_along_axis(d2, order[..., 1:2], -1)[..., 0])
        lab = np.where(is_pore[first], 0, 1).astype(np.uint8)
        lab[(d2nd - d1) < gb_width] = 2
        label[z] = lab
    return label


def grf_mask(shape, corr_len: float, solid_fraction: float, seed: int):
    """Porous two-phase mask from a thresholded Gaussian random field.

    White N(0,1) noise is smoothed by a periodic Gaussian filter of standard
    deviation ``corr_len`` voxels (applied in Fourier space); the
    ``round(solid_fraction * N)`` lowest values (ties broken by linear index)
    become solid.  Returns uint8, 1 = solid."""
    nz, ny, nx = shape
    noise = normal(seed, nz * ny * nx).reshape(shape)
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    filt = np.exp(-2.0 * (np.pi * corr_len) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    field_ = np.fft.irfftn(np.fft.rfftn(noise) * filt, s=shape, axes=(0, 1, 2))
    flat = field_.ravel()
    n_solid = int(np.floor(solid_fraction * flat.size + 0.5))
    order = np.lexsort((np.arange(flat.size), flat))          # by value, then index
    solid = np.zeros(flat.size, dtype=np.uint8)
    solid[order[:n_solid]] = 1
    return solid.reshape(shape)


# ---------------------------------------------------------------- workloads

def config0(seed: int = 11) -> Domain:
    """24^3, 12 solid spheres of radius 3..6, D = 1 pore / 0 solid, r = 3,
    40 sub-steps at the stability-derived dt, c0 ~ U[0,1] in pore, 0 in solid."""
    n = 24
    solid, _, _ = spheres(n, 12, 3.0, 6.0, seed)
    c0 = uniform(seed + 1, n ** 3).reshape(n, n, n)
    c0[solid == 1] = 0.0
    return Domain(label=solid, d_phase=np.array([1.0, 0.0]), c0=c0, r=3, n_sub=40,
                  dt=0.0, name="spheres24_fp64")


def config1(seed: int = 12) -> Domain:
    """96^3 three-phase Voronoi (200 seeds, boundary width 2), log10 D per
    phase ~ U[-4, 0], r = 8, 200 sub-steps, c0 ~ U[0,1]."""
    n = 96
    label = voronoi3(n, 200, 2.0, 0.3, seed)
    dphase = 10.0 ** (-4.0 * uniform(seed + 1, 3))
    c0 = uniform(seed + 2, n ** 3).reshape(n, n, n)
    return Domain(label=label, d_phase=dphase, c0=c0, r=8, n_sub=200, dt=0.0,
                  name="voronoi96_fp32")


def config2(seed: int = 13, n: int = 192) -> Domain:
    """192^3 porous GRF mask (correlation length 6, solid fraction 0.35),
    D_pore = 1, D_solid = 1e-6, r = 8, 200 sub-steps, c0 ~ U[0,1]."""
    solid = grf_mask((n, n, n), 6.0, 0.35, seed)
    c0 = uniform(seed + 1, n ** 3).reshape(n, n, n)
    return Domain(label=solid, d_phase=np.array([1.0, 1e-6]), c0=c0, r=8, n_sub=200,
                  dt=0.0, name=f"grf{n}_mixed")


def n_sub_for_radius(r: int) -> int:
    """Sub-steps for a window radius in the batched workload: keeps the
    spread-to-radius ratio of the r = 8 / 200-step case (200 * (r/8)^2,
    rounded half up)."""
    return int(np.floor(200.0 * (r / 8.0) ** 2 + 0.5))


def config3(seed: int = 14, count: int = 64, lo: int = 32, hi: int = 128):
    """``count`` independent GRF domains with edges ~ U{lo..hi} per axis,
    contrast K log-uniform in [1e2, 1e6] (D_pore = 1, D_solid = 1/K) and
    r ~ U{4, 6, 8}; c0 ~ U[0,1]."""
    doms = []
    for i in range(count):
        s = seed + i
        u = uniform(s * 1000 + 7, 5)
        dims = [lo + int(np.floor(u[k] * (hi - lo + 1))) for k in range(3)]   # (nx, ny, nz)
        K = 10.0 ** (2.0 + 4.0 * u[3])
        r = (4, 6, 8)[int(np.floor(u[4] * 3))]
        shape = (dims[2], dims[1], dims[0])
        solid = grf_mask(shape, 6.0, 0.35, s)
        c0 = uniform(s * 1000 + 9, solid.size).reshape(shape)
        doms.append(Domain(label=solid, d_phase=np.array([1.0, 1.0 / K]), c0=c0, r=r,
                           n_sub=n_sub_for_radius(r), dt=0.0, name=f"batch{i}",
                           meta={"K": K}))
    return doms


# Values of the wasteform-particle case (Table 1, particle radius 50 h): grid
# spacing, fast sub-step and big step, diffusivity and free-energy coefficient
# (A / RT) per phase, equilibrium and initial concentrations, rate constant of
# the interface reaction and the far-field liquid volume (1.80e-10 mL = 1.8e8
# cells of (10 nm)^3).  Plain data; the solver decides what to do with them.
TABLE1 = {
    "h": 10e-9, "dt_fd": 0.5e-6, "dt": 500e-6,
    "D_S": 1.0e-17, "D_L": 1.0e-14, "A_S_RT": 2.0e3, "A_L_RT": 2.0e3,
    "c_eq_S": 1.0, "c_eq_L": 1.0e-5, "c0_S": 1.0e-6, "c0_L": 2.12e-3,
    "k": 0.05, "V_ff_cells": 1.8e8,
}

# phase labels of the particle geometry
PHASE_NEAR_LIQUID, PHASE_SOLID, PHASE_FAR_LIQUID = 0, 1, 2


def particle(n: int, r_p: float, shell: float = 5.0, porosity: float = 0.3, corr_len: float = 3.0,
             seed: int = 21):
    """Porous particle of radius ``r_p`` centred in an n^3 grid (the geometry of
    Fig. 1): cells whose centre lies within ``r_p`` of the grid centre are
    solid unless a thresholded Gaussian random field (``grf_mask`` with the
    given correlation length, a ``porosity`` share of the grid) marks them as
    pore; pores and the liquid shell up to ``r_p + shell`` are the near-field
    liquid, every other cell is far-field liquid.  Returns uint8 labels
    (PHASE_NEAR_LIQUID / PHASE_SOLID / PHASE_FAR_LIQUID)."""
    g = np.arange(n, dtype=np.float64) + 0.5 - 0.5 * n
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    d2 = xx * xx + yy * yy + zz * zz
    pore = grf_mask((n, n, n), corr_len, 1.0 - porosity, seed) == 0
    label = np.full((n, n, n), PHASE_FAR_LIQUID, dtype=np.uint8)
    label[d2 <= (r_p + shell) ** 2] = PHASE_NEAR_LIQUID
    label[(d2 <= r_p * r_p) & ~pore] = PHASE_SOLID
    return label


def particle_case(n: int = 192, r_p: float = 50.0, r: int = 8, n_sub: int = 200, seed: int = 21):
    """The wasteform-particle workload: ``particle`` labels, Table 1 values,
    the initial concentrations c0_S in the solid and c0_L in every liquid cell,
    window radius r and n_sub fast sub-steps of dt_fd per big step.  Returns
    (Domain, dict of the Table 1 values)."""
    t = dict(TABLE1)
    label = particle(n, r_p, seed=seed)
    c0 = np.where(label == PHASE_SOLID, t["c0_S"], t["c0_L"])
    d_phase = np.array([t["D_L"], t["D_S"], t["D_L"]])
    return Domain(label=label, d_phase=d_phase, c0=c0, r=r, n_sub=n_sub, dt=t["dt_fd"], h=t["h"],
                  name=f"particle{n}_R{int(r_p)}"), t


def random_small(shape, n_phase: int, r: int, n_sub: int, seed: int, dt: float = 0.0,
                 d_zero_phase: bool = True) -> Domain:
    """Small random multi-phase domain for parity and edge-case tests.

    Labels uniform over ``n_phase`` phases; D of phase 0 is 1, the others
    10**U[-4, 0]; if ``d_zero_phase`` the last phase is impermeable (D = 0)."""
    nz, ny, nx = shape
    u = uniform(seed, nx * ny * nz)
    label = np.minimum((u * n_phase).astype(np.int64), n_phase - 1).astype(np.uint8).reshape(shape)
    dv = 10.0 ** (-4.0 * uniform(seed + 1, n_phase))
    dv[0] = 1.0
    if d_zero_phase and n_phase > 1:
        dv[-1] = 0.0
    c0 = uniform(seed + 2, nx * ny * nz).reshape(shape)
    return Domain(label=label, d_phase=dv, c0=c0, r=r, n_sub=n_sub, dt=dt,
                  name=f"rand{nx}x{ny}x{nz}")


def sub_block_sources(shape, block: int, origin=None):
    """Boolean mask selecting a block^3 cube of source cells (centred unless an
    ``origin`` (z, y, x) is given) — used to restrict a big-grid step to sources
    the CPU oracle can afford, by zeroing c0 outside it."""
    nz, ny, nx = shape
    if origin is None:
        origin = ((nz - block) // 2, (ny - block) // 2, (nx - block) // 2)
    m = np.zeros(shape, dtype=bool)
    z0, y0, x0 = origin
    m[z0:z0 + block, y0:y0 + block, x0:x0 + block] = True
    return m
