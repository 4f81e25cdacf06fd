"""CPU FP64 oracle of the FDiRW fast-diffusion step (arXiv 2408.11376).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  The product library never loads it
and the two share no code; they only consume the same seeded arrays from
``synth``.

The arithmetic lives in ``fdirw_oracle.c`` (plain loops, FP64, compiled with
-ffp-contract=off).  This module only marshals numpy arrays in and out.

Functions (and the passage each follows):
  resolve_dt      sub-step from the explicit stability limit (reading of the
                  unstated FD scheme, Sec. 3.1)
  coefficients    per-face lambda = harmonic-mean D * dt / h^2 (Eq. 1 D per phase)
  kernels         unit point-source responses = columns of P (Sec. 3.1, Eq. 9),
                  optionally with a steady flow (upwind advection, Sec. 5)
  step            superposition c_new = P c_old (Eq. 8, column/scatter form)
  field_sum       compensated FP64 mass of a field (mass balance, Eq. 7 role)
  global_fd       the same explicit update on the whole domain (test reference;
                  optionally with Dirichlet cells, the far-field boundary of Eq. 8)
  support         structural support of a kernel (integer BFS, test reference)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdirw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        lib.fo_resolve_dt.argtypes = [i32, i32, i32, P, P, f64, f64]
        lib.fo_resolve_dt.restype = f64
        lib.fo_coefficients.argtypes = [i32, i32, i32, P, P, f64, f64, P, P, P]
        lib.fo_coefficients.restype = None
        lib.fo_kernels.argtypes = [i32, i32, i32, P, P, P, i32, i32, P, i64, P, P]
        lib.fo_kernels.restype = None
        lib.fo_kernels_fixed.argtypes = [i32, i32, i32, P, P, P, i32, i32, P, i64, P, P, P]
        lib.fo_kernels_fixed.restype = None
        lib.fo_global_fd_fixed.argtypes = [i32, i32, i32, P, P, P, i32, P, P, P, f64]
        lib.fo_global_fd_fixed.restype = None
        lib.fo_kernels_general.argtypes = [i32, i32, i32, P, P, P, i32, i32, P, i64, P, P, P, P, P, P]
        lib.fo_kernels_general.restype = None
        lib.fo_global_fd_general.argtypes = [i32, i32, i32, P, P, P, i32, P, P, P, f64, P, P, P]
        lib.fo_global_fd_general.restype = None
        lib.fo_step.argtypes = [i32, i32, i32, P, P, P, i32, i32, P, P, P]
        lib.fo_step.restype = i64
        lib.fo_global_fd.argtypes = [i32, i32, i32, P, P, P, i32, P, P]
        lib.fo_global_fd.restype = None
        lib.fo_support.argtypes = [i32, i32, i32, P, P, P, i32, i32, i64, P]
        lib.fo_support.restype = None
        lib.fo_sum.argtypes = [P, i64]
        lib.fo_sum.restype = f64
        lib.fo_num_threads.argtypes = []
        lib.fo_num_threads.restype = i32
        lib.fo_set_num_threads.argtypes = [i32]
        lib.fo_set_num_threads.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _grid(label: np.ndarray):
    label = np.ascontiguousarray(label, dtype=np.uint8)
    nz, ny, nx = label.shape
    return label, nx, ny, nz


def num_threads() -> int:
    return int(_load().fo_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    _load().fo_set_num_threads(int(n))


def resolve_dt(label, d_phase, h: float = 1.0, dt: float = 0.0) -> float:
    label, nx, ny, nz = _grid(label)
    d_phase = np.ascontiguousarray(d_phase, dtype=np.float64)
    return float(_load().fo_resolve_dt(nx, ny, nz, _p(label), _p(d_phase), h, dt))


def coefficients(label, d_phase, h: float = 1.0, dt: float = 0.0):
    """(lam_x, lam_y, lam_z, dt): owned +x/+y/+z face coefficients, float64 [nz,ny,nx]."""
    label, nx, ny, nz = _grid(label)
    d_phase = np.ascontiguousarray(d_phase, dtype=np.float64)
    dt = resolve_dt(label, d_phase, h, dt)
    lx = np.empty(label.shape)
    ly = np.empty(label.shape)
    lz = np.empty(label.shape)
    _load().fo_coefficients(nx, ny, nz, _p(label), _p(d_phase), h, dt, _p(lx), _p(ly), _p(lz))
    return lx, ly, lz, dt


class Problem:
    """A domain with its face coefficients, ready for kernels/step calls.

    velocity (optional): [3, nz, ny, nx] steady flow on the owned +x, +y, +z
    face of every cell (h per unit time, positive towards +x / +y / +z); the
    kernels then include first-order upwind advection with Courant numbers
    u dt / h (the steady-flow extension of P, Sec. 5)."""

    def __init__(self, label, d_phase, r: int, n_sub: int, h: float = 1.0, dt: float = 0.0, velocity=None):
        self.label, self.nx, self.ny, self.nz = _grid(label)
        self.d_phase = np.ascontiguousarray(d_phase, dtype=np.float64)
        self.r, self.n_sub, self.h = int(r), int(n_sub), float(h)
        self.lx, self.ly, self.lz, self.dt = coefficients(self.label, self.d_phase, h, dt)
        self.nu = None
        if velocity is not None:
            u = np.asarray(velocity, dtype=np.float64).reshape((3,) + self.label.shape)
            self.nu = [np.ascontiguousarray(u[a] * self.dt / self.h) for a in range(3)]

    @classmethod
    def from_domain(cls, dom):
        return cls(dom.label, dom.d_phase, dom.r, dom.n_sub, dom.h, dom.dt)

    @property
    def W(self):
        return 2 * self.r + 1

    def _dims(self):
        return self.nx, self.ny, self.nz, _p(self.lx), _p(self.ly), _p(self.lz)

    def kernels(self, src, fixed=None):
        """G [n_src, W, W, W] (z, y, x relative to s - r) and mass [n_src].
        fixed: optional bool grid of Dirichlet cells held at 0 (absorbing)."""
        src = np.ascontiguousarray(src, dtype=np.int64).ravel()
        W = self.W
        G = np.empty((src.size, W, W, W))
        mass = np.empty(src.size)
        if src.size:
            f = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8).reshape(self.label.shape)
            nu = self.nu if self.nu is not None else [None, None, None]
            _load().fo_kernels_general(*self._dims(), self.r, self.n_sub, _p(src), src.size, _p(G), _p(mass),
                                       None if f is None else _p(f),
                                       *[None if v is None else _p(v) for v in nu])
        return G, mass

    def step(self, c_old):
        """One big step; returns (c_new, n_sources_used, (kmass_min, kmass_max))."""
        c_old = np.ascontiguousarray(c_old, dtype=np.float64).reshape(self.label.shape)
        c_new = np.empty_like(c_old)
        mm = np.empty(2)
        used = _load().fo_step(*self._dims(), self.r, self.n_sub, _p(c_old), _p(c_new), _p(mm))
        return c_new, int(used), (float(mm[0]), float(mm[1]))

    def global_fd(self, c, n_sub=None, fixed=None, fval: float = 0.0):
        """Whole-domain explicit FD; fixed: optional bool grid of Dirichlet
        cells holding fval from the start."""
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(self.label.shape)
        out = np.empty_like(c)
        n = self.n_sub if n_sub is None else int(n_sub)
        f = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8).reshape(self.label.shape)
        nu = self.nu if self.nu is not None else [None, None, None]
        _load().fo_global_fd_general(*self._dims(), n, _p(c), _p(out), None if f is None else _p(f), float(fval),
                                     *[None if v is None else _p(v) for v in nu])
        return out

    def support(self, s: int):
        out = np.empty((self.W,) * 3, dtype=np.uint8)
        _load().fo_support(*self._dims(), self.r, self.n_sub, int(s), _p(out))
        return out


def field_sum(c) -> float:
    c = np.ascontiguousarray(c, dtype=np.float64).ravel()
    return float(_load().fo_sum(_p(c), c.size))
