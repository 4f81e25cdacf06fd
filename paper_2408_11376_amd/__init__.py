"""MI355X (gfx950) FDiRW fast-diffusion library: thin Python binding.

Every function below marshals arguments into the C ABI of ``libfdirw.so``
(declared in ``include/fdirw.h``) and does nothing else: all arithmetic of the
step runs in the library's HIP kernels.  PyTorch supplies device memory and
the current stream.  There is no CPU fallback: if the library is missing the
import of a function raises.

Names follow the ABI:
    fdirw_coefficients, fdirw_kernels, fdirw_kernels_flow, fdirw_step, fdirw_run,
    fdirw_field_sum, fdirw_last_error, fdirw_release, fdirw_abi_version,
    fdirw_nn_create, fdirw_nn_destroy, fdirw_nn_num_params,
    fdirw_nn_set_params, fdirw_nn_get_params, fdirw_nn_forward,
    fdirw_nn_backward, fdirw_nn_adam, fdirw_nn_save, fdirw_nn_load,
    fdirw_coarse_create, fdirw_coarse_step, fdirw_coarse_step_far_field,
    fdirw_coarse_shape, fdirw_coarse_matrix, fdirw_coarse_pbc,
    fdirw_coarse_destroy (wrapped by ``Coarse``)
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdirw.so")

# precision modes (fdirw_prec)
FP64, FP32, FP16X32, BF16X32, FP16_STATE, BF16_STATE, FP16_BANK, BF16_BANK = range(8)
PREC_NAMES = {"fp64": FP64, "fp32": FP32, "fp16x32": FP16X32, "bf16x32": BF16X32,
              "fp16_state": FP16_STATE, "bf16_state": BF16_STATE,
              "fp16_bank": FP16_BANK, "bf16_bank": BF16_BANK}
GEN_FD, GEN_NN = 0, 1

OK, E_ARG, E_UNSTABLE, E_NOMEM, E_DEVICE, E_UNSUPPORTED, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_UNSTABLE", -3: "E_NOMEM", -4: "E_DEVICE",
                -5: "E_UNSUPPORTED", -6: "E_NONFINITE"}
MAX_RADIUS = 8


class FdirwError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class fdirw_domain(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double),
                ("label", ctypes.c_void_p),
                ("d_phase", ctypes.POINTER(ctypes.c_double)),
                ("n_phase", ctypes.c_int32),
                ("r", ctypes.c_int32),
                ("n_sub", ctypes.c_int32),
                ("dt", ctypes.c_double)]


class fdirw_opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("gen", ctypes.c_int32),
                ("nn", ctypes.c_void_p),
                ("audit_tol", ctypes.c_double),
                ("audit_samples", ctypes.c_int32),
                ("deterministic", ctypes.c_int32),
                ("bank_budget_bytes", ctypes.c_size_t),
                ("stream", ctypes.c_void_p),
                ("tune", ctypes.c_int32)]


class fdirw_stats(ctypes.Structure):
    _fields_ = [("mass_in", ctypes.c_double), ("mass_out", ctypes.c_double),
                ("kmass_min", ctypes.c_double), ("kmass_max", ctypes.c_double),
                ("audit_l1", ctypes.c_double), ("seconds", ctypes.c_double),
                ("fallback_used", ctypes.c_int32), ("tuned_config_id", ctypes.c_int32),
                ("n_sources", ctypes.c_int64),
                ("bank_used", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("kernel_seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


ABI_FUNCTIONS = ("fdirw_coefficients", "fdirw_kernels", "fdirw_kernels_flow", "fdirw_step", "fdirw_step_noalloc",
                 "fdirw_run",
                 "fdirw_field_sum", "fdirw_last_error", "fdirw_release", "fdirw_abi_version",
                 "fdirw_nn_num_params", "fdirw_nn_create", "fdirw_nn_destroy", "fdirw_nn_set_params",
                 "fdirw_nn_get_params", "fdirw_nn_forward", "fdirw_nn_backward", "fdirw_nn_adam",
                 "fdirw_nn_save", "fdirw_nn_load", "fdirw_coarse_create", "fdirw_coarse_set_arith",
                 "fdirw_coarse_step", "fdirw_coarse_apply_ensemble",
                 "fdirw_coarse_step_far_field", "fdirw_coarse_shape", "fdirw_coarse_matrix", "fdirw_coarse_pbc",
                 "fdirw_coarse_destroy", "fdirw_mp_create", "fdirw_mp_step", "fdirw_mp_info", "fdirw_mp_destroy")
NN_RADIUS = 8

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfdirw.so and declare its signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: build it with "
                           f"`python -m paper_2408_11376_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.POINTER(fdirw_domain)
    O = ctypes.POINTER(fdirw_opts)
    S = ctypes.POINTER(fdirw_stats)
    PP = ctypes.POINTER(ctypes.c_void_p)
    lib.fdirw_coefficients.argtypes = [D, P, P, ctypes.POINTER(ctypes.c_double)]
    lib.fdirw_kernels.argtypes = [D, O, P, ctypes.c_int64, P, P]
    lib.fdirw_kernels_flow.argtypes = [D, O, P, P, ctypes.c_int64, P, P]
    lib.fdirw_step.argtypes = [D, ctypes.c_int32, O, PP, PP, S]
    lib.fdirw_step_noalloc.argtypes = [D, O, P, P, S]
    lib.fdirw_run.argtypes = [D, ctypes.c_int32, O, ctypes.c_int32, PP, PP, S]
    lib.fdirw_field_sum.argtypes = [P, ctypes.c_int64, P, ctypes.POINTER(ctypes.c_double)]
    lib.fdirw_last_error.argtypes = []
    lib.fdirw_last_error.restype = ctypes.c_char_p
    lib.fdirw_release.argtypes = []
    lib.fdirw_abi_version.argtypes = []
    lib.fdirw_nn_num_params.argtypes = []
    lib.fdirw_nn_num_params.restype = ctypes.c_int64
    lib.fdirw_nn_create.argtypes = [ctypes.c_int32, ctypes.c_uint64, PP]
    lib.fdirw_nn_destroy.argtypes = [P]
    lib.fdirw_nn_set_params.argtypes = [P, P]
    lib.fdirw_nn_get_params.argtypes = [P, P]
    lib.fdirw_nn_forward.argtypes = [P, D, P, ctypes.c_int64, P, P, P, P]
    lib.fdirw_nn_backward.argtypes = [P, D, P, ctypes.c_int64, P, P, ctypes.POINTER(ctypes.c_double), P]
    lib.fdirw_nn_adam.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
    lib.fdirw_nn_save.argtypes = [P, ctypes.c_char_p]
    lib.fdirw_nn_load.argtypes = [P, ctypes.c_char_p]
    lib.fdirw_coarse_create.argtypes = [D, ctypes.c_int32, ctypes.c_int32, P, P, P, P, PP,
                                        ctypes.POINTER(ctypes.c_double)]
    lib.fdirw_coarse_step.argtypes = [P, P, P, P, S]
    lib.fdirw_coarse_set_arith.argtypes = [P, ctypes.c_int32]
    lib.fdirw_coarse_apply_ensemble.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.POINTER(ctypes.c_double)]
    lib.fdirw_coarse_step_far_field.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                                ctypes.c_double, P, S]
    lib.fdirw_coarse_pbc.argtypes = [P, P]
    lib.fdirw_coarse_shape.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.fdirw_coarse_matrix.argtypes = [P, P]
    lib.fdirw_coarse_destroy.argtypes = [P]
    lib.fdirw_mp_create.argtypes = [D, ctypes.POINTER(fdirw_mp_params), ctypes.c_int32, ctypes.c_int32, P, PP,
                                    ctypes.POINTER(ctypes.c_double)]
    lib.fdirw_mp_step.argtypes = [P, P, ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_int32, P, P, S]
    lib.fdirw_mp_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), PP]
    lib.fdirw_mp_destroy.argtypes = [P]
    for f in ("fdirw_coefficients", "fdirw_kernels", "fdirw_kernels_flow", "fdirw_step", "fdirw_step_noalloc",
              "fdirw_run",
              "fdirw_field_sum",
              "fdirw_release", "fdirw_abi_version", "fdirw_nn_create", "fdirw_nn_destroy",
              "fdirw_nn_set_params", "fdirw_nn_get_params", "fdirw_nn_forward", "fdirw_nn_backward",
              "fdirw_nn_adam", "fdirw_nn_save", "fdirw_nn_load", "fdirw_coarse_create",
              "fdirw_coarse_step", "fdirw_coarse_set_arith", "fdirw_coarse_apply_ensemble",
              "fdirw_coarse_step_far_field", "fdirw_coarse_shape",
              "fdirw_coarse_matrix",
              "fdirw_coarse_pbc", "fdirw_coarse_destroy", "fdirw_mp_create", "fdirw_mp_step", "fdirw_mp_info",
              "fdirw_mp_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        msg = load_library().fdirw_last_error()
        raise FdirwError(status, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Domain:
    """A domain for the library: labels on the device, the D table on the host.

    ``label`` is a [nz, ny, nx] uint8 tensor (or numpy array, copied to the
    current device)."""

    def __init__(self, label, d_phase, r: int, n_sub: int, h: float = 1.0, dt: float = 0.0):
        torch = _torch()
        if isinstance(label, np.ndarray):
            label = torch.from_numpy(np.ascontiguousarray(label, dtype=np.uint8)).cuda()
        self.label = _dev_tensor(label, torch.uint8, "label")
        if self.label.dim() != 3:
            raise ValueError("label must be [nz, ny, nx]")
        self.d_phase = np.ascontiguousarray(d_phase, dtype=np.float64)
        self.r, self.n_sub, self.h, self.dt = int(r), int(n_sub), float(h), float(dt)

    @classmethod
    def from_synth(cls, dom):
        return cls(dom.label, dom.d_phase, dom.r, dom.n_sub, dom.h, dom.dt)

    @property
    def shape(self):
        return tuple(self.label.shape)

    @property
    def n(self):
        return int(self.label.numel())

    @property
    def W(self):
        return 2 * self.r + 1

    def c_struct(self) -> fdirw_domain:
        nz, ny, nx = self.shape
        s = fdirw_domain()
        s.nx, s.ny, s.nz = nx, ny, nz
        s.h = self.h
        s.label = ctypes.c_void_p(self.label.data_ptr())
        s.d_phase = self.d_phase.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.n_phase = int(self.d_phase.size)
        s.r, s.n_sub, s.dt = self.r, self.n_sub, self.dt
        return s


def _prec(prec) -> int:
    return PREC_NAMES[prec.lower()] if isinstance(prec, str) else int(prec)


def make_opts(prec=FP32, stream=None, bank_budget_bytes: int = 0, tune: int = -1,
              deterministic: int = 0, gen: int = GEN_FD, nn=None, audit_tol: float = 1e-3,
              audit_samples: int = 1024) -> fdirw_opts:
    if isinstance(prec, str):
        prec = PREC_NAMES[prec.lower()]
    o = fdirw_opts()
    o.prec = int(prec)
    o.gen = int(gen)
    o.nn = nn.handle if isinstance(nn, Surrogate) else nn
    o.audit_tol = float(audit_tol)
    o.audit_samples = int(audit_samples)
    o.deterministic = int(deterministic)
    o.bank_budget_bytes = int(bank_budget_bytes)
    o.stream = _stream_ptr(stream)
    o.tune = int(tune)
    return o


# ----------------------------------------------------------------- ABI calls

def fdirw_abi_version() -> int:
    return int(load_library().fdirw_abi_version())


def fdirw_last_error() -> str:
    m = load_library().fdirw_last_error()
    return m.decode() if m else ""


def fdirw_release() -> None:
    _check(load_library().fdirw_release())


def fdirw_coefficients(dom: Domain, lam=None, stream=None):
    """Face coefficients [3, nz, ny, nx] float64 (device) and dt."""
    torch = _torch()
    if lam is None:
        lam = torch.empty((3,) + dom.shape, dtype=torch.float64, device=dom.label.device)
    _dev_tensor(lam, torch.float64, "lam")
    if lam.numel() != 3 * dom.n:
        raise ValueError("lam must hold 3 N doubles")
    dt = ctypes.c_double(0.0)
    ds = dom.c_struct()
    _check(load_library().fdirw_coefficients(ctypes.byref(ds), _stream_ptr(stream),
                                             ctypes.c_void_p(lam.data_ptr()), ctypes.byref(dt)))
    return lam, dt.value


def fdirw_kernels(dom: Domain, src, prec=FP32, stream=None, G=None, mass=None, tune: int = -1):
    """Window kernels of the sources in ``src`` (int64 device tensor of linear
    indices): G [n_src, W, W, W] (float64 for FP64, else float32) and mass."""
    torch = _torch()
    o = make_opts(prec, stream, tune=tune)
    src = _dev_tensor(src, torch.int64, "src")
    n_src = src.numel()
    W = dom.W
    gdt = torch.float64 if o.prec == FP64 else torch.float32
    if G is None:
        G = torch.empty((n_src, W, W, W), dtype=gdt, device=src.device)
    _dev_tensor(G, gdt, "G")
    if G.numel() != n_src * W ** 3:
        raise ValueError("G has the wrong size")
    if mass is None:
        mass = torch.empty(n_src, dtype=torch.float64, device=src.device)
    _dev_tensor(mass, torch.float64, "mass")
    ds = dom.c_struct()
    _check(load_library().fdirw_kernels(ctypes.byref(ds), ctypes.byref(o),
                                        ctypes.c_void_p(src.data_ptr()), n_src,
                                        ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(mass.data_ptr())))
    return G, mass


def fdirw_kernels_flow(dom: Domain, velocity, src, prec=FP32, stream=None, G=None, mass=None):
    """Window kernels with the steady flow ``velocity`` (float64 device tensor
    [3, nz, ny, nx]: u on the owned +x, +y, +z faces, h per unit time)."""
    torch = _torch()
    o = make_opts(prec, stream)
    src = _dev_tensor(src, torch.int64, "src")
    _dev_tensor(velocity, torch.float64, "velocity")
    if velocity.numel() != 3 * dom.n:
        raise ValueError("velocity must hold 3 N doubles")
    n_src = src.numel()
    W = dom.W
    gdt = torch.float64 if o.prec == FP64 else torch.float32
    if G is None:
        G = torch.empty((n_src, W, W, W), dtype=gdt, device=src.device)
    _dev_tensor(G, gdt, "G")
    if G.numel() != n_src * W ** 3:
        raise ValueError("G has the wrong size")
    if mass is None:
        mass = torch.empty(n_src, dtype=torch.float64, device=src.device)
    _dev_tensor(mass, torch.float64, "mass")
    ds = dom.c_struct()
    _check(load_library().fdirw_kernels_flow(ctypes.byref(ds), ctypes.byref(o), ctypes.c_void_p(velocity.data_ptr()),
                                             ctypes.c_void_p(src.data_ptr()), n_src, ctypes.c_void_p(G.data_ptr()),
                                             ctypes.c_void_p(mass.data_ptr())))
    return G, mass


def _ptr_array(ts):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr()
    return arr


def fdirw_step(doms, c_in, c_out=None, prec=FP32, stream=None, stats: bool = False, tune: int = -1,
               nn=None, audit_tol: float = 1e-3, audit_samples: int = 1024, deterministic: bool = False):
    """One big step for one domain or a list of domains.  Returns c_out (and
    a list of stats dicts if ``stats``).  ``nn``: a Surrogate to generate the
    kernels with (GEN_NN, audited against FD).  ``deterministic``: no
    floating-point atomics (bitwise reproducible results)."""
    torch = _torch()
    single = isinstance(doms, Domain)
    doms = [doms] if single else list(doms)
    c_in = [c_in] if single else list(c_in)
    if c_out is None:
        c_out = [torch.empty_like(c) for c in c_in]
    elif single:
        c_out = [c_out]
    for i, (d, a, b) in enumerate(zip(doms, c_in, c_out)):
        _dev_tensor(a, torch.float64, f"c_in[{i}]")
        _dev_tensor(b, torch.float64, f"c_out[{i}]")
        if a.numel() != d.n or b.numel() != d.n:
            raise ValueError(f"field {i} does not match its domain")
    o = make_opts(prec, stream, tune=tune, gen=GEN_NN if nn is not None else GEN_FD, nn=nn,
                  audit_tol=audit_tol, audit_samples=audit_samples, deterministic=int(bool(deterministic)))
    nd = len(doms)
    ds = (fdirw_domain * nd)(*[d.c_struct() for d in doms])
    st = (fdirw_stats * nd)() if stats else None
    _check(load_library().fdirw_step(ds, nd, ctypes.byref(o), _ptr_array(c_in), _ptr_array(c_out),
                                     st if st is not None else None))
    out = c_out[0] if single else c_out
    if stats:
        sd = [s.as_dict() for s in st]
        return out, (sd[0] if single else sd)
    return out


def fdirw_step_noalloc(dom, c_in, c_out, prec=FP32, stream=None, stats: bool = False, tune: int = -1):
    """fdirw_step of one domain through the entry point that allocates
    nothing (its scratch is a fixed device array).  c_out must be given.
    Returns c_out (and the stats dict if ``stats``)."""
    torch = _torch()
    _dev_tensor(c_in, torch.float64, "c_in")
    _dev_tensor(c_out, torch.float64, "c_out")
    if c_in.numel() != dom.n or c_out.numel() != dom.n:
        raise ValueError("field does not match the domain")
    o = make_opts(prec, stream, tune=tune)
    ds = dom.c_struct()
    st = fdirw_stats() if stats else None
    _check(load_library().fdirw_step_noalloc(ctypes.byref(ds), ctypes.byref(o), ctypes.c_void_p(c_in.data_ptr()),
                                             ctypes.c_void_p(c_out.data_ptr()),
                                             ctypes.byref(st) if st is not None else None))
    return (c_out, st.as_dict()) if stats else c_out


def fdirw_run(doms, c, n_steps: int, scratch=None, prec=FP32, stream=None, stats: bool = False,
              bank_budget_bytes: int = 0, tune: int = -1, deterministic: bool = False):
    """``n_steps`` big steps in place on ``c`` (one tensor or a list)."""
    torch = _torch()
    single = isinstance(doms, Domain)
    doms = [doms] if single else list(doms)
    c = [c] if single else list(c)
    if scratch is None:
        scratch = [torch.empty_like(x) for x in c]
    elif single:
        scratch = [scratch]
    for i, (d, a, b) in enumerate(zip(doms, c, scratch)):
        _dev_tensor(a, torch.float64, f"c[{i}]")
        _dev_tensor(b, torch.float64, f"scratch[{i}]")
        if a.numel() != d.n or b.numel() != d.n:
            raise ValueError(f"field {i} does not match its domain")
    o = make_opts(prec, stream, bank_budget_bytes=bank_budget_bytes, tune=tune,
                  deterministic=int(bool(deterministic)))
    nd = len(doms)
    ds = (fdirw_domain * nd)(*[d.c_struct() for d in doms])
    st = (fdirw_stats * nd)() if stats else None
    _check(load_library().fdirw_run(ds, nd, ctypes.byref(o), int(n_steps), _ptr_array(c),
                                    _ptr_array(scratch), st if st is not None else None))
    out = c[0] if single else c
    if stats:
        sd = [s.as_dict() for s in st]
        return out, (sd[0] if single else sd)
    return out


def fdirw_field_sum(c, stream=None) -> float:
    torch = _torch()
    _dev_tensor(c, torch.float64, "c")
    out = ctypes.c_double(0.0)
    _check(load_library().fdirw_field_sum(ctypes.c_void_p(c.data_ptr()), c.numel(), _stream_ptr(stream),
                                          ctypes.byref(out)))
    return out.value


# ----------------------------------------------------------------- coarse mesh

def _phase_flags(dom: Domain, flags, name):
    if flags is None:
        return None
    g = np.ascontiguousarray(flags, dtype=np.uint8)
    if g.size != len(dom.d_phase):
        raise ValueError(f"{name} needs one flag per phase")
    return (ctypes.c_uint8 * g.size)(*g.tolist())


def fdirw_coarse_create(dom: Domain, block: int, prec=FP16_BANK, grouped=None, reservoir=None, velocity=None,
                        stream=None):
    """Handle and build seconds of the coarse operator of ``dom``; ``grouped``:
    per-phase flags of the grouped (fast) phases, None for every D > 0;
    ``reservoir``: per-phase flags of the far-field boundary phases;
    ``velocity``: optional steady flow (float64 device tensor [3, nz, ny, nx])."""
    h = ctypes.c_void_p()
    sec = ctypes.c_double(0.0)
    ds = dom.c_struct()
    vptr = None
    if velocity is not None:
        _dev_tensor(velocity, _torch().float64, "velocity")
        if velocity.numel() != 3 * dom.n:
            raise ValueError("velocity must hold 3 N doubles")
        vptr = ctypes.c_void_p(velocity.data_ptr())
    _check(load_library().fdirw_coarse_create(ctypes.byref(ds), int(block), _prec(prec),
                                              _phase_flags(dom, grouped, "grouped"),
                                              _phase_flags(dom, reservoir, "reservoir"), vptr, _stream_ptr(stream),
                                              ctypes.byref(h), ctypes.byref(sec)))
    return h, sec.value


def fdirw_coarse_step_far_field(handle, c_in, c_out, c_ff: float, m_total: float, v_ff: float, stream=None,
                                stats: bool = False):
    """Returns the new far-field concentration (and the stats dict)."""
    st = fdirw_stats() if stats else None
    cff = ctypes.c_double(float(c_ff))
    _check(load_library().fdirw_coarse_step_far_field(handle, ctypes.c_void_p(c_in.data_ptr()),
                                                      ctypes.c_void_p(c_out.data_ptr()), ctypes.byref(cff),
                                                      float(m_total), float(v_ff), _stream_ptr(stream),
                                                      ctypes.byref(st) if st is not None else None))
    return (cff.value, st.as_dict()) if stats else cff.value


def fdirw_coarse_pbc(handle, out: np.ndarray):
    _check(load_library().fdirw_coarse_pbc(handle, ctypes.c_void_p(out.ctypes.data)))
    return out


COARSE_ARITH = {"fp64": 0, "fp32": 1, "mixed": 2, "fp16": 3}


def fdirw_coarse_set_arith(handle, arith) -> None:
    a = COARSE_ARITH[arith] if isinstance(arith, str) else int(arith)
    _check(load_library().fdirw_coarse_set_arith(handle, a))


def fdirw_coarse_step(handle, c_in, c_out, stream=None, stats: bool = False):
    st = fdirw_stats() if stats else None
    _check(load_library().fdirw_coarse_step(handle, ctypes.c_void_p(c_in.data_ptr()),
                                            ctypes.c_void_p(c_out.data_ptr()), _stream_ptr(stream),
                                            ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def fdirw_coarse_apply_ensemble(handle, C_in, C_out, n_ens: int, stream=None, timed: bool = False):
    ks = ctypes.c_double(0.0)
    _check(load_library().fdirw_coarse_apply_ensemble(handle, ctypes.c_void_p(C_in.data_ptr()),
                                                      ctypes.c_void_p(C_out.data_ptr()), int(n_ens),
                                                      _stream_ptr(stream), ctypes.byref(ks) if timed else None))
    return ks.value if timed else None


def fdirw_coarse_shape(handle):
    shp = (ctypes.c_int32 * 5)()
    nn = ctypes.c_int64(0)
    _check(load_library().fdirw_coarse_shape(handle, shp, ctypes.byref(nn)))
    return tuple(shp), nn.value


def fdirw_coarse_matrix(handle, out: np.ndarray):
    _check(load_library().fdirw_coarse_matrix(handle, ctypes.c_void_p(out.ctypes.data)))
    return out


def fdirw_coarse_destroy(handle) -> None:
    _check(load_library().fdirw_coarse_destroy(handle))


class Coarse:
    """Coarse-mesh FDiRW operator of one geometry (Sec. 3.1, Eqs. 10-15):
    ``block``^3 groups of the grouped phases' cells (default: every D > 0),
    P stored in ``prec`` (fp64, fp32, fp16_bank or bf16_bank); with
    ``reservoir`` phases, the far-field boundary of Eqs. 7 and 14."""

    def __init__(self, dom: Domain, block: int = 5, prec=FP16_BANK, grouped=None, reservoir=None, velocity=None,
                 stream=None):
        self.handle, self.build_seconds = fdirw_coarse_create(dom, block, prec, grouped, reservoir, velocity, stream)
        shp, self.n_nodes = fdirw_coarse_shape(self.handle)
        self.coarse_shape = tuple(shp[:3])
        self.K, self.block = shp[3], shp[4]
        self.n = dom.n

    def set_arith(self, arith):
        """Arithmetic of the product: "fp64", "fp32", "mixed" or "fp16"."""
        fdirw_coarse_set_arith(self.handle, arith)

    def step(self, c_in, c_out=None, stream=None, stats: bool = False):
        torch = _torch()
        _dev_tensor(c_in, torch.float64, "c_in")
        if c_out is None:
            c_out = torch.empty_like(c_in)
        _dev_tensor(c_out, torch.float64, "c_out")
        if c_in.numel() != self.n or c_out.numel() != self.n:
            raise ValueError("field does not match the domain")
        st = fdirw_coarse_step(self.handle, c_in, c_out, stream, stats)
        return (c_out, st) if stats else c_out

    def step_far_field(self, c_in, c_ff: float, m_total: float, v_ff: float, c_out=None, stream=None,
                       stats: bool = False):
        """One step with the far field: (c_out, new c_ff[, stats])."""
        torch = _torch()
        _dev_tensor(c_in, torch.float64, "c_in")
        if c_out is None:
            c_out = torch.empty_like(c_in)
        _dev_tensor(c_out, torch.float64, "c_out")
        if c_in.numel() != self.n or c_out.numel() != self.n:
            raise ValueError("field does not match the domain")
        r = fdirw_coarse_step_far_field(self.handle, c_in, c_out, c_ff, m_total, v_ff, stream, stats)
        return (c_out,) + tuple(r) if stats else (c_out, r)

    def apply_ensemble(self, C_in, C_out=None, stream=None, timed: bool = False):
        """Eq. 14 for an ensemble: C_in (device, float64, [n_ens, n_nodes])
        -> P C_in[e] per member, mixed FP32/FP16 on the matrix cores.
        Returns C_out, or (C_out, device seconds) when ``timed``."""
        torch = _torch()
        _dev_tensor(C_in, torch.float64, "C_in")
        if C_in.dim() != 2 or C_in.shape[1] != self.n_nodes:
            raise ValueError("C_in must be [n_ens, n_nodes]")
        if C_out is None:
            C_out = torch.empty_like(C_in)
        _dev_tensor(C_out, torch.float64, "C_out")
        if tuple(C_out.shape) != tuple(C_in.shape):
            raise ValueError("C_out must have C_in's shape")
        ks = fdirw_coarse_apply_ensemble(self.handle, C_in, C_out, C_in.shape[0], stream, timed)
        return (C_out, ks) if timed else C_out

    def p_bc(self) -> np.ndarray:
        return fdirw_coarse_pbc(self.handle, np.empty(self.n_nodes))

    def matrix(self) -> np.ndarray:
        """P as [(2K+1)^3, n_nodes] float64: entry [o, I] = P[I][I - (o - K)]."""
        kw = 2 * self.K + 1
        return fdirw_coarse_matrix(self.handle, np.empty((kw ** 3, self.n_nodes)))

    def close(self):
        if self.handle:
            fdirw_coarse_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- integrated solver

ROLE_LIQUID, ROLE_SOLID, ROLE_FAR_FIELD = 0, 1, 2


class fdirw_mp_params(ctypes.Structure):
    _fields_ = [("role", ctypes.POINTER(ctypes.c_uint8)), ("a_over_rt", ctypes.POINTER(ctypes.c_double)),
                ("k", ctypes.c_double), ("c_eq_liquid", ctypes.c_double), ("c_eq_solid", ctypes.c_double),
                ("n_sub_solid", ctypes.c_int32), ("v_far_field", ctypes.c_double)]


class Multiphysics:
    """The integrated near-field solver of one geometry (Sec. 2, Eqs. 1-7):
    per-phase ``role`` (ROLE_*), ``a_over_rt`` (A / RT, None for 1), the
    interface law (``k``, ``c_eq_liquid``, ``c_eq_solid``), ``n_sub_solid``
    solid sub-steps per big step and the far-field volume ``v_far_field`` in
    cells; the liquid's coarse operator with ``block`` and ``prec``.
    ``dom.dt`` is the fast sub-step, the big step is ``dom.n_sub * dom.dt``."""

    def __init__(self, dom: Domain, role, k: float, c_eq_liquid: float, c_eq_solid: float, v_far_field: float,
                 a_over_rt=None, n_sub_solid: int = 1, block: int = 5, prec=FP16_BANK, stream=None):
        n_phase = len(dom.d_phase)
        self._role = np.ascontiguousarray(role, dtype=np.uint8)
        if self._role.size != n_phase:
            raise ValueError("role needs one entry per phase")
        self._a = None if a_over_rt is None else np.ascontiguousarray(a_over_rt, dtype=np.float64)
        if self._a is not None and self._a.size != n_phase:
            raise ValueError("a_over_rt needs one entry per phase")
        p = fdirw_mp_params()
        p.role = self._role.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        p.a_over_rt = None if self._a is None else self._a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.k, p.c_eq_liquid, p.c_eq_solid = float(k), float(c_eq_liquid), float(c_eq_solid)
        p.n_sub_solid, p.v_far_field = int(n_sub_solid), float(v_far_field)
        self.dom = dom                         # the solver reads dom.label while it lives
        self.n = dom.n
        self.v_far_field = float(v_far_field)
        h = ctypes.c_void_p()
        sec = ctypes.c_double(0.0)
        ds = dom.c_struct()
        _check(load_library().fdirw_mp_create(ctypes.byref(ds), ctypes.byref(p), int(block), _prec(prec),
                                              _stream_ptr(stream), ctypes.byref(h), ctypes.byref(sec)))
        self.handle, self.build_seconds = h, sec.value
        nf = ctypes.c_int64(0)
        ch = ctypes.c_void_p()
        _check(load_library().fdirw_mp_info(self.handle, ctypes.byref(nf), ctypes.byref(ch)))
        self.n_faces = int(nf.value)
        shp, self.n_nodes = fdirw_coarse_shape(ch)
        self.K, self.block = shp[3], shp[4]

    def step(self, c, c_ff: float, m_total: float, n_steps: int = 1, stream=None, stats: bool = False):
        """n_steps big steps on the float64 device tensor c (in place); returns
        (c_ff after the last step, history [n_steps, 3] of Q_L, Q_S, c_ff[, stats])."""
        torch = _torch()
        _dev_tensor(c, torch.float64, "c")
        if c.numel() != self.n:
            raise ValueError("field does not match the domain")
        cff = ctypes.c_double(float(c_ff))
        hist = np.zeros((int(n_steps), 3))
        st = fdirw_stats() if stats else None
        _check(load_library().fdirw_mp_step(self.handle, ctypes.c_void_p(c.data_ptr()), ctypes.byref(cff),
                                            float(m_total), int(n_steps), ctypes.c_void_p(hist.ctypes.data),
                                            _stream_ptr(stream), ctypes.byref(st) if st is not None else None))
        return (cff.value, hist, st.as_dict()) if stats else (cff.value, hist)

    def close(self):
        if self.handle:
            fdirw_mp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fdirw_mp_destroy(handle):
    _check(load_library().fdirw_mp_destroy(handle))


# ----------------------------------------------------------------- surrogate

def fdirw_nn_num_params() -> int:
    return int(load_library().fdirw_nn_num_params())


class Surrogate:
    """Handle of the learned window-kernel generator (r = NN_RADIUS) on the
    current device.  Thin wrapper of the fdirw_nn_* calls."""

    def __init__(self, n_sub: int, seed: int = 0):
        self.handle = fdirw_nn_create(n_sub, seed)
        self.n_sub = int(n_sub)

    def close(self):
        if self.handle is not None:
            fdirw_nn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        fdirw_nn_set_params(self.handle, theta)

    def get_params(self):
        return fdirw_nn_get_params(self.handle)

    def forward(self, dom, src, stream=None, G=True, support=False, logits=False):
        return fdirw_nn_forward(self.handle, dom, src, stream=stream, G=G, support=support, logits=logits)

    def backward(self, dom, src, target=None, stream=None, grad=False):
        return fdirw_nn_backward(self.handle, dom, src, target=target, stream=stream, grad=grad)

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        fdirw_nn_adam(self.handle, lr, beta1, beta2, eps, stream=stream)

    def save(self, path):
        fdirw_nn_save(self.handle, path)

    def load(self, path):
        fdirw_nn_load(self.handle, path)


def fdirw_nn_create(n_sub: int, seed: int = 0):
    h = ctypes.c_void_p()
    _check(load_library().fdirw_nn_create(int(n_sub), ctypes.c_uint64(int(seed)), ctypes.byref(h)))
    return h.value


def fdirw_nn_destroy(handle) -> None:
    _check(load_library().fdirw_nn_destroy(handle))


def fdirw_nn_set_params(handle, theta) -> None:
    th = np.ascontiguousarray(theta, dtype=np.float32)
    if th.size != fdirw_nn_num_params():
        raise ValueError("theta has the wrong size")
    _check(load_library().fdirw_nn_set_params(handle, th.ctypes.data_as(ctypes.c_void_p)))


def fdirw_nn_get_params(handle) -> np.ndarray:
    th = np.empty(fdirw_nn_num_params(), dtype=np.float32)
    _check(load_library().fdirw_nn_get_params(handle, th.ctypes.data_as(ctypes.c_void_p)))
    return th


def _nn_src(dom, src):
    torch = _torch()
    if dom.r != NN_RADIUS:
        raise ValueError(f"the surrogate needs r = {NN_RADIUS}")
    return _dev_tensor(src, torch.int64, "src")


def fdirw_nn_forward(handle, dom: Domain, src, stream=None, G=True, support=False, logits=False):
    """Surrogate kernels of the sources ``src``.  Returns a dict with the
    requested [n_src, W, W, W] tensors ``G`` (float32), ``support`` (uint8) and
    ``logits`` (float32)."""
    torch = _torch()
    src = _nn_src(dom, src)
    n_src = src.numel()
    W = dom.W
    out = {}
    if G:
        out["G"] = torch.empty((n_src, W, W, W), dtype=torch.float32, device=src.device)
    if support:
        out["support"] = torch.empty((n_src, W, W, W), dtype=torch.uint8, device=src.device)
    if logits:
        out["logits"] = torch.empty((n_src, W, W, W), dtype=torch.float32, device=src.device)
    ptr = lambda k: ctypes.c_void_p(out[k].data_ptr()) if k in out else None
    ds = dom.c_struct()
    _check(load_library().fdirw_nn_forward(handle, ctypes.byref(ds), ctypes.c_void_p(src.data_ptr()), n_src,
                                           ptr("G"), ptr("support"), ptr("logits"), _stream_ptr(stream)))
    return out


def fdirw_nn_backward(handle, dom: Domain, src, target=None, stream=None, grad=False):
    """Mean loss (KL, L1) over the windows of ``src`` against ``target``
    (float32 [n_src, W, W, W] device tensor, or None for FD kernels) and,
    if ``grad``, the gradient as a float32 device tensor."""
    torch = _torch()
    src = _nn_src(dom, src)
    n_src = src.numel()
    tp = None
    if target is not None:
        _dev_tensor(target, torch.float32, "target")
        if target.numel() != n_src * dom.W ** 3:
            raise ValueError("target has the wrong size")
        tp = ctypes.c_void_p(target.data_ptr())
    g = torch.empty(fdirw_nn_num_params(), dtype=torch.float32, device=src.device) if grad else None
    loss = (ctypes.c_double * 2)()
    ds = dom.c_struct()
    _check(load_library().fdirw_nn_backward(handle, ctypes.byref(ds), ctypes.c_void_p(src.data_ptr()), n_src, tp,
                                            ctypes.c_void_p(g.data_ptr()) if g is not None else None, loss,
                                            _stream_ptr(stream)))
    return (loss[0], loss[1]), g


def fdirw_nn_adam(handle, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None) -> None:
    _check(load_library().fdirw_nn_adam(handle, float(lr), float(beta1), float(beta2), float(eps),
                                        _stream_ptr(stream)))


def fdirw_nn_save(handle, path: str) -> None:
    _check(load_library().fdirw_nn_save(handle, os.fsencode(path)))


def fdirw_nn_load(handle, path: str) -> None:
    _check(load_library().fdirw_nn_load(handle, os.fsencode(path)))
