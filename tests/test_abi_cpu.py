"""CPU-side checks of the C ABI: the library loads (no GPU call is made),
exports every function the header declares, and the ctypes mirrors of the
structs have the header's layout."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_2408_11376_amd as fd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdirw.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdirw_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert _declared_functions() == sorted(fd.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(fd.LIB_PATH):
        pytest.skip("library not built")
    out = subprocess.run(["nm", "-D", "--defined-only", fd.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (fdirw_\w+)", out))
    for name in _declared_functions():
        assert name in exported, name
    lib = fd.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name)
    assert fd.fdirw_abi_version() == 1


def test_struct_layouts_match_header():
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "fdirw.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("sizeof.fdirw_domain %zu\n", sizeof(fdirw_domain));
  printf("sizeof.fdirw_opts %zu\n", sizeof(fdirw_opts));
  printf("sizeof.fdirw_stats %zu\n", sizeof(fdirw_stats));
  printf("sizeof.fdirw_mp_params %zu\n", sizeof(fdirw_mp_params));
  P(fdirw_mp_params, role) P(fdirw_mp_params, a_over_rt) P(fdirw_mp_params, k) P(fdirw_mp_params, c_eq_liquid)
  P(fdirw_mp_params, c_eq_solid) P(fdirw_mp_params, n_sub_solid) P(fdirw_mp_params, v_far_field)
  P(fdirw_domain, h) P(fdirw_domain, label) P(fdirw_domain, d_phase) P(fdirw_domain, n_phase)
  P(fdirw_domain, r) P(fdirw_domain, n_sub) P(fdirw_domain, dt)
  P(fdirw_opts, nn) P(fdirw_opts, audit_tol) P(fdirw_opts, bank_budget_bytes) P(fdirw_opts, stream) P(fdirw_opts, tune)
  P(fdirw_stats, seconds) P(fdirw_stats, fallback_used) P(fdirw_stats, n_sources) P(fdirw_stats, bank_used) P(fdirw_stats, kernel_seconds)
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), "-o", exe, c])
        out = subprocess.run([exe], capture_output=True, text=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    assert int(got["sizeof.fdirw_domain"]) == ctypes.sizeof(fd.fdirw_domain)
    assert int(got["sizeof.fdirw_opts"]) == ctypes.sizeof(fd.fdirw_opts)
    assert int(got["sizeof.fdirw_stats"]) == ctypes.sizeof(fd.fdirw_stats)
    assert int(got["sizeof.fdirw_mp_params"]) == ctypes.sizeof(fd.fdirw_mp_params)
    for key, val in got.items():
        t, f = key.split(".")
        if t == "sizeof":
            continue
        cls = getattr(fd, t)
        assert getattr(cls, f).offset == int(val), key


def test_missing_library_fails_loudly(tmp_path):
    import importlib
    saved = fd._lib
    try:
        fd._lib = None
        with pytest.raises(RuntimeError, match="missing"):
            fd.load_library(str(tmp_path / "nope.so"))
    finally:
        fd._lib = saved
