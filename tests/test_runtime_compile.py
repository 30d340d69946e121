"""Runtime payload sources compile for gfx950 with hipRTC on the CPU (no GPU
needed); compile errors come back with the compiler's log; the host versions
build and compute the escape-time definition on their own."""
import ctypes as C
import struct

import numpy as np

import paper_1805_02755_amd as ce
from oracle import oracle as O

from paper_1805_02755_amd import rt_examples as rt_util


def test_payload_sources_compile():
    for name, entry in (("escape.hiprtc", "escape_item"), ("axpy2.hiprtc", "axpy2_item")):
        st, log = ce.ce_rt_compile_check(rt_util.source(name), entry)
        assert st == ce.CE_OK, log


def test_compile_errors_return_the_log():
    st, log = ce.ce_rt_compile_check("__device__ void f(uint64_t i, const ce_rt_args* a) { g(i); }", "f")
    assert st == ce.CE_E_INVALID and "payload.hip" in log and "undeclared" in log
    st, log = ce.ce_rt_compile_check("__device__ void f(uint64_t i, const ce_rt_args* a) {}", "f(")
    assert st == ce.CE_E_INVALID and "identifier" in log
    # the entry must have the work-item signature
    st, log = ce.ce_rt_compile_check("__device__ void f(int i) {}", "f")
    assert st == ce.CE_E_INVALID


class _Args(C.Structure):
    _fields_ = [("buf", C.c_void_p * 4), ("scalars", C.c_ubyte * 128)]


def test_host_escape_version_matches_the_oracle():
    w, h, it = 64, 23, 100
    x0, y0, dx, dy = -2.1, -1.3, 2.7 / 64, 2.6 / 23
    out = np.zeros(w * h, np.uint32)
    a = _Args()
    a.buf[0] = out.ctypes.data
    sc = rt_util.escape_scalars(w, x0, y0, dx, dy, it)
    C.memmove(a.scalars, sc, len(sc))
    fn = rt_util.host_lib().escape_host
    fn.argtypes = [C.c_uint64, C.c_uint64, C.POINTER(_Args)]
    fn(0, 700, C.byref(a))
    fn(700, w * h, C.byref(a))
    assert np.array_equal(out.reshape(h, w), O.escape(w, h, x0, y0, dx, dy, it))
