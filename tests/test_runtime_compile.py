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


def test_runtime_module_has_no_packed_fp32_or_scratch(tmp_path):
    """The module hipRTC builds is compiled like the library's own device
    code: no packed FP32 instructions, no scratch (private) memory."""
    import os
    import subprocess
    objdump = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "llvm-objdump")
    if not os.path.exists(objdump):
        import pytest
        pytest.skip("llvm-objdump not available")
    for name, entry in (("escape.hiprtc", "escape_item"), ("axpy2.hiprtc", "axpy2_item")):
        co = ce.ce_rt_code_object(rt_util.source(name), entry)
        path = tmp_path / (entry + ".co")
        path.write_bytes(co)
        asm = subprocess.run([objdump, "-d", "--mcpu=gfx950", str(path)], check=True, capture_output=True,
                             text=True).stdout
        assert "k_persistent" in asm and "k_bare" in asm
        assert "v_fma_f32" in asm or "v_mul_f32" in asm or "v_add_f32" in asm
        for bad in ("v_pk_fma_f32", "v_pk_mul_f32", "v_pk_add_f32", "scratch_store", "scratch_load"):
            assert bad not in asm, (name, bad)
