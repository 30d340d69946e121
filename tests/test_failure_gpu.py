"""Failure paths on the GPU, forced from the host so every kernel still ends
normally (errors are collected, not thrown: section 6.1):

- a dispenser wait bound far below what a claim takes makes the GPU's
  waiting workgroups give up: the run ends with CE_E_TIMEOUT naming the
  dispenser (or, if no workgroup had to wait, completes correctly), and the
  next run on the same engine is bit-exact again;
- a runtime payload whose host version fails makes the run return
  CE_E_DEVICE naming the failed items, and the engine runs correctly after."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import paper_1805_02755_amd as ce
from paper_1805_02755_amd import rt_examples, synth
from oracle import oracle as O

from gpu_util import BOTH, check_trace, diff_report, escape_params, run_payload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    e = ce.Engine()
    yield e
    e.close()


@pytest.fixture(scope="module")
def escape_ref():
    p = synth.escape_small()
    return p, O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)


@pytest.mark.parametrize("sched", ["dynamic", "hguided", "dynamic50"])
def test_tiny_dispenser_bound(eng, escape_ref, sched):
    p, ref = escape_ref
    outcomes = set()
    for _ in range(3):
        eng.wait_bounds(1e-7, 0.0)
        try:
            eng.use(BOTH, 0, 4)
            st = None
            try:
                out, st_, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [p.w, p.h], None, [],
                                           (p.h, p.w), np.uint32, BOTH, sched, host_threads=4)
                st = ce.CE_OK
                assert np.array_equal(out, ref), diff_report(out, ref, tr)
            except ce.CoexecError as ex:
                st = ex.status
                assert st == ce.CE_E_TIMEOUT, ex
                assert any("dispenser" in m for m in ex.messages), ex.messages
            outcomes.add(st)
        finally:
            eng.clear_errors()
            eng.wait_bounds(0.0, 0.0)
        # the engine is whole again: the same run with the default bounds is exact
        out, st_, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [p.w, p.h], None, [], (p.h, p.w),
                                   np.uint32, BOTH, sched, host_threads=4)
        assert np.array_equal(out, ref), diff_report(out, ref, tr)
        check_trace(tr, p.h, 2)
    assert outcomes <= {ce.CE_OK, ce.CE_E_TIMEOUT}


FAILING_HOST = r"""
#include <stdint.h>
typedef struct { void* buf[4]; unsigned char scalars[128]; } rt_args;
/* fails on every call, writing nothing */
int32_t always_fails(uint64_t i0, uint64_t i1, const rt_args* a) { (void)i0; (void)i1; (void)a; return 7; }
"""


@pytest.fixture(scope="module")
def failing_host(tmp_path_factory):
    d = tmp_path_factory.mktemp("fail")
    src = d / "f.c"
    src.write_text(FAILING_HOST)
    so = str(d / "libf.so")
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-o", so, str(src)], check=True, capture_output=True)
    L = C.CDLL(so)
    return L, C.cast(L.always_fails, C.c_void_p).value


@pytest.mark.parametrize("devs", ["host", "both"])
def test_failing_host_version(eng, failing_host, devs):
    import torch
    p = synth.escape_small()
    ref = O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter).ravel()
    n = p.w * p.h
    dm = BOTH if devs == "both" else ce.CE_DEV_HOST
    scal = rt_examples.escape_scalars(p.w, *p.as_f32(), p.max_iter)
    src = rt_examples.source("escape.hiprtc")
    out_d = torch.empty(n, dtype=torch.int32, device="cuda:0")
    out_h = np.empty(n, np.uint32)
    for host_fn, want in ((failing_host[1], ce.CE_E_DEVICE), (rt_examples.host_fn("escape_host"), ce.CE_OK)):
        eng.use(dm, 0, 4)
        eng.work_items([n], [64])
        eng.program_source(src, "escape_item", host=host_fn, n_in=0, n_out=1, out_item_bytes=4, scalars=scal)
        if devs == "both":
            eng.program_out(0, dev=out_d, nbytes=n * 4)
        else:
            eng.program_out(0, host=out_h)
        # a fixed share for the host, so its version surely runs (with Dynamic
        # packages the GPU's batched claims may leave it none)
        if devs == "both":
            eng.scheduler(kind=ce.CE_SCHED_STATIC, props=[0.75], order=ce.CE_ORDER_GPU_FIRST)
        else:
            eng.scheduler(kind=ce.CE_SCHED_DYNAMIC, package_granules=256)
        st = eng.run_status()
        msgs = eng.errors()
        eng.clear_errors()
        assert st == want, (st, msgs)
        if want == ce.CE_E_DEVICE:
            assert any("host version failed with code 7" in m for m in msgs), msgs
        else:
            got = out_d.cpu().numpy().view(np.uint32) if devs == "both" else out_h
            assert np.array_equal(got, ref)
