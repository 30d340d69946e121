"""Payloads supplied as HIP source at run time (per-device kernels, section
6.2), compiled with hipRTC for gfx950 and co-executed with a separate host
version: the escape-time program bit-exact against the oracle for every
scheduler, device set and residency, ragged granules, the plain launch, a
two-input two-output payload, and a module replaced by another."""
import numpy as np
import pytest
import torch

import paper_1805_02755_amd as ce
from oracle import oracle as O

from gpu_util import BOTH, DEV, _sched_for, check_trace
from paper_1805_02755_amd import rt_examples as rt_util

pytestmark = pytest.mark.gpu
DEVSETS = {"gpu": ce.CE_DEV_GPU, "host": ce.CE_DEV_HOST, "both": BOTH}
X0, Y0, DX, DY = -2.1, -1.3, 2.7 / 256, 2.6 / 97


@pytest.fixture(scope="module")
def eng():
    e = ce.Engine()
    yield e
    e.close()


def program_escape(eng, w, max_iter, gws, lws):
    eng.work_items([gws], [lws])
    return eng.program_source(rt_util.source("escape.hiprtc"), "escape_item", host=rt_util.host_fn("escape_host"),
                              n_in=0, n_out=1, out_item_bytes=4,
                              scalars=rt_util.escape_scalars(w, X0, Y0, DX, DY, max_iter))


def run_escape(eng, w, h, max_iter, lws, devs, sched, mode):
    program_escape(eng, w, max_iter, w * h, lws)
    eng.use(devs, 0, 0)
    eng.scheduler(**_sched_for(sched, devs))
    out_h = np.full(w * h, 0xFFFFFFFF, np.uint32) if mode in ("host", "both") else None
    out_d = torch.full((w * h,), -1, dtype=torch.int32, device=DEV) if mode in ("dev", "both") else None
    torch.cuda.synchronize()
    eng.program_out(0, host=out_h, dev=out_d, nbytes=w * h * 4)
    eng.run()
    st, tr = eng.stats(), eng.trace()
    res = out_h if mode == "host" else out_d.cpu().numpy().view(np.uint32)
    if mode == "both":
        assert np.array_equal(res, out_h)
    return res.reshape(h, w), st, tr


@pytest.mark.parametrize("mode", ["dev", "host", "both"])
@pytest.mark.parametrize("sched", ["static", "dynamic", "hguided"])
@pytest.mark.parametrize("devs", ["gpu", "host", "both"])
def test_runtime_escape_bitexact(eng, devs, sched, mode):
    w, h, it = 256, 97, 200
    ref = O.escape(w, h, X0, Y0, DX, DY, it)
    out, st, tr = run_escape(eng, w, h, it, w, DEVSETS[devs], sched, mode)
    assert np.array_equal(out, ref)
    check_trace(tr, h, st.n_devices)


@pytest.mark.parametrize("lws", [1, 100, 1000, 4096, 24832, 30000])
def test_runtime_escape_ragged_granules(eng, lws):
    # granules that do not divide the space, tiles of 2048 items cut inside granules
    w, h, it = 256, 97, 64
    ref = O.escape(w, h, X0, Y0, DX, DY, it)
    out, st, tr = run_escape(eng, w, h, it, lws, BOTH, "hguided", "dev")
    assert np.array_equal(out, ref)
    check_trace(tr, -(-w * h // lws), st.n_devices)


def test_runtime_plain_launch(eng):
    w, h, it = 1024, 333, 256
    program_escape(eng, w, it, w * h, w)
    out = torch.full((w * h,), -1, dtype=torch.int32, device=DEV)
    eng.bare_run_source(w * h, w, [], [out])
    assert np.array_equal(out.cpu().numpy().view(np.uint32).reshape(h, w), O.escape(w, h, X0, Y0, DX, DY, it))


def test_runtime_two_inputs_two_outputs_and_module_swap(eng):
    n, lws, alpha = 100_003, 256, np.float32(1.7)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(n).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    ref0 = (alpha * x) + y
    ref1 = x - y
    # first an escape payload, then replace it by this one on the same engine
    w, h, it = 256, 10, 32
    out_e, _, _ = run_escape(eng, w, h, it, w, BOTH, "dynamic", "dev")
    assert np.array_equal(out_e, O.escape(w, h, X0, Y0, DX, DY, it))
    eng.work_items([n], [lws])
    eng.program_source(rt_util.source("axpy2.hiprtc"), "axpy2_item", host=rt_util.host_fn("axpy2_host"), n_in=2,
                       n_out=2, in_bytes=[x.nbytes, y.nbytes], out_item_bytes=4,
                       scalars=np.array([alpha], np.float32).tobytes())
    xd, yd = torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV)
    z0 = torch.empty(n, device=DEV)
    z1 = torch.empty(n, device=DEV)
    torch.cuda.synchronize()
    eng.program_in(0, host=x, dev=xd, nbytes=x.nbytes)
    eng.program_in(1, host=y, dev=yd, nbytes=y.nbytes)
    eng.program_out(0, dev=z0, nbytes=n * 4)
    eng.program_out(1, dev=z1, nbytes=n * 4)
    for sched in ("static", "hguided", "dynamic"):
        eng.use(BOTH, 0, 0)
        eng.scheduler(**_sched_for(sched, BOTH))
        z0.fill_(float("nan"))
        z1.fill_(float("nan"))
        torch.cuda.synchronize()
        eng.run()
        assert np.array_equal(z0.cpu().numpy().view(np.uint32), ref0.view(np.uint32)), sched
        assert np.array_equal(z1.cpu().numpy().view(np.uint32), ref1.view(np.uint32)), sched
    # the plain launch of the same module
    z0.zero_()
    z1.zero_()
    eng.bare_run_source(n, lws, [xd, yd], [z0, z1])
    assert np.array_equal(z0.cpu().numpy().view(np.uint32), ref0.view(np.uint32))
    assert np.array_equal(z1.cpu().numpy().view(np.uint32), ref1.view(np.uint32))


@pytest.mark.parametrize("sched", ["dynamic", "hguided"])
def test_runtime_escape_gather_merge(eng, sched):
    # the host's rows reach HBM through gather workgroups of the runtime module's own persistent kernel
    w, h, it = 256, 97, 100
    ref = O.escape(w, h, X0, Y0, DX, DY, it)
    eng.output_merge(ce.CE_MERGE_GPU_GATHER)
    try:
        out, st, tr = run_escape(eng, w, h, it, w, BOTH, sched, "dev")
    finally:
        eng.output_merge(ce.CE_MERGE_DMA)
    assert np.array_equal(out, ref)
    check_trace(tr, h, st.n_devices)


def test_runtime_compile_error_leaves_engine_unbound(eng):
    eng.work_items([1000], [10])
    with pytest.raises(ce.CoexecError) as ei:
        eng.program_source("__device__ void f(uint64_t i, const ce_rt_args* a) { undeclared(i); }", "f", n_out=1)
    assert ei.value.status == ce.CE_E_INVALID and "undeclared" in str(ei.value)
    assert eng.run_status() == ce.CE_E_STATE
