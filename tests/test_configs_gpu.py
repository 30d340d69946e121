"""The benchmark configurations exactly as configured, compared with the
oracle element by element through the C ABI:

- escape-time 1024 x 1024 over [-2, 1] x [-1.5, 1.5], max_iter 256, Static
  split into 8 packages (section 5.3 Static with equal bands) over the GPU and
  ONE host thread, in both delivery orders and every buffer residency;
- n-body with Dynamic packages of one 256-body granule (section 5.3 Dynamic),
  the GPU's persistent kernel plus every host thread, device- and host-resident:
  the full output at 16,384 bodies (64 packages, so GPU claims take many
  one-tile packages at once), and at 65,536 bodies the first and the last body
  of every one of the 256 packages plus one body inside each.

Integer outputs and strict-mode FP32 outputs are bit-exact."""
import numpy as np
import pytest

import paper_1805_02755_amd as ce
from paper_1805_02755_amd import synth
from oracle import oracle as O

from gpu_util import BOTH, SCHEDULES, check_trace, diff_report, escape_params, run_payload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    e = ce.Engine()
    yield e
    e.close()


@pytest.fixture(scope="module")
def escape_ref():
    p = synth.escape_small()
    assert (p.w, p.h, p.max_iter) == (1024, 1024, 256)
    return p, O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)


STATIC8 = {
    "gpu7_host1": dict(kind=ce.CE_SCHED_STATIC, props=[0.875], order=ce.CE_ORDER_HOST_FIRST, n_packages=8),
    "half_rev": dict(kind=ce.CE_SCHED_STATIC, props=[0.5], order=ce.CE_ORDER_GPU_FIRST, n_packages=8),
    "gpu1_host7": dict(kind=ce.CE_SCHED_STATIC, props=[0.125], order=ce.CE_ORDER_HOST_FIRST, n_packages=8),
}


@pytest.mark.parametrize("mode", ["dev", "host", "both"])
@pytest.mark.parametrize("plan", list(STATIC8))
def test_escape_static8_one_host_thread(eng, escape_ref, monkeypatch, mode, plan):
    p, ref = escape_ref
    monkeypatch.setitem(SCHEDULES, "c1", STATIC8[plan])
    out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [p.w, p.h], None, [], (p.h, p.w),
                              np.uint32, BOTH, "c1", mode=mode, host_threads=1)
    assert np.array_equal(out, ref), diff_report(out, ref, tr)
    check_trace(tr, p.h, 2)
    assert st.host_threads == 1
    # eight 128-row bands, each device at least one
    assert len(tr) == 8 and all((e - b) == 128 for _, b, e, _, _ in tr)
    bands = {d: sum(1 for dd, *_ in tr if dd == d) for d in (0, 1)}
    want_gpu = {"gpu7_host1": 7, "half_rev": 4, "gpu1_host7": 1}[plan]
    assert bands[0] == want_gpu and bands[1] == 8 - want_gpu
    assert sum(st.items[:2]) == p.w * p.h


C3_SCHED = dict(kind=ce.CE_SCHED_DYNAMIC, package_granules=1)


@pytest.fixture(scope="module")
def bodies_16k():
    pos = synth.nbody_bodies(16384, seed=0x4B0D1)
    return pos, O.nbody_acc(pos, 1e-6, True)


@pytest.mark.parametrize("mode", ["dev", "host"])
@pytest.mark.parametrize("devs", ["gpu", "both"])
def test_nbody_dynamic_one_granule_full_16384(eng, bodies_16k, monkeypatch, mode, devs):
    pos, ref = bodies_16k
    n = pos.shape[0]
    monkeypatch.setitem(SCHEDULES, "c3", C3_SCHED)
    dm = BOTH if devs == "both" else ce.CE_DEV_GPU
    out, st, tr = run_payload(eng, ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(n, 1e-6, 1), [n], [256], [pos],
                              (n, 4), np.float32, dm, "c3", mode=mode, host_threads=0)
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), diff_report(out, ref, tr)
    check_trace(tr, n // 256, st.n_devices)
    # every package is one granule, whoever ran it
    assert len(tr) == n // 256 and all(e - b == 1 for _, b, e, _, _ in tr)


@pytest.mark.parametrize("mode", ["dev", "host"])
def test_nbody_dynamic_one_granule_65536_every_package(eng, mode, monkeypatch):
    n = 65536
    pos = synth.nbody_bodies(n)
    monkeypatch.setitem(SCHEDULES, "c3", C3_SCHED)
    out, st, tr = run_payload(eng, ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(n, 1e-6, 1), [n], [256], [pos],
                              (n, 4), np.float32, BOTH, "c3", mode=mode, host_threads=0)
    check_trace(tr, 256, 2)
    assert len(tr) == 256
    rng = np.random.default_rng(0xC3)
    inner = rng.integers(1, 255, size=256)
    for g in range(256):
        for i in (g * 256, g * 256 + 255, g * 256 + int(inner[g])):
            want = O.nbody_acc_body(pos, 1e-6, i, True)
            assert np.array_equal(out[i].view(np.uint32), want.view(np.uint32)), (g, i, out[i], want)


@pytest.mark.parametrize("host_threads", [1, 0])
@pytest.mark.parametrize("sched", ["c1", "hguided", "dynamic"])
def test_device_times_lie_inside_the_run(eng, escape_ref, monkeypatch, host_threads, sched):
    """T_d (section 7.3) of each device, mapped from the GPU's clock to the
    host's, ends before the run returns, and the GPU's own span fits it."""
    p, ref = escape_ref
    monkeypatch.setitem(SCHEDULES, "c1", STATIC8["gpu7_host1"])
    for _ in range(5):
        out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [p.w, p.h], None, [], (p.h, p.w),
                                  np.uint32, BOTH, sched, host_threads=host_threads)
        assert np.array_equal(out, ref)
        for d in range(st.n_devices):
            if st.packages[d] == 0:  # a device that got no package has T_d = 0 (G-7)
                assert st.t_device[d] == 0.0
                continue
            assert 0.0 < st.t_device[d] <= st.t_run + 10e-6, (d, st.t_device[d], st.t_run, st.t_gpu_kernel)
        assert st.t_gpu_kernel <= st.t_device[0] + 10e-6, (st.t_gpu_kernel, st.t_device[0])
        for d, b, e, tc, te in tr:
            assert -10e-6 <= tc <= te <= st.t_run + 10e-6, (d, b, e, tc, te, st.t_run)
