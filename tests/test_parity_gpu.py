"""Parity of the HIP + host co-execution path with the oracle, through the C
ABI. Integer outputs and strict-mode FP32 outputs must be bit-exact (the
payloads fix one FP32 operation sequence); fast-mode n-body is checked with
the scale-aware bound ||a - a_ref|| <= 1e-5 * sum_j ||term_ij||."""
import numpy as np
import pytest
import torch

import paper_1805_02755_amd as ce
from paper_1805_02755_amd import synth
from oracle import oracle as O

from gpu_util import BOTH, DEV, SCHEDULES, check_trace, diff_report, escape_params, run_payload

pytestmark = pytest.mark.gpu

DEVSETS = {"gpu": ce.CE_DEV_GPU, "host": ce.CE_DEV_HOST, "both": BOTH}


@pytest.fixture(scope="module")
def eng():
    e = ce.Engine()
    yield e
    e.close()


@pytest.fixture(scope="module")
def escape_small_ref():
    p = synth.escape_small()
    return p, O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)


# ------------------------------------------------------------------ escape
@pytest.mark.parametrize("devs", ["gpu", "host", "both"])
@pytest.mark.parametrize("sched", ["static8", "static_rev", "dynamic", "dynamic50", "hguided", "hguided_default"])
def test_escape_1024_all_schedules(eng, escape_small_ref, devs, sched):
    p, ref = escape_small_ref
    out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [p.w, p.h], None, [], (p.h, p.w),
                              np.uint32, DEVSETS[devs], sched)
    assert np.array_equal(out, ref), diff_report(out, ref, tr)
    check_trace(tr, p.h, st.n_devices)
    assert sum(st.granules[:st.n_devices]) == p.h
    assert sum(st.items[:st.n_devices]) == p.w * p.h
    assert 0.0 <= st.balance <= 1.0


@pytest.mark.parametrize("mode", ["dev", "host", "both"])
def test_escape_ragged_residency(eng, mode):
    p = synth.escape_region(333, 77, -1.9, 0.7, -1.1, 1.3, 700)
    ref = O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)
    for sched in ("hguided", "dynamic", "static"):
        out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [p.w, p.h], None, [], (p.h, p.w),
                                  np.uint32, BOTH, sched, mode=mode)
        assert np.array_equal(out, ref), (sched, diff_report(out, ref, tr))
        check_trace(tr, p.h, 2)


@pytest.mark.parametrize("w,h", [(1, 1), (1, 9), (7, 1), (64, 16), (65, 17), (2048, 3)])
def test_escape_edge_shapes(eng, w, h):
    p = synth.escape_region(w, h, -2.0, 0.5, -1.0, 1.0, 300)
    ref = O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)
    for devs in ("gpu", "both"):
        out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [w, h], None, [], (h, w), np.uint32,
                                  DEVSETS[devs], "hguided")
        assert np.array_equal(out, ref)
        check_trace(tr, h, st.n_devices)


# -------------------------------------------------------------------- blur
@pytest.mark.parametrize("w,h", [(1, 1), (2, 3), (5, 5), (203, 77), (1001, 37), (1024, 40), (4099, 23), (3, 2000)])
def test_blur_shapes(eng, w, h):
    img = synth.blur_image(w, h, seed=w * 7919 + h)
    wt = ce.ce_gauss5_weights(1.0)
    ref = O.blur5(img, O.gauss5_weights(1.0))
    for devs in ("gpu", "host", "both"):
        for sched in ("hguided", "dynamic", "static_rev"):
            out, st, tr = run_payload(eng, ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(w, h), [w, h], None, [img, wt],
                                      (h, w), np.float32, DEVSETS[devs], sched)
            assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), (devs, sched, diff_report(out, ref, tr))
            check_trace(tr, h, st.n_devices)


def test_blur_asymmetric_weights_host_mode(eng):
    rng = np.random.default_rng(4)
    wt = rng.random(25).astype(np.float32)
    img = synth.blur_image(517, 61, seed=77)
    ref = O.blur5(img, wt)
    out, st, tr = run_payload(eng, ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(517, 61), [517, 61], None, [img, wt],
                              (61, 517), np.float32, BOTH, "dynamic", mode="host")
    assert np.array_equal(out, ref)


def test_blur_full_size_8192(eng):
    w = h = 8192
    img = synth.blur_image(w, h)
    wt = ce.ce_gauss5_weights(1.0)
    ref = O.blur5(img, O.gauss5_weights(1.0))
    out, st, tr = run_payload(eng, ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(w, h), [w, h], None, [img, wt], (h, w),
                              np.float32, BOTH, "hguided_default")
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), diff_report(out, ref, tr)
    check_trace(tr, h, 2)


# ------------------------------------------------------------------ n-body
@pytest.mark.parametrize("n", [1, 7, 256, 1000, 4097])
def test_nbody_strict_bitexact(eng, n):
    pos = synth.nbody_bodies(n, seed=n)
    ref = O.nbody_acc(pos, 1e-6, True)
    G = (n + 255) // 256
    for devs in ("gpu", "host", "both"):
        for sched in ("dynamic", "hguided", "static"):
            out, st, tr = run_payload(eng, ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(n, 1e-6, 1), [n], [256], [pos],
                                      (n, 4), np.float32, DEVSETS[devs], sched)
            assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), (devs, sched, diff_report(out, ref, tr))
            check_trace(tr, G, st.n_devices)


def test_nbody_fast_within_tolerance(eng):
    n = 2000
    pos = synth.nbody_bodies(n, seed=12)
    eps2 = 1e-6
    out, st, tr = run_payload(eng, ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(n, eps2, 0), [n], [256], [pos],
                              (n, 4), np.float32, BOTH, "dynamic")
    p = pos.astype(np.float64)
    ref = O.nbody_acc_f64(pos, eps2)
    d = p[None, :, :3] - p[:, None, :3]
    r2 = (d ** 2).sum(-1) + eps2
    scale = (p[None, :, 3] * np.sqrt((d ** 2).sum(-1)) / r2 ** 1.5).sum(1)
    err = np.linalg.norm(out[:, :3].astype(np.float64) - ref, axis=1)
    assert np.all(err <= 1e-5 * scale)
    assert np.all(out[:, 3] == 0)


def test_nbody_full_size_sampled(eng):
    n = 65536
    pos = synth.nbody_bodies(n)
    out, st, tr = run_payload(eng, ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(n, 1e-6, 1), [n], [256], [pos],
                              (n, 4), np.float32, BOTH, "dynamic")
    check_trace(tr, 256, 2)
    rng = np.random.default_rng(8)
    idx = list(rng.choice(n, 96, replace=False)) + [0, 255, 256, n - 1]
    for i in idx:
        assert np.array_equal(out[i].view(np.uint32), O.nbody_acc_body(pos, 1e-6, int(i), True).view(np.uint32)), i


# ------------------------------------------------- invariance and baseline
def test_schedule_invariance_bytes(eng):
    p = synth.escape_region(640, 480, -0.8, -0.6, 0.0, 0.2, 2000)
    outs = []
    for devs in ("gpu", "host", "both"):
        for sched in SCHEDULES:
            o, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [p.w, p.h], None, [], (p.h, p.w),
                                    np.uint32, DEVSETS[devs], sched)
            outs.append(o.copy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_bare_run_matches_oracle():
    p = synth.escape_small()
    out = torch.empty((p.h, p.w), dtype=torch.int32, device=DEV)
    ce.ce_bare_run(ce.CE_KERNEL_ESCAPE, escape_params(p), [], out)
    ref = O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref)
    img = synth.blur_image(777, 333, seed=1)
    wt = ce.ce_gauss5_weights(1.0)
    i_d, w_d = torch.from_numpy(img).to(DEV), torch.from_numpy(wt).to(DEV)
    o_d = torch.empty_like(i_d)
    ce.ce_bare_run(ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(777, 333), [i_d, w_d], o_d)
    assert np.array_equal(o_d.cpu().numpy(), O.blur5(img, O.gauss5_weights(1.0)))
    pos = synth.nbody_bodies(900, seed=2)
    p_d = torch.from_numpy(pos).to(DEV)
    o_d = torch.empty_like(p_d)
    ce.ce_bare_run(ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(900, 1e-6, 1), [p_d], o_d)
    assert np.array_equal(o_d.cpu().numpy(), O.nbody_acc(pos, 1e-6, True))


# ------------------------------------------------------------ error paths
def test_error_paths(eng):
    eng.clear_errors()
    e2 = ce.Engine()
    assert e2.run_status() == ce.CE_E_STATE  # nothing bound
    assert ce.lib().ce_engine_has_errors(e2._h)
    with pytest.raises(ce.CoexecError) as ei:
        e2.use(0)
    assert ei.value.status == ce.CE_E_INVALID
    e2.program_kernel(ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(16, 16))
    with pytest.raises(ce.CoexecError) as ei:
        e2.program_in(0, host=np.zeros(10, np.float32))
    assert ei.value.status == ce.CE_E_INVALID
    with pytest.raises(ce.CoexecError) as ei:
        e2.program_out_pattern(1, 255)
    assert ei.value.status == ce.CE_E_UNSUPPORTED
    e2.use(ce.CE_DEV_GPU)
    e2.work_items([16, 15])
    e2.scheduler(ce.CE_SCHED_DYNAMIC, package_granules=2)
    img = np.zeros((16, 16), np.float32)
    e2.program_in(0, host=img)
    e2.program_in(1, host=np.zeros(25, np.float32))
    e2.program_out(0, host=np.zeros((16, 16), np.float32))
    assert e2.run_status() == ce.CE_E_INVALID  # space does not match the image
    with pytest.raises(ce.CoexecError):
        e2.program_kernel(ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(10, 0.0, 1))
    # empty index spaces are refused, not run
    for kid, prm in ((ce.CE_KERNEL_ESCAPE, ce.ce_escape_params(0, 4, -2, -1, 0.01, 0.01, 8)),
                     (ce.CE_KERNEL_ESCAPE, ce.ce_escape_params(4, 0, -2, -1, 0.01, 0.01, 8)),
                     (ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(0, 0)),
                     (ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(0, 1e-6, 1))):
        with pytest.raises(ce.CoexecError) as ei:
            e2.program_kernel(kid, prm)
        assert ei.value.status == ce.CE_E_INVALID
    e2.close()


# ------------------------------------------------- repeated runs (races)
def test_repeated_coexecution_runs_cover_every_item(eng):
    """Many back-to-back runs of configurations whose GPU workgroups wait for
    packages at the end of the run: every run must write every item (a
    workgroup once paired a stale published-tile count with the end flag and
    left with a ticket that had been published)."""
    p = synth.escape_small()
    ref_e = O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)
    img = synth.blur_image(1024, 40, seed=1024 * 7919 + 40)
    wt = ce.ce_gauss5_weights(1.0)
    ref_b = O.blur5(img, O.gauss5_weights(1.0))
    pr = synth.escape_region(333, 77, -1.9, 0.7, -1.1, 1.3, 700)  # ragged rows share cache lines
    ref_r = O.escape(pr.w, pr.h, *[float(v) for v in pr.as_f32()], pr.max_iter)
    for rep in range(12):
        merge = (ce.CE_MERGE_DMA, ce.CE_MERGE_GPU_GATHER)[rep % 2]
        for sched in ("dynamic", "hguided"):
            out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(pr), [pr.w, pr.h], None, [],
                                      (pr.h, pr.w), np.uint32, BOTH, sched, merge=merge)
            assert np.array_equal(out, ref_r), (rep, sched, merge, diff_report(out, ref_r, tr))
        for sched in ("static8", "hguided", "dynamic"):
            out, st, tr = run_payload(eng, ce.CE_KERNEL_ESCAPE, escape_params(p), [p.w, p.h], None, [], (p.h, p.w),
                                      np.uint32, BOTH, sched, merge=merge)
            assert np.array_equal(out, ref_e), (rep, sched, diff_report(out, ref_e, tr))
            out, st, tr = run_payload(eng, ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(1024, 40), [1024, 40], None,
                                      [img, wt], (40, 1024), np.float32, BOTH, sched, merge=merge)
            assert np.array_equal(out.view(np.uint32), ref_b.view(np.uint32)), (rep, sched, diff_report(out, ref_b, tr))


@pytest.mark.parametrize("merge", [ce.CE_MERGE_DMA, ce.CE_MERGE_GPU_GATHER])
def test_output_merge_modes_ragged(eng, merge):
    """Both ways of moving the host's share into a device-resident output, on
    ragged shapes whose rows share cache lines across package boundaries."""
    for (w, h) in [(203, 77), (1001, 37), (4099, 23)]:
        img = synth.blur_image(w, h, seed=w + 3 * h)
        ref = O.blur5(img, O.gauss5_weights(1.0))
        for sched in ("hguided", "dynamic", "static_rev"):
            out, st, tr = run_payload(eng, ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(w, h), [w, h], None,
                                      [img, ce.ce_gauss5_weights(1.0)], (h, w), np.float32, BOTH, sched, merge=merge)
            assert np.array_equal(out.view(np.uint32), ref.view(np.uint32)), (w, h, sched, diff_report(out, ref, tr))
    n = 3000
    pos = synth.nbody_bodies(n, seed=31)
    ref = O.nbody_acc(pos, 1e-6, True)
    out, st, tr = run_payload(eng, ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(n, 1e-6, 1), [n], [256], [pos], (n, 4),
                              np.float32, BOTH, "hguided", merge=merge)
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))


def test_dma_output_seen_by_later_kernels(eng):
    """Host rows copied into HBM by the copy engines are read correctly by the
    next kernel on the caller's stream, also where the same buffer's lines
    were just written by a GPU kernel (a fill) and may sit in the GPU's caches."""
    w, h = 1001, 37
    img = synth.blur_image(w, h, seed=w + 3 * h)
    wt = ce.ce_gauss5_weights(1.0)
    ref = torch.from_numpy(O.blur5(img, O.gauss5_weights(1.0)).view(np.int32)).to(DEV)
    img_d, wt_d = torch.from_numpy(img).to(DEV), torch.from_numpy(wt).to(DEV)
    out = torch.empty((h, w), dtype=torch.int32, device=DEV)
    eng.use(BOTH, 0, 4)
    eng.output_merge(ce.CE_MERGE_DMA)
    eng.work_items([w, h])
    eng.program_kernel(ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(w, h))
    eng.program_in(0, host=img, dev=img_d, nbytes=img.nbytes)
    eng.program_in(1, host=wt, dev=wt_d, nbytes=wt.nbytes)
    eng.program_out(0, dev=out, nbytes=out.numel() * 4)
    copied = 0
    for rep in range(16):
        sched = ("hguided", "dynamic", "static", "static_rev")[rep % 4]
        eng.scheduler(**SCHEDULES[sched])
        out.fill_(-1 - rep)  # a kernel writes every line of the buffer
        torch.cuda.synchronize()
        eng.run()
        copied += eng.stats().gathered_bytes
        same = torch.eq(out, ref).all().item()  # read by a kernel on the caller's stream
        assert same, (rep, sched, int((out != ref).sum().item()))
    assert copied > 0  # the host did take rows
