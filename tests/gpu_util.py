"""Helpers for the GPU tests: run one payload through the C ABI with a given
device set, scheduler and buffer residency."""
import numpy as np
import torch

import paper_1805_02755_amd as ce

DEV = torch.device("cuda:0")
BOTH = ce.CE_DEV_GPU | ce.CE_DEV_HOST

SCHEDULES = {
    "static": dict(kind=ce.CE_SCHED_STATIC, props=[0.75], order=ce.CE_ORDER_HOST_FIRST),
    "static_rev": dict(kind=ce.CE_SCHED_STATIC, props=[0.75], order=ce.CE_ORDER_GPU_FIRST),
    "static8": dict(kind=ce.CE_SCHED_STATIC, props=[0.875], order=ce.CE_ORDER_HOST_FIRST, n_packages=8),
    "dynamic": dict(kind=ce.CE_SCHED_DYNAMIC, package_granules=4),
    "dynamic50": dict(kind=ce.CE_SCHED_DYNAMIC, n_packages=50),
    "hguided": dict(kind=ce.CE_SCHED_HGUIDED, power=[16, 1], k=2, min_granules=[8, 1]),
    "hguided_default": dict(kind=ce.CE_SCHED_HGUIDED, power=[40, 1], k=2),
}


def _sched_for(name, devs):
    s = dict(SCHEDULES[name])
    if devs != BOTH:
        # one device: drop the per-device arrays down to one entry
        for key in ("props",):
            s.pop(key, None)
        for key in ("power", "min_granules"):
            if key in s:
                s[key] = s[key][:1]
    return s


def run_payload(eng, kernel_id, params, gws, lws, inputs, out_shape, out_dtype, devs, sched, mode="dev",
                host_threads=0, merge=ce.CE_MERGE_DMA):
    """inputs: list of numpy arrays. mode: 'dev' (device-resident in and out,
    host mirror of inputs), 'host' (host pointers only), 'pinned' (host
    pointers only, into pinned host memory the GPU reads and writes over
    PCIe), 'both' (everything bound on both sides). Returns (output ndarray,
    stats, trace)."""
    if mode == "pinned":
        inputs = [pinned_copy(a) for a in inputs]
    eng.use(devs, 0, host_threads)
    eng.output_merge(merge)
    eng.work_items(gws, lws)
    eng.scheduler(**_sched_for(sched, devs))
    eng.program_kernel(kernel_id, params)
    keep = []
    for slot, a in enumerate(inputs):
        if mode in ("host", "pinned"):
            eng.program_in(slot, host=a)
        else:
            d = torch.from_numpy(a).to(DEV)
            keep.append(d)
            eng.program_in(slot, host=a, dev=d, nbytes=a.nbytes)
    torch.cuda.synchronize()
    nbytes_out = int(np.prod(out_shape)) * np.dtype(out_dtype).itemsize
    out_h = (np.full(nbytes_out, 0xFF, dtype=np.uint8).view(out_dtype).reshape(out_shape)
             if mode in ("host", "both") else None)
    if mode == "pinned":
        out_h = pinned_copy(np.full(nbytes_out, 0xFF, dtype=np.uint8)).view(out_dtype).reshape(out_shape)
    out_d = None
    if mode in ("dev", "both"):
        nbytes = int(np.prod(out_shape)) * np.dtype(out_dtype).itemsize
        out_d = torch.full((nbytes,), 0xFF, dtype=torch.uint8, device=DEV)
        torch.cuda.synchronize()
    eng.program_out(0, host=out_h, dev=out_d,
                    nbytes=(out_h.nbytes if out_h is not None else out_d.numel()))
    eng.run()
    st = eng.stats()
    tr = eng.trace()
    if mode in ("host", "pinned"):
        res = out_h
    else:
        res = out_d.cpu().numpy().view(out_dtype).reshape(out_shape)
        if mode == "both":
            assert np.array_equal(res.view(np.uint8), out_h.view(np.uint8)), "host and device copies differ"
    del keep
    return res, st, tr


_PINNED_KEEP = []


def pinned_copy(a):
    """A copy of a numpy array in pinned host memory (hipHostMalloc through
    torch); the tensor is kept alive for the module's lifetime."""
    t = torch.empty(a.nbytes, dtype=torch.uint8, pin_memory=True)
    _PINNED_KEEP.append(t)
    if len(_PINNED_KEEP) > 64:
        del _PINNED_KEEP[:32]
    v = t.numpy().view(a.dtype).reshape(a.shape)
    v[...] = a
    return v


def diff_report(out, ref, tr=None):
    """Text naming where two 2-D (rows x items) outputs differ, for assertion
    messages: mismatching rows, whether they hold the untouched fill
    pattern, and which device's package covered them in the trace."""
    a = np.ascontiguousarray(out).view(np.uint32).reshape(out.shape[0], -1)
    b = np.ascontiguousarray(ref).view(np.uint32).reshape(ref.shape[0], -1)
    bad = np.nonzero((a != b).any(axis=1))[0]
    lines = [f"{len(bad)} of {a.shape[0]} rows differ: {bad[:24].tolist()}"]
    for r in bad[:6]:
        cols = np.nonzero(a[r] != b[r])[0]
        unfilled = int((a[r, cols] == 0xFFFFFFFF).sum())
        lines.append(f"row {r}: {len(cols)} items differ (first {cols[:8].tolist()}), {unfilled} still 0xFFFFFFFF, "
                     f"got {a[r, cols[:3]].tolist()} want {b[r, cols[:3]].tolist()}")
    if tr is not None:
        lines.append("trace (device, begin, end): " + str([(d, b_, e) for d, b_, e, _, _ in tr][:64]))
    return "\n".join(lines)


def check_trace(tr, G, n_dev):
    """Packages of the trace cover [0, G) exactly once; devices are valid."""
    cnt = np.zeros(G, dtype=np.int32)
    for d, b, e, tc, te in tr:
        assert 0 <= d < n_dev
        assert 0 <= b < e <= G
        cnt[b:e] += 1
    assert np.all(cnt == 1), (int((cnt == 0).sum()), int((cnt > 1).sum()))


def escape_params(p):
    return ce.ce_escape_params(p.w, p.h, *p.as_f32(), p.max_iter)
