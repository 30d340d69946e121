#!/usr/bin/env python3
"""Co-execution bench on one MI355X plus the host CPU cores.

Default workload: 5x5 Gaussian blur of an 8192 x 8192 FP32 image (pixels
uniform in [0, 1), seed 0xB1), HGuided scheduler, GPU + every host core. A
step is one ce_engine_run over the whole image. `value` is K steps timed back
to back with inputs resident in HBM (and mirrored in host memory for the host
workers) and the output ending in HBM (the host's rows copied in by the SDMA
engines during the run).

Beside it, on the same line:
- the measurement protocol of section 7.3: three sets of runs with the first
  of each set discarded (20 runs per set; 100 for the overhead), median, p5
  and p95 of the plain single-GPU launch, the engine with the GPU alone, the
  host alone and the co-execution; speedup, S_max, efficiency and balance of
  section 7.3 from those medians; the work each device took;
- the host-resident run (section 7.3's T includes the transfers): the same
  image in pinned host buffers, which the GPU streams over PCIe, against the
  best plain single-GPU launch with its transfers;
- the roofline of the persistent GPU kernel (HIP events on its stream) and a
  streaming-copy reference, and the oracle timed on one host core.

Other workloads (--workload): escape (1024^2, max_iter 256, Static split into
8 packages over the GPU and ONE host thread, as configured; HGuided over every
core beside it), nbody (65,536 bodies, Dynamic 256-body packages, GPU + every
core; the hardware 1/sqrt beside the strict one), escape-roofline (8192^2,
max_iter 4096, GPU), runtime, nbody-step, binomial, batch, serve, copy.
--sched-grid adds the paper's scheduler grid (Static, Static rev, Dynamic 50
and 150 packages, HGuided) and --sweep the overhead and the co-execution
efficiency against problem size.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "work-items/s co-executed (GPU+host) vs plain 1-GPU launch; balance efficiency"
HBM_PEAK_GBS = 8000.0
# Published dense FP32 vector peak (it counts packed FP32, two lanes' FMAs per
# instruction); this build issues no packed FP32, so each lane retires at most
# one FMA (two flops) per clock: half of it.
FP32_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 78.6
# VALU issue rate without packed FP32: 256 CUs x 64 lanes per clock x 2.4 GHz.
VALU_ISSUE_TOPS = 256 * 64 * 2.4e9 / 1e12
# Section 7.3's protocol: sets of runs, the first run of each set discarded.
SETS, RUNS, OVERHEAD_RUNS = 3, 20, 100

DEVICE_SOURCES = ("paper_1805_02755_amd/csrc/kernels.hip", "paper_1805_02755_amd/csrc/device_tiles.hpp",
                  "paper_1805_02755_amd/csrc/device_atomics.hpp", "paper_1805_02755_amd/csrc/device_payloads.hpp",
                  "paper_1805_02755_amd/csrc/common.hpp", "paper_1805_02755_amd/csrc/sched_device.hpp",
                  "paper_1805_02755_amd/csrc/rt_tile.hpp")


def measured(name):
    """A committed counter summary (profiles/NAME, JSON) if the device sources
    it was taken from are unchanged, else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec.get("device_sources", DEVICE_SOURCES):
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("device_source_sha256"):
        return None
    return rec


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="blur",
                    choices=["blur", "escape", "escape-roofline", "runtime", "nbody", "nbody-step", "binomial",
                             "batch", "serve", "copy"])
    ap.add_argument("--serve-jobs", type=int, default=2000)
    ap.add_argument("--trace-out", default=None,
                    help="write the last co-executed run's package trace here (Chrome trace JSON)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-host-resident", action="store_true", help="skip the host-resident leg")
    ap.add_argument("--sched-grid", action="store_true", help="add the scheduler grid of section 7.3")
    ap.add_argument("--sweep", action="store_true",
                    help="add the overhead and the co-execution efficiency against problem size")
    ap.add_argument("--merge", choices=["dma", "gpu"], default="dma",
                    help="how the host's share reaches a device output: the GPU's copy engines (dma) or "
                         "gather workgroups inside its kernel (gpu)")
    ap.add_argument("--host-threads", type=int, default=0)
    ap.add_argument("--quick", action="store_true",
                    help="one set of two runs per quantity (for profilers; not the protocol of section 7.3)")
    return ap.parse_args()


class HipEvents:
    """Raw hipEvent_t handles from the HIP runtime, recorded by the engine on
    the stream its kernel runs on."""

    def __init__(self):
        import ctypes as C
        self.C = C
        self.L = C.CDLL("libamdhip64.so")
        self.L.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.L.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.L.hipEventSynchronize.argtypes = [C.c_void_p]
        self.L.hipEventDestroy.argtypes = [C.c_void_p]
        self.L.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
        self.L.hipHostGetDevicePointer.argtypes = [C.POINTER(C.c_void_p), C.c_void_p, C.c_uint]

    def create(self):
        ev = self.C.c_void_p()
        if self.L.hipEventCreate(self.C.byref(ev)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return ev.value

    def elapsed_ms(self, a, b):
        f = self.C.c_float()
        if self.L.hipEventSynchronize(b) != 0 or self.L.hipEventElapsedTime(self.C.byref(f), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(f.value)

    def record(self, ev, stream):
        if self.L.hipEventRecord(ev, stream) != 0:
            raise RuntimeError("hipEventRecord failed")

    def destroy(self, ev):
        self.L.hipEventDestroy(ev)

    def device_view(self, host_ptr):
        """The GPU's address of pinned host memory."""
        d = self.C.c_void_p()
        if self.L.hipHostGetDevicePointer(self.C.byref(d), self.C.c_void_p(host_ptr), 0) != 0:
            raise RuntimeError("hipHostGetDevicePointer failed")
        return d.value


def timed_runs(fn, warmup, steps, sync):
    for _ in range(warmup):
        fn()
    sync()
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return ts


def med(v):
    return statistics.median(v) if v else float("nan")


def pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=float), q)) if v else float("nan")


def dist_ms(v):
    """Median, p5 and p95 (ms) of run times in seconds."""
    return {"median_ms": med(v) * 1e3, "p5_ms": pct(v, 5) * 1e3, "p95_ms": pct(v, 95) * 1e3, "runs": len(v)}


def protocol(fn, sets=None, per_set=None, after=None):
    """Section 7.3: `sets` sets of per_set + 1 runs, the first of each set
    discarded. Returns the kept run times (s) and after()'s value per kept run."""
    sets = SETS if sets is None else sets
    per_set = RUNS if per_set is None else per_set
    times, extra = [], []
    for _ in range(sets):
        for i in range(per_set + 1):
            t0 = time.perf_counter()
            fn()
            dt = time.perf_counter() - t0
            if i == 0:
                continue
            times.append(dt)
            if after is not None:
                extra.append(after())
    return times, extra


def runs_for(t_one, budget_s, lo=2, hi=None):
    """Runs per set that fit the sets into budget_s, given one run's time."""
    hi = RUNS if hi is None else hi
    return int(max(min(lo, hi), min(hi, budget_s / max(1e-9, SETS * t_one))))


def chrome_trace(trace, stats, path, title):
    """The package trace as Chrome trace events (chrome://tracing, Perfetto):
    one row per device, one slice per package, times in microseconds from
    the start of the run."""
    names = {0: "GPU", 1: "host"}
    ev = [{"ph": "M", "name": "process_name", "pid": 0, "args": {"name": title}}]
    for d in sorted({r[0] for r in trace}):
        ev.append({"ph": "M", "name": "thread_name", "pid": 0, "tid": int(d),
                   "args": {"name": names.get(stats.device_kind[d] - 1, str(d)) if hasattr(stats, "device_kind")
                            else str(d)}})
    for d, b, e, tc, te in trace:
        ev.append({"ph": "X", "pid": 0, "tid": int(d), "name": f"granules [{b}, {e})", "ts": tc * 1e6,
                   "dur": max(0.0, (te - tc) * 1e6), "args": {"g0": int(b), "g1": int(e)}})
    for d in range(stats.n_devices):
        ev.append({"ph": "i", "pid": 0, "tid": d, "name": "device end", "ts": stats.t_device[d] * 1e6, "s": "t"})
    with open(path, "w") as f:
        json.dump({"traceEvents": ev, "displayTimeUnit": "ms"}, f)


def work_distribution(trace, stats, items_of):
    """Granules, items and package sizes per device of one run (section 8.4)."""
    out = {}
    for d in range(stats.n_devices):
        sizes = sorted(int(e - b) for dd, b, e, _, _ in trace if dd == d)
        kind = "gpu" if stats.device_kind[d] == 1 else "host"
        out[kind] = {"packages": len(sizes), "granules": int(sum(sizes)),
                     "items": int(sum(items_of(b, e) for dd, b, e, _, _ in trace if dd == d)),
                     "package_granules": {"min": sizes[0] if sizes else 0, "median": med(sizes) if sizes else 0,
                                          "max": sizes[-1] if sizes else 0, "first": [int(e - b) for dd, b, e, _, _
                                                                                      in sorted(trace, key=lambda r: r[3])
                                                                                      if dd == d][:8]}}
    return out


# ------------------------------------------------------------------ workloads
class Spec:
    """One workload: its kernel, inputs (host arrays and HBM copies), output,
    index space, configured scheduler and host threads."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def make_spec(wl, args, ce, synth, np, torch, dev, strict=1):
    if wl == "blur":
        w = h = 8192
        log("generating 8192x8192 image")
        img = synth.blur_image(w, h)
        wt = ce.ce_gauss5_weights(1.0)
        return Spec(kid=ce.CE_KERNEL_BLUR5, params=ce.ce_blur5_params(w, h), gws=[w, h], lws=None,
                    ins=[img, wt], out_shape=(h, w), out_dtype=np.float32, n_items=w * h, G=h,
                    items_of=lambda b, e: (e - b) * w, host_threads=args.host_threads,
                    sched=dict(kind=ce.CE_SCHED_HGUIDED, k=2), dtype="f32", bound="hbm",
                    config={"workload": "blur5x5 8192x8192 fp32, sigma 1, clamp-to-edge", "scheduler": "hguided",
                            "devices": "gpu+host", "output_merge": args.merge})
    if wl in ("escape", "runtime"):
        p = synth.escape_small()
        s = Spec(kid=ce.CE_KERNEL_ESCAPE, params=ce.ce_escape_params(p.w, p.h, *p.as_f32(), p.max_iter),
                 gws=[p.w, p.h], lws=None, ins=[], out_shape=(p.h, p.w), out_dtype=np.uint32, n_items=p.w * p.h,
                 G=p.h, items_of=lambda b, e: (e - b) * p.w, host_threads=1,
                 sched=dict(kind=ce.CE_SCHED_STATIC, n_packages=8), dtype="u32", bound="alu", esc=p,
                 config={"workload": "escape-time 1024x1024 over [-2,1]x[-1.5,1.5], max_iter 256",
                         "scheduler": "static, 8 packages", "devices": "gpu+1 host thread"})
        if wl == "runtime":
            s.rt_lws = 64
            s.G = s.n_items // 64
            s.items_of = lambda b, e: (e - b) * 64
            s.host_threads = args.host_threads
            s.sched = dict(kind=ce.CE_SCHED_HGUIDED, k=2)
            s.config = {"workload": s.config["workload"] + ", supplied as HIP source at run time (hipRTC) with a C "
                                    "host version", "granule": "64 pixels", "scheduler": "hguided",
                        "devices": "gpu+host"}
        return s
    n = 65536
    bodies = synth.nbody_bodies(n)
    return Spec(kid=ce.CE_KERNEL_NBODY_ACC, params=ce.ce_nbody_params(n, 1e-6, strict), gws=[n], lws=[256],
                ins=[bodies], out_shape=(n, 4), out_dtype=np.float32, n_items=n, G=n // 256,
                items_of=lambda b, e: (min(e * 256, n) - b * 256), host_threads=args.host_threads,
                sched=dict(kind=ce.CE_SCHED_DYNAMIC, package_granules=1), dtype="f32", bound="alu", exact=bool(strict),
                config={"workload": "nbody acceleration 65536 bodies fp32, eps2 1e-6, "
                                    + ("strict (Lomont) rsqrt" if strict else "hardware rsqrt"),
                        "scheduler": "dynamic 256-body packages", "devices": "gpu+host"})


def coexec_leg(ce, sp, mode, args, stream, hev, torch, np, sched=None, host_threads=None, K=None, events=True):
    """Measures one workload in one residency mode: plain launch, engine
    with the GPU alone, the host alone, the co-execution (section 7.3
    protocol), K timed co-executed steps and the GPU kernel's events.
    mode 'device': inputs and output in HBM (host mirrors of the inputs);
    mode 'host': inputs and output in pinned host buffers only."""
    dev = torch.device("cuda:0")
    sync = torch.cuda.synchronize
    K = K or args.steps
    W = args.warmup
    sched = dict(sched or sp.sched)
    host_threads = sp.host_threads if host_threads is None else host_threads
    nbytes_out = int(np.prod(sp.out_shape)) * np.dtype(sp.out_dtype).itemsize
    keep = []
    if mode == "device":
        ins_dev = [torch.from_numpy(a).to(dev) for a in sp.ins]
        out_dev = torch.empty(nbytes_out, dtype=torch.uint8, device=dev)
        ins_host, out_host = sp.ins, None
        bare_ins, bare_out = ins_dev, out_dev
    else:
        def pinned(a):
            t = torch.empty(a.nbytes, dtype=torch.uint8, pin_memory=True)
            keep.append(t)
            v = t.numpy().view(a.dtype).reshape(a.shape)
            v[...] = a
            return v
        ins_host = [pinned(a) for a in sp.ins]
        out_host = pinned(np.zeros(nbytes_out, np.uint8))
        ins_dev, out_dev = None, None
        # plain launches over the same pinned buffers (read and written over PCIe)
        bare_ins = [hev.device_view(a.ctypes.data) for a in ins_host]
        bare_out = hev.device_view(out_host.ctypes.data)
        # and the plain launch with explicit copies through HBM
        ins_stage = [torch.empty(a.nbytes, dtype=torch.uint8, device=dev) for a in sp.ins]
        out_stage = torch.empty(nbytes_out, dtype=torch.uint8, device=dev)
        ins_pin_t = [torch.from_numpy(a.view(np.uint8).reshape(-1)) for a in ins_host]
        out_pin_t = torch.from_numpy(out_host.view(np.uint8).reshape(-1))
    sync()
    res = {"mode": mode}

    # ------------------------------------------------ plain single-GPU launch
    log(f"[{mode}] plain launch")
    rt = getattr(sp, "rt_lws", None)
    eng = ce.Engine()
    eng.stream(stream.cuda_stream)
    eng.output_merge(ce.CE_MERGE_DMA if args.merge == "dma" else ce.CE_MERGE_GPU_GATHER)
    if rt:
        from paper_1805_02755_amd import rt_examples
        p = sp.esc
        eng.work_items([sp.n_items], [rt])
        t_c = time.perf_counter()
        eng.program_source(rt_examples.source("escape.hiprtc"), "escape_item",
                           host=rt_examples.host_fn("escape_host"), n_in=0, n_out=1, out_item_bytes=4,
                           scalars=rt_examples.escape_scalars(p.w, *p.as_f32(), p.max_iter))
        res["compile_s"] = time.perf_counter() - t_c
    else:
        eng.work_items(sp.gws, sp.lws)
        eng.program_kernel(sp.kid, sp.params)

    def bare_once(sync_=True):
        if rt:
            eng.bare_run_source(sp.n_items, rt, [], [bare_out], stream=stream.cuda_stream, sync=sync_)
        else:
            ce.ce_bare_run(sp.kid, sp.params, bare_ins, bare_out, stream=stream.cuda_stream, sync=sync_)

    for _ in range(W):
        bare_once()
    t_bare, _ = protocol(bare_once, per_set=OVERHEAD_RUNS)
    res["t_bare"] = dist_ms(t_bare)
    T_bare = med(t_bare)
    if mode == "host":
        def bare_copies():
            with torch.cuda.stream(stream):
                for s_, d_ in zip(ins_stage, ins_pin_t):
                    s_.copy_(d_, non_blocking=True)
                ce.ce_bare_run(sp.kid, sp.params, ins_stage, out_stage, stream=stream.cuda_stream, sync=False)
                out_pin_t.copy_(out_stage, non_blocking=True)
            stream.synchronize()
        for _ in range(W):
            bare_copies()
        t_bc, _ = protocol(bare_copies)
        res["t_bare_zero_copy"] = res["t_bare"]
        res["t_bare_with_copies"] = dist_ms(t_bc)
        # the faster plain launch is the baseline
        if med(t_bc) < T_bare:
            T_bare = med(t_bc)
            res["t_bare"] = res["t_bare_with_copies"]
        res["bare_form"] = "copies" if T_bare == med(t_bc) else "zero-copy"
    k_bare = []
    if events and mode == "device":
        ev = [(hev.create(), hev.create()) for _ in range(K)]
        for a, b in ev:
            hev.record(a, stream.cuda_stream)
            bare_once(False)
            hev.record(b, stream.cuda_stream)
        sync()
        k_bare = [hev.elapsed_ms(a, b) for a, b in ev]
        for a, b in ev:
            hev.destroy(a)
            hev.destroy(b)
        res["t_bare_kernel_ms"] = med(k_bare)

    # ------------------------------------------------ bind the engine
    for slot in range(len(sp.ins)):
        if mode == "device":
            eng.program_in(slot, host=ins_host[slot], dev=ins_dev[slot], nbytes=ins_host[slot].nbytes)
        else:
            eng.program_in(slot, host=ins_host[slot])
    if mode == "device":
        eng.program_out(0, dev=out_dev, nbytes=nbytes_out)
    else:
        eng.program_out(0, host=out_host)

    # ------------------------------------------------ engine, GPU alone
    log(f"[{mode}] engine GPU only")
    eng.use(ce.CE_DEV_GPU, 0, 0)
    eng.scheduler(ce.CE_SCHED_STATIC)
    for _ in range(W):
        eng.run()
    t_gpu, _ = protocol(eng.run, per_set=OVERHEAD_RUNS)
    res["t_engine_gpu"] = dist_ms(t_gpu)
    T_gpu = med(t_gpu)
    res["gpu_workgroups"] = eng.stats().gpu_workgroups
    if events:
        ev = [(hev.create(), hev.create()) for _ in range(K)]
        kg = []
        for a, b in ev:
            eng.kernel_events(a, b)
            eng.run()
            kg.append(hev.elapsed_ms(a, b))
        eng.kernel_events(None, None)
        for a, b in ev:
            hev.destroy(a)
            hev.destroy(b)
        res["t_engine_gpu_kernel_ms"] = med(kg)
    if mode == "device":
        ref = out_dev.clone()

    # ------------------------------------------------ engine, host alone
    log(f"[{mode}] engine host only")
    eng.use(ce.CE_DEV_HOST, 0, host_threads)
    eng.scheduler(ce.CE_SCHED_STATIC)
    t0 = time.perf_counter()
    eng.run()
    t_one = time.perf_counter() - t0
    t_host, _ = protocol(eng.run, per_set=runs_for(t_one, 6.0))
    res["t_engine_host"] = dist_ms(t_host)
    T_host = med(t_host)
    res["host_threads"] = eng.stats().host_threads

    # ------------------------------------------------ co-execution
    if sched["kind"] == ce.CE_SCHED_HGUIDED and "power" not in sched:
        # computing powers (G-3): integers proportional to the standalone
        # throughputs, the faster device at 4096
        t_min = min(T_gpu, T_host)
        sched["power"] = [max(1, int(round(4096 * t_min / T_gpu))), max(1, int(round(4096 * t_min / T_host)))]
    elif sched["kind"] == ce.CE_SCHED_STATIC and "props" not in sched:
        # the GPU's share from the standalone times (G-9: default props from calibration)
        sched["props"] = [max(0.0, min(1.0, T_host / (T_gpu + T_host)))]
    log(f"[{mode}] co-execution {sched}")
    eng.use(ce.CE_DEV_GPU | ce.CE_DEV_HOST, 0, host_threads)
    eng.scheduler(**sched)
    for _ in range(W):
        eng.run()
    t0 = time.perf_counter()
    eng.run()
    t_one = time.perf_counter() - t0
    t_co, st_co = protocol(eng.run, per_set=runs_for(t_one, 6.0), after=eng.stats)
    res["t_coexec"] = dist_ms(t_co)
    T_co = med(t_co)
    # K steps back to back, nothing else in the loop: the line's value
    sync()
    t0 = time.perf_counter()
    for _ in range(K):
        eng.run()
    sync()
    T_total = time.perf_counter() - t0
    kern = []
    if events:
        ev = [(hev.create(), hev.create()) for _ in range(K)]
        for a, b in ev:
            eng.kernel_events(a, b)
            eng.run()
            kern.append(hev.elapsed_ms(a, b))
        eng.kernel_events(None, None)
        for a, b in ev:
            hev.destroy(a)
            hev.destroy(b)
        res["t_coexec_kernel_ms"] = med(kern)
    st = eng.stats()
    trace = eng.trace()
    if mode == "device":
        if getattr(sp, "exact", True):
            assert torch.equal(out_dev, ref), "co-executed output differs from the GPU alone"
        res["_out"] = out_dev
    else:
        res["_out"] = out_host
    if args.trace_out and mode == "device":
        chrome_trace(trace, st, args.trace_out, sp.config["workload"])
    # Section 7.3: both speedups are over the fastest single device (the plain
    # GPU launch, or the host alone where it is faster, as with host buffers).
    s_real = min(T_bare, T_host) / T_co
    s_max = min(T_bare, T_host) * (1.0 / T_bare + 1.0 / T_host)
    gpu_items = [s_.items[0] for s_ in st_co]
    res.update({
        "value": sp.n_items * K / T_total, "ms_per_step": T_total / K * 1e3, "steps": K,
        "plain_gpu_items_per_s": sp.n_items / T_bare, "vs_plain_gpu": T_bare / T_co,
        "s_real": s_real, "s_max": s_max, "efficiency": s_real / s_max,
        "balance": med([s_.balance for s_ in st_co]),
        "balance_p5_p95": [pct([s_.balance for s_ in st_co], 5), pct([s_.balance for s_ in st_co], 95)],
        "overhead_pct_gpu_only": (T_gpu - T_bare) / T_bare * 100.0,
        "gpu_share": med(gpu_items) / sp.n_items,
        "packages": {"gpu": med([s_.packages[0] for s_ in st_co]), "host": med([s_.packages[1] for s_ in st_co])},
        "t_device_ms": [med([s_.t_device[0] for s_ in st_co]) * 1e3, med([s_.t_device[1] for s_ in st_co]) * 1e3],
        "scheduler": {k: (list(v) if isinstance(v, (list, tuple)) else v) for k, v in sched.items()},
        "work_distribution": work_distribution(trace, st, sp.items_of),
        "_kern_ms": kern, "_gpu_items": gpu_items,
    })
    eng.close()
    del keep
    return res


def public(d):
    return {k: v for k, v in d.items() if not k.startswith("_")}


def escape_iterations(out_u32, np):
    """Iterations of an escape-time output and the lane efficiency of the
    row-strip tiles: each wave runs 64 consecutive pixels of a row for as many
    iterations as the longest of them, so efficiency = sum of counts /
    sum over 64-pixel strips of 64 x their largest count."""
    c = out_u32.astype(np.int64)
    h, w = c.shape
    pad = (-w) % 64
    cp = np.pad(c, ((0, 0), (0, pad)))
    strips = cp.reshape(h, -1, 64)
    used = int(c.sum())
    issued = int((strips.max(axis=2) * 64).sum())
    # padding lanes of a ragged strip are idle lanes of that wave
    return used, used / issued if issued else 1.0


def alu_roofline(flops, lane_ops, kern_ms, kernel, counters_name=None):
    achieved = flops / (kern_ms * 1e-3) / 1e12
    r = {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
         "frac": achieved / FP32_PEAK_TFLOPS, "frac_of_nonpacked_peak": achieved / FP32_NONPACKED_TFLOPS,
         "traffic": None, "kernel": kernel, "kernel_ms": kern_ms,
         "issue": {"lane_ops": lane_ops, "achieved_T_lane_ops_per_s": lane_ops / (kern_ms * 1e-3) / 1e12,
                   "peak_T_lane_ops_per_s": VALU_ISSUE_TOPS,
                   "frac": lane_ops / (kern_ms * 1e-3) / 1e12 / VALU_ISSUE_TOPS}}
    if counters_name:
        rec = measured(counters_name)
        r["counters"] = {k: rec[k] for k in ("valu_busy", "valu_utilization", "valu_insts_per_dispatch",
                                             "valu_issue_frac_from_counts", "fp32_arith_issue_frac",
                                             "fp32_tflops_from_counts", "kernel_us_median_trace")
                         if k in rec} if rec else None
        if rec:
            r["counters"]["summary"] = "profiles/" + counters_name.replace(".json", ".md")
    return r


def cpu_baseline_for(wl, sp, np, budget=10.0):
    from oracle import oracle as O
    log("oracle CPU baseline")
    t0 = time.perf_counter()
    done = 0
    if wl == "blur":
        wt_o = O.gauss5_weights(1.0)
        passes = 0
        while passes < 4 and time.perf_counter() - t0 < budget:
            O.blur5(sp.ins[0], wt_o)
            passes += 1
        done = passes * sp.n_items
        sample = f"{passes} full passes over the 8192x8192 image"
    elif wl in ("escape", "runtime"):
        p = sp.esc
        passes = 0
        while passes < 40 and time.perf_counter() - t0 < budget:
            O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)
            passes += 1
        done = passes * sp.n_items
        sample = f"{passes} full passes over the 1024x1024 grid"
    else:
        i = 0
        while time.perf_counter() - t0 < budget:
            O.nbody_acc_body(sp.ins[0], 1e-6, i, True)
            i += 1
        done = i
        sample = f"{i} bodies (each against all 65536)"
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "work-items/s", "cores": 1, "kind": "oracle", "sample": sample,
            "seconds": dt}


def copy_reference(ce, torch, stream, hev, nbytes, K):
    """The streaming-copy kernel over nbytes: achievable bandwidth (GB/s)."""
    dev = torch.device("cuda:0")
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        ce.ce_stream_copy(b, a, nbytes, stream=stream.cuda_stream)
    ms = []
    s0, s1 = hev.create(), hev.create()
    for _ in range(K):
        hev.record(s0, stream.cuda_stream)
        ce.ce_stream_copy(b, a, nbytes, stream=stream.cuda_stream, sync=False)
        hev.record(s1, stream.cuda_stream)
        ms.append(hev.elapsed_ms(s0, s1))
    hev.destroy(s0)
    hev.destroy(s1)
    assert torch.equal(a, b)
    return {"kernel": "k_stream_copy (one non-temporal 16-byte load and store per thread)", "bytes": 2 * nbytes,
            "ms_median": med(ms), "GBps": 2 * nbytes / (med(ms) * 1e-3) / 1e9}


def roofline_for(wl, sp, leg, ce, torch, np, stream, hev, K):
    kern = med(leg["_kern_ms"])
    share = med(leg["_gpu_items"]) / sp.n_items
    if wl == "blur":
        bytes_launch = 8.0 * med(leg["_gpu_items"])
        achieved = bytes_launch / (kern * 1e-3) / 1e9
        rec = measured("blur5_8192_hbm_traffic.json")
        ref = copy_reference(ce, torch, stream, hev, 256 << 20, K)
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": rec.get("traffic_bytes_per_dispatch") if rec else None,
                "traffic_unit": "bytes per launch", "kernel": "k_persistent<Blur5Tile>", "kernel_ms": kern,
                "algorithmic_bytes_per_item": 8.0, "algorithmic_bytes_per_launch": bytes_launch,
                "copy_reference": ref, "frac_of_copy": achieved / ref["GBps"]}
    if wl in ("escape", "runtime"):
        out = leg["_out"].cpu().numpy().view(np.uint32).reshape(sp.out_shape)
        iters, eff = escape_iterations(out, np)
        r = alu_roofline(8.0 * iters * share, 8.0 * iters * share, kern,
                         "k_persistent<RtTile> (hipRTC)" if wl == "runtime" else "k_persistent<EscapeTile>",
                         None if wl == "runtime" else "escape_1024_valu.json")
        r.update({"iterations": iters, "flops_per_iteration": 8, "lane_efficiency": eff})
        return r
    n = sp.n_items
    strict = getattr(sp, "exact", True)
    # VALU lane-ops per interaction: 3 subs, 3 fmas, the 1/sqrt (strict: Lomont's
    # estimate and three Newton steps, 12; fast: one v_rsq_f32), 3 muls, 3 fmas
    lane = 24 if strict else 13
    r = alu_roofline(20.0 * n * n * share, lane * n * n * share, kern,
                     "k_persistent<NbodyTile<true>>" if strict else "k_persistent<NbodyTile<false>>",
                     "nbody_65536_valu.json" if strict else "nbody_65536_fast_valu.json")
    r.update({"flops_per_interaction": 20, "lane_ops_per_interaction": lane})
    return r


def main():
    global SETS, RUNS, OVERHEAD_RUNS
    args = parse()
    if args.quick:
        SETS, RUNS, OVERHEAD_RUNS = 1, 2, 2
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1805_02755_amd as ce
    from paper_1805_02755_amd import synth

    ce.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    wl = args.workload
    if wl == "batch":
        return bench_batch(args, ce, synth, torch, np, stream)
    if wl == "serve":
        return bench_serve(args, ce, synth, torch, np, stream)
    if wl == "copy":
        return bench_copy(args, ce, torch, stream)
    if wl == "nbody-step":
        return bench_nbody_step(args, ce, synth, torch, np, stream)
    if wl == "binomial":
        return bench_binomial(args, ce, synth, torch, np, stream)
    if wl == "escape-roofline":
        return bench_escape_roofline(args, ce, synth, torch, np, stream)

    hev = HipEvents()
    sp = make_spec(wl, args, ce, synth, np, torch, dev)
    leg = coexec_leg(ce, sp, "device", args, stream, hev, torch, np)
    roof = roofline_for(wl, sp, leg, ce, torch, np, stream, hev, args.steps)
    res = {
        "metric": METRIC, "value": leg["value"], "unit": "work-items/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": leg["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": sp.dtype,
        "data": "synthetic (seeded SplitMix64 inputs, paper_1805_02755_amd/synth.py)",
        "config": dict(sp.config, residency="device"),
        "roofline": roof,
        "cpu_baseline": None,
        "protocol": {"sets": SETS, "runs_per_set": RUNS, "overhead_runs_per_set": OVERHEAD_RUNS,
                     "first_run_of_each_set_discarded": True, "host_cores": os.cpu_count()},
        "coexec": public(leg),
    }
    if wl == "blur" and not args.no_host_resident:
        hl = coexec_leg(ce, sp, "host", args, stream, hev, torch, np, K=max(3, args.steps // 4))
        res["host_resident"] = dict(public(hl), note="inputs and output in pinned host buffers; the GPU streams its "
                                    "rows over PCIe; T includes every transfer (section 7.3)")
    if wl == "escape":
        hg = coexec_leg(ce, sp, "device", args, stream, hev, torch, np, sched=dict(kind=ce.CE_SCHED_HGUIDED, k=2),
                        host_threads=args.host_threads)
        res["hguided_all_cores"] = public(hg)
    if wl == "nbody":
        fsp = make_spec("nbody", args, ce, synth, np, torch, dev, strict=0)
        fl = coexec_leg(ce, fsp, "device", args, stream, hev, torch, np, K=max(3, args.steps // 2))
        out_fast = fl["_out"].cpu().numpy().view(np.float32).reshape(-1, 4)
        fr = roofline_for("nbody", fsp, fl, ce, torch, np, stream, hev, args.steps)
        res["fast_rsqrt"] = dict(public(fl), roofline=fr, note="v_rsq_f32 on the GPU, 1/sqrtf on the host")
        del out_fast
    if args.sched_grid:
        res["sched_grid"] = sched_grid(ce, sp, args, stream, hev, torch, np)
    if args.sweep:
        res["size_sweep"] = size_sweep(wl, ce, synth, args, stream, torch, np)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_for(wl, sp, np)
    print(json.dumps(res), flush=True)


def sched_grid(ce, sp, args, stream, hev, torch, np):
    """Section 7.3's scheduler configurations on this workload: Static
    (proportions from the standalone times), Static rev, Dynamic with 50 and
    150 packages, HGuided."""
    grid = {"static": dict(kind=ce.CE_SCHED_STATIC, order=ce.CE_ORDER_HOST_FIRST),
            "static_rev": dict(kind=ce.CE_SCHED_STATIC, order=ce.CE_ORDER_GPU_FIRST),
            "dynamic_50": dict(kind=ce.CE_SCHED_DYNAMIC, n_packages=50),
            "dynamic_150": dict(kind=ce.CE_SCHED_DYNAMIC, n_packages=150),
            "hguided": dict(kind=ce.CE_SCHED_HGUIDED, k=2)}
    out = {}
    for name, s in grid.items():
        log(f"scheduler grid: {name}")
        leg = coexec_leg(ce, sp, "device", args, stream, hev, torch, np, sched=s, host_threads=args.host_threads,
                         K=3, events=False)
        out[name] = {k: leg[k] for k in ("s_real", "s_max", "efficiency", "balance", "balance_p5_p95",
                                         "t_coexec", "t_bare", "t_engine_host", "gpu_share", "packages",
                                         "scheduler")}
    return out


def size_sweep(wl, ce, synth, args, stream, torch, np):
    """Overhead and co-execution efficiency across problem sizes (sections
    8.2 and 8.3): at each size the plain launch, the engine with the GPU
    alone, the host alone and HGuided over the GPU and every core (powers
    from the standalone times), each timed by the protocol within a few
    seconds."""
    dev = torch.device("cuda:0")
    rows = []
    if wl == "blur":
        cases = [(s, s) for s in (1024, 2048, 4096, 8192, 16384)]
    elif wl in ("escape", "runtime"):
        cases = [(s, s) for s in (256, 512, 1024, 2048, 4096, 8192)]
    else:
        cases = [(n,) for n in (4096, 8192, 16384, 32768, 65536)]
    for c in cases:
        log(f"size sweep {wl} {c}")
        if wl == "blur":
            w, h = c
            ins_h = [synth.blur_image(w, h, seed=w), ce.ce_gauss5_weights(1.0)]
            kid, prm, gws, lws, items = ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(w, h), [w, h], None, w * h
            out = torch.empty((h, w), dtype=torch.float32, device=dev)
        elif wl in ("escape", "runtime"):
            w, h = c
            p = synth.escape_region(w, h, -2.0, 1.0, -1.5, 1.5, 256)
            ins_h = []
            kid, prm, gws, lws, items = (ce.CE_KERNEL_ESCAPE, ce.ce_escape_params(w, h, *p.as_f32(), 256), [w, h],
                                         None, w * h)
            out = torch.empty((h, w), dtype=torch.int32, device=dev)
        else:
            n = c[0]
            ins_h = [synth.nbody_bodies(n)]
            kid, prm, gws, lws, items = ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(n, 1e-6, 1), [n], [256], n
            out = torch.empty((n, 4), dtype=torch.float32, device=dev)
        ins = [torch.from_numpy(a).to(dev) for a in ins_h]
        torch.cuda.synchronize()
        bare = lambda: ce.ce_bare_run(kid, prm, ins, out, stream=stream.cuda_stream, sync=True)
        for _ in range(3):
            bare()
        t0 = time.perf_counter()
        bare()
        per = runs_for(time.perf_counter() - t0, 3.0, lo=5, hi=OVERHEAD_RUNS)
        tb, _ = protocol(bare, per_set=per)
        eng = ce.Engine()
        eng.stream(stream.cuda_stream)
        eng.work_items(gws, lws)
        eng.program_kernel(kid, prm)
        for s_, (a_, d_) in enumerate(zip(ins_h, ins)):
            eng.program_in(s_, host=a_, dev=d_, nbytes=a_.nbytes)
        eng.program_out(0, dev=out, nbytes=out.numel() * out.element_size())
        eng.use(ce.CE_DEV_GPU, 0, 0)
        eng.scheduler(ce.CE_SCHED_STATIC)
        for _ in range(3):
            eng.run()
        tg, _ = protocol(eng.run, per_set=per)
        eng.use(ce.CE_DEV_HOST, 0, args.host_threads)
        t0 = time.perf_counter()
        eng.run()
        th, _ = protocol(eng.run, per_set=runs_for(time.perf_counter() - t0, 2.0, lo=2))
        T_b, T_g, T_h = med(tb), med(tg), med(th)
        t_min = min(T_g, T_h)
        eng.use(ce.CE_DEV_GPU | ce.CE_DEV_HOST, 0, args.host_threads)
        eng.scheduler(kind=ce.CE_SCHED_HGUIDED, k=2,
                      power=[max(1, int(round(4096 * t_min / T_g))), max(1, int(round(4096 * t_min / T_h)))])
        for _ in range(3):
            eng.run()
        t0 = time.perf_counter()
        eng.run()
        tc, stc = protocol(eng.run, per_set=runs_for(time.perf_counter() - t0, 2.0, lo=2), after=eng.stats)
        eng.close()
        T_c = med(tc)
        s_max = min(T_b, T_h) * (1.0 / T_b + 1.0 / T_h)
        rows.append({"size": list(c), "items": items, "t_bare": dist_ms(tb), "t_engine_gpu": dist_ms(tg),
                     "t_engine_host": dist_ms(th), "t_coexec": dist_ms(tc),
                     "overhead_pct": (T_g - T_b) / T_b * 100.0, "s_real": min(T_b, T_h) / T_c, "s_max": s_max,
                     "efficiency": (min(T_b, T_h) / T_c) / s_max, "balance": med([s_.balance for s_ in stc]),
                     "gpu_share": med([s_.items[0] for s_ in stc]) / items})
        del ins, out
    return rows


def bench_escape_roofline(args, ce, synth, torch, np, stream):
    """The escape-time kernel where it is compute-bound: 8192 x 8192 over
    [-2,1]x[-1.5,1.5], max_iter 4096, on the GPU (plain launch and the engine
    with the GPU alone): FP32 flops and lane efficiency from the iteration
    counts."""
    hev = HipEvents()
    K, W = args.steps, args.warmup
    w = h = 8192
    p = synth.escape_region(w, h, -2.0, 1.0, -1.5, 1.5, 4096)
    prm = ce.ce_escape_params(w, h, *p.as_f32(), p.max_iter)
    dev = torch.device("cuda:0")
    out = torch.empty((h, w), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    ev = [(hev.create(), hev.create()) for _ in range(K)]

    def timed(fn):
        for _ in range(W):
            fn(True)
        ms = []
        for a, b in ev:
            hev.record(a, stream.cuda_stream)
            fn(False)
            hev.record(b, stream.cuda_stream)
            ms.append(hev.elapsed_ms(a, b))
        return ms

    log("escape roofline: plain launch")
    kb = timed(lambda s: ce.ce_bare_run(ce.CE_KERNEL_ESCAPE, prm, [], out, stream=stream.cuda_stream, sync=s))
    ref = out.clone()
    eng = ce.Engine()
    eng.stream(stream.cuda_stream)
    eng.use(ce.CE_DEV_GPU, 0, 0)
    eng.work_items([w, h])
    eng.program_kernel(ce.CE_KERNEL_ESCAPE, prm)
    eng.program_out(0, dev=out, nbytes=out.numel() * 4)
    eng.scheduler(ce.CE_SCHED_STATIC)
    log("escape roofline: engine, GPU alone")
    for _ in range(W):
        eng.run()
    kg = []
    for a, b in ev:
        eng.kernel_events(a, b)
        eng.run()
        kg.append(hev.elapsed_ms(a, b))
    eng.kernel_events(None, None)
    assert torch.equal(out, ref)
    eng.close()
    iters, eff = escape_iterations(out.cpu().numpy().view(np.uint32), np)
    r = alu_roofline(8.0 * iters, 8.0 * iters, med(kg), "k_persistent<EscapeTile>", "escape_8192_4096_valu.json")
    r.update({"iterations": iters, "lane_efficiency": eff, "flops_per_iteration": 8})
    rb = alu_roofline(8.0 * iters, 8.0 * iters, med(kb), "k_bare<EscapeTile>")
    res = {"metric": METRIC, "value": w * h / (med(kg) * 1e-3), "unit": "work-items/s", "n_gpus": 1, "steps": K,
           "warmup": W, "ms_per_step": med(kg), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u32", "data": "synthetic (no random input)",
           "config": {"workload": "escape-time 8192x8192 over [-2,1]x[-1.5,1.5], max_iter 4096", "devices": "gpu",
                      "scheduler": "static"},
           "roofline": r, "plain_launch": {"kernel_ms": med(kb), "roofline": rb}, "cpu_baseline": None}
    print(json.dumps(res), flush=True)


def bench_copy(args, ce, torch, stream):
    """The streaming-copy reference over 256 MiB and 1 GiB, timed with HIP
    events."""
    hev = HipEvents()
    res = [copy_reference(ce, torch, stream, hev, nb, args.steps) for nb in (256 << 20, 1 << 30)]
    print(json.dumps({"workload": "streaming copy", "copies": res}), flush=True)


def bench_nbody_step(args, ce, synth, torch, np, stream):
    """Time stepping of 65,536 bodies (positions and velocities in HBM,
    alternating between two pairs of buffers), one co-executed integration
    step per bench step: Dynamic 256-body packages, GPU + every host core.
    With device-only buffers the engine downloads the two inputs for the
    host workers at the start of each step and copies the host's rows of
    both outputs into HBM."""
    K, W = args.steps, args.warmup
    n, eps2, dt = 65536, 1e-6, 1e-3
    dev = torch.device("cuda:0")
    pos, vel = synth.nbody_bodies(n), synth.nbody_velocities(n)
    bufs = [[torch.from_numpy(pos).to(dev), torch.from_numpy(vel).to(dev)],
            [torch.empty((n, 4), device=dev), torch.empty((n, 4), device=dev)]]
    sync = torch.cuda.synchronize
    sync()
    params = ce.ce_nbody_step_params(n, eps2, dt, 1)
    kid = ce.CE_KERNEL_NBODY_STEP
    nbytes = n * 16

    def bind(eng, k):
        a, b = k % 2, 1 - k % 2
        for s_ in range(2):
            eng.program_in(s_, dev=bufs[a][s_], nbytes=nbytes)
            eng.program_out(s_, dev=bufs[b][s_], nbytes=nbytes)

    hev = HipEvents()
    ev_s = [hev.create() for _ in range(K)]
    ev_e = [hev.create() for _ in range(K)]
    # plain launch: one grid over all bodies, two outputs
    log("bare launch")
    def bare():
        ce.ce_bare_run_outs(kid, params, bufs[0], bufs[1], stream=stream.cuda_stream, sync=True)
    t_bare = timed_runs(bare, W, K, sync)
    for i in range(K):
        hev.record(ev_s[i], stream.cuda_stream)
        ce.ce_bare_run_outs(kid, params, bufs[0], bufs[1], stream=stream.cuda_stream, sync=False)
        hev.record(ev_e[i], stream.cuda_stream)
    sync()
    k_bare_ms = med([hev.elapsed_ms(ev_s[i], ev_e[i]) for i in range(K)])

    eng = ce.Engine()
    eng.stream(stream.cuda_stream)
    eng.work_items([n], [256])
    eng.program_kernel(kid, params)
    bind(eng, 0)
    log("engine GPU only")
    eng.use(ce.CE_DEV_GPU, 0, 0)
    eng.scheduler(ce.CE_SCHED_STATIC)
    t_gpu = timed_runs(eng.run, W, K, sync)
    log("engine host only")
    eng.use(ce.CE_DEV_HOST, 0, args.host_threads)
    t_host = timed_runs(eng.run, 1, min(K, 3), sync)
    host_threads_used = eng.stats().host_threads

    log("co-execution")
    eng.use(ce.CE_DEV_GPU | ce.CE_DEV_HOST, 0, args.host_threads)
    eng.scheduler(ce.CE_SCHED_DYNAMIC, package_granules=1)
    for k in range(W):
        bind(eng, k)
        eng.run()
    per_run = []
    sync()
    t0 = time.perf_counter()
    for k in range(K):
        a = time.perf_counter()
        bind(eng, W + k)
        eng.run()
        per_run.append(time.perf_counter() - a)
    sync()
    T_total = time.perf_counter() - t0
    stats = []
    for k in range(K):
        bind(eng, W + K + k)
        eng.kernel_events(ev_s[k], ev_e[k])
        eng.run()
        stats.append(eng.stats())
    eng.kernel_events(None, None)
    kern_ms = [hev.elapsed_ms(ev_s[i], ev_e[i]) for i in range(K)]
    for ev in ev_s + ev_e:
        hev.destroy(ev)
    T_bare, T_gpu, T_host = med(t_bare), med(t_gpu), med(t_host)
    s_real = min(T_bare, T_host) / med(per_run)
    s_max = min(T_bare, T_host) * (1.0 / T_bare + 1.0 / T_host)
    gpu_share = sum(s_.items[0] for s_ in stats) / (K * n)
    cpu_base = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        from oracle import oracle as O
        t0c = time.perf_counter()
        i = 0
        while time.perf_counter() - t0c < 10.0:
            O.nbody_step_body(pos, vel, eps2, dt, i, True)
            i += 1
        dtc = time.perf_counter() - t0c
        cpu_base = {"value": i / dtc, "unit": "work-items/s", "cores": 1, "kind": "oracle",
                    "sample": f"{i} bodies stepped (each against all {n})", "seconds": dtc}
    res = {
        "metric": METRIC, "value": n * K / T_total, "unit": "work-items/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": T_total / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded SplitMix64 inputs, paper_1805_02755_amd/synth.py)",
        "config": {"workload": "nbody integration step, 65536 bodies fp32, eps2 1e-6, dt 1e-3, strict rsqrt, "
                               "resident ping-pong buffers", "scheduler": "dynamic 256-body packages",
                   "devices": "gpu+host", "residency": "device"},
        "roofline": dict(alu_roofline(20.0 * n * n * gpu_share, 24.0 * n * n * gpu_share, med(kern_ms),
                                      "k_persistent<NbodyStepTile<true>>", "nbody_step_65536_valu.json"),
                         flops_per_interaction=20, lane_ops_per_interaction=24),
        "cpu_baseline": cpu_base,
        "coexec": {
            "plain_gpu_items_per_s": n / T_bare, "vs_plain_gpu": T_bare / med(per_run), "s_real": s_real, "s_max": s_max,
            "efficiency": s_real / s_max, "balance": med([s_.balance for s_ in stats]),
            "overhead_pct_gpu_only": (T_gpu - T_bare) / T_bare * 100.0,
            "t_bare_ms": T_bare * 1e3, "t_bare_kernel_ms": k_bare_ms, "t_engine_gpu_ms": T_gpu * 1e3,
            "t_engine_host_ms": T_host * 1e3, "t_coexec_ms_median": med(per_run) * 1e3,
            "host_threads": host_threads_used, "gpu_share": gpu_share,
            "packages_gpu": med([s_.packages[0] for s_ in stats]), "packages_host": med([s_.packages[1] for s_ in stats]),
            "t_device_ms": [med([s_.t_device[0] for s_ in stats]) * 1e3, med([s_.t_device[1] for s_ in stats]) * 1e3],
        },
    }
    print(json.dumps(res), flush=True)
    eng.close()


def bench_binomial(args, ce, synth, torch, np, stream):
    """Binomial option pricing at the paper's listing size: 16,777,216 calls
    (4,194,304 work-groups of 255 work-items, 254 steps), spots uniform in
    [50, 150), strike 100, sigma 0.3, rate 0.05, T 1; HGuided over GPU + every
    host core, inputs resident in HBM with host mirrors, output in HBM. The
    host alone is timed on 16,384 groups and scaled to the full size (a full
    host-only run would take tens of seconds)."""
    K, W = args.steps, args.warmup
    n_groups, steps = 4194304, 254
    dev = torch.device("cuda:0")
    spots = synth.binomial_spots(n_groups)
    f, pu, pd = ce.ce_binomial_table(steps, 0.3, 0.05, 1.0)
    params = ce.ce_binomial_params(n_groups, steps, 100.0, pu, pd)
    kid = ce.CE_KERNEL_BINOMIAL
    s_d, f_d = torch.from_numpy(spots).to(dev), torch.from_numpy(f).to(dev)
    out_d = torch.empty((n_groups, 4), device=dev)
    sync = torch.cuda.synchronize
    sync()
    items = (steps + 1) * n_groups
    hev = HipEvents()
    ev_s = [hev.create() for _ in range(K)]
    ev_e = [hev.create() for _ in range(K)]
    log("bare launch")
    def bare():
        ce.ce_bare_run(kid, params, [s_d, f_d], out_d, stream=stream.cuda_stream, sync=True)
    t_bare = timed_runs(bare, W, K, sync)
    for i in range(K):
        hev.record(ev_s[i], stream.cuda_stream)
        ce.ce_bare_run(kid, params, [s_d, f_d], out_d, stream=stream.cuda_stream, sync=False)
        hev.record(ev_e[i], stream.cuda_stream)
    sync()
    k_bare_ms = med([hev.elapsed_ms(ev_s[i], ev_e[i]) for i in range(K)])

    def engine_for(ng, sp, sd, od):
        e = ce.Engine()
        e.stream(stream.cuda_stream)
        e.work_items([(steps + 1) * ng], [steps + 1])
        e.program_kernel(kid, ce.ce_binomial_params(ng, steps, 100.0, pu, pd))
        e.program_out_pattern(1, steps + 1)
        e.program_in(0, host=sp, dev=sd, nbytes=sp.nbytes)
        e.program_in(1, host=f, dev=f_d, nbytes=f.nbytes)
        e.program_out(0, dev=od, nbytes=od.numel() * 4)
        return e

    eng = engine_for(n_groups, spots, s_d, out_d)
    log("engine GPU only")
    eng.use(ce.CE_DEV_GPU, 0, 0)
    eng.scheduler(ce.CE_SCHED_STATIC)
    t_gpu = timed_runs(eng.run, W, K, sync)
    log("engine host only (16,384 groups, scaled)")
    sub = 16384
    small = engine_for(sub, spots[:sub].copy(), s_d[:sub], torch.empty((sub, 4), device=dev))
    small.use(ce.CE_DEV_HOST, 0, args.host_threads)
    small.scheduler(ce.CE_SCHED_STATIC)
    t_host_small = timed_runs(small.run, 1, 2, sync)
    host_threads_used = small.stats().host_threads
    small.close()
    T_bare, T_gpu = med(t_bare), med(t_gpu)
    T_host = med(t_host_small) * n_groups / sub
    log("co-execution")
    power = [max(1, min(1 << 20, int(round(T_host / T_gpu)))), 1]
    eng.use(ce.CE_DEV_GPU | ce.CE_DEV_HOST, 0, args.host_threads)
    eng.scheduler(ce.CE_SCHED_HGUIDED, power=power, k=2)
    for _ in range(W):
        eng.run()
    per_run = []
    sync()
    t0 = time.perf_counter()
    for _ in range(K):
        a = time.perf_counter()
        eng.run()
        per_run.append(time.perf_counter() - a)
    sync()
    T_total = time.perf_counter() - t0
    stats = []
    for i in range(K):
        eng.kernel_events(ev_s[i], ev_e[i])
        eng.run()
        stats.append(eng.stats())
    eng.kernel_events(None, None)
    kern_ms = [hev.elapsed_ms(ev_s[i], ev_e[i]) for i in range(K)]
    for ev in ev_s + ev_e:
        hev.destroy(ev)
    s_real = min(T_bare, T_host) / med(per_run)
    s_max = min(T_bare, T_host) * (1.0 / T_bare + 1.0 / T_host)
    gpu_share = sum(s_.items[0] for s_ in stats) / (K * items)
    # per call: steps+1 leaves (a mul, a sub and a max: two flops, three lane-ops) and
    # steps*(steps+1)/2 node updates (two muls and an add)
    nodes = steps * (steps + 1) / 2
    flops = 4.0 * n_groups * (2.0 * (steps + 1) + 3.0 * nodes) * gpu_share
    lane_ops = 4.0 * n_groups * (3.0 * (steps + 1) + 3.0 * nodes) * gpu_share
    cpu_base = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        from oracle import oracle as O
        t0c = time.perf_counter()
        k = 0
        flat = spots.reshape(-1)
        while time.perf_counter() - t0c < 10.0:
            O.binomial_price(float(flat[k]), 100.0, steps, f, pu, pd)
            k += 1
        dtc = time.perf_counter() - t0c
        cpu_base = {"value": k * (steps + 1) / 4 / dtc, "unit": "work-items/s", "cores": 1, "kind": "oracle",
                    "sample": f"{k} calls priced ({k / dtc:.0f} calls/s; 255 work-items per four calls)",
                    "seconds": dtc}
    res = {
        "metric": METRIC, "value": items * K / T_total, "unit": "work-items/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": T_total / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded SplitMix64 inputs, paper_1805_02755_amd/synth.py)",
        "config": {"workload": "binomial options: 16777216 European calls, 254 steps, 4194304 work-groups of 255, "
                               "out pattern 1:255", "scheduler": "hguided", "devices": "gpu+host",
                   "residency": "device", "options_per_s": 4 * n_groups * K / T_total},
        "roofline": alu_roofline(flops, lane_ops, med(kern_ms), "k_persistent<BinomialTile>",
                                 "binomial_4194304x254_valu.json"),
        "cpu_baseline": cpu_base,
        "coexec": {
            "plain_gpu_items_per_s": items / T_bare, "vs_plain_gpu": T_bare / med(per_run), "s_real": s_real, "s_max": s_max,
            "efficiency": s_real / s_max, "balance": med([s_.balance for s_ in stats]),
            "overhead_pct_gpu_only": (T_gpu - T_bare) / T_bare * 100.0,
            "t_bare_ms": T_bare * 1e3, "t_bare_kernel_ms": k_bare_ms, "t_engine_gpu_ms": T_gpu * 1e3,
            "t_engine_host_ms_scaled": T_host * 1e3, "t_coexec_ms_median": med(per_run) * 1e3,
            "host_threads": host_threads_used, "gpu_share": gpu_share, "scheduler": {"power": power, "k": 2},
            "packages_gpu": med([s_.packages[0] for s_ in stats]), "packages_host": med([s_.packages[1] for s_ in stats]),
            "t_device_ms": [med([s_.t_device[0] for s_ in stats]) * 1e3, med([s_.t_device[1] for s_ in stats]) * 1e3],
        },
    }
    print(json.dumps(res), flush=True)
    eng.close()


def bench_batch(args, ce, synth, torch, np, stream):
    """256 escape-time jobs of uneven sizes (sides log-uniform in [64, 2048],
    max_iter uniform in [64, 4096], seed 0xBA7C4) as one persistent,
    graph-captured launch with an autotuned tile shape and package size,
    against one plain launch per job."""
    K, W = args.steps, args.warmup
    jobs = synth.batch_jobs()
    dev = torch.device("cuda:0")
    outs = [torch.empty((p.h, p.w), dtype=torch.int32, device=dev) for p in jobs]
    torch.cuda.synchronize()
    b = ce.Batch(stream.cuda_stream)
    for p, o in zip(jobs, outs):
        b.add_escape(ce.ce_escape_params(p.w, p.h, *p.as_f32(), p.max_iter), o)
    n_items = sum(p.w * p.h for p in jobs)
    log("separate launches")
    for _ in range(W):
        b.run_separate()
    t_sep, g_sep = [], []
    for _ in range(K):
        b.run_separate()
        st = b.stats()
        t_sep.append(st.t_run)
        g_sep.append(st.t_gpu_ms)
    log("autotune")
    chosen = b.tune(reps=2)
    for _ in range(W):
        b.run()
    torch.cuda.synchronize()
    per_run, kern = [], []
    t0 = time.perf_counter()
    for _ in range(K):
        b.run()
        st = b.stats()
        per_run.append(st.t_run)
        kern.append(st.t_gpu_ms)
    T = time.perf_counter() - t0
    iters = int(sum(int(o.to(torch.int64).sum().item()) for o in outs))
    cpu_base = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        t0 = time.perf_counter()
        done = 0
        nj = 0
        for p in jobs:
            O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)
            done += p.w * p.h
            nj += 1
            if time.perf_counter() - t0 > 10.0:
                break
        dt = time.perf_counter() - t0
        cpu_base = {"value": done / dt, "unit": "work-items/s", "cores": 1, "kind": "oracle",
                    "sample": f"the first {nj} jobs of the batch", "seconds": dt}
    res = {
        "metric": METRIC, "value": n_items * K / T, "unit": "work-items/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": T / K * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic (seeded SplitMix64 inputs, paper_1805_02755_amd/synth.py)",
        "config": {"workload": "batched escape-time: 256 jobs, side log-uniform [64,2048], max_iter U[64,4096]",
                   "form": "one persistent hipGraph launch", "tile_rows": chosen[0], "tile_cols": chosen[1],
                   "package_tiles": chosen[2]},
        "roofline": dict(alu_roofline(8.0 * iters, 8.0 * iters, med(kern), "k_batch_escape",
                                      "batch_escape_256jobs_valu.json"), iterations=iters),
        "cpu_baseline": cpu_base,
        "batch": {"separate_launch_ms": med(t_sep) * 1e3, "separate_gpu_ms": med(g_sep),
                  "graph_launch_ms": med(per_run) * 1e3, "graph_gpu_ms": med(kern),
                  "speedup_vs_separate": med(t_sep) / med(per_run), "jobs": len(jobs), "items": n_items},
    }
    print(json.dumps(res), flush=True)
    b.close()


def bench_serve(args, ce, synth, torch, np, stream):
    """Serving (continuous batching) under calibrated load. A trace of escape,
    blur and n-body jobs (sizes log-uniform, kinds in thirds; seed 0x5E2E) is
    first run saturated, all jobs submitted at once, which measures the
    serving kernel's capacity (jobs/s) and one plain launch per job back to
    back. The trace's Poisson arrivals are then replayed at rate
    rho x capacity for rho in 0.5, 0.7, 0.9, against the serving kernel and
    against one plain launch per job in arrival order; latency is arrival to
    completion. Inputs come from resident pools in HBM (a job of side s reads
    the first s*s pixels of one 16384^2 image; a job of n bodies the first n
    of 131,072); outputs are allocated per job from the HBM budget."""
    import threading
    n_jobs = args.serve_jobs
    trace = synth.serve_trace(n_jobs)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(synth.blur_image(16384, 16384, seed=0x5E21)).to(dev)
    bodies = torch.from_numpy(synth.nbody_bodies(131072, seed=0x5E22)).to(dev)
    wt = torch.from_numpy(ce.ce_gauss5_weights(1.0)).to(dev)
    eps2 = 1e-6

    def job_args(j):
        if j.kind == "escape":
            p = synth.escape_region(j.size, j.size, *j.region, j.max_iter)
            return ce.CE_KERNEL_ESCAPE, ce.ce_escape_params(p.w, p.h, *p.as_f32(), p.max_iter), [], j.size * j.size
        if j.kind == "blur":
            return ce.CE_KERNEL_BLUR5, ce.ce_blur5_params(j.size, j.size), [img, wt], j.size * j.size
        return ce.CE_KERNEL_NBODY_ACC, ce.ce_nbody_params(j.size, eps2, 0), [bodies], j.size

    specs = [job_args(j) for j in trace]
    n_items = sum(s[3] for s in specs)
    out_bytes = max(s[3] for s in specs) * 16
    budget = max(4 << 30, 8 * out_bytes)
    torch.cuda.synchronize()
    scratch = torch.empty(out_bytes, dtype=torch.uint8, device=dev)

    def plain(kid, prm, ins):
        ce.ce_bare_run(kid, prm, ins, scratch, stream=stream.cuda_stream, sync=True)

    # warm both paths
    for kid, prm, ins, _ in specs[:8]:
        plain(kid, prm, ins)
    srv = ce.Server(budget, keep_outputs=False, session_timeout_s=30.0)
    for t in [srv.submit(*s_[:2], *s_[2]) for s_ in specs[:8]]:
        srv.wait(t, 120.0)
    srv.drain(120.0)
    srv.close()

    # ------------------------------------------------ saturated: capacity
    log(f"serving: {n_jobs} jobs saturated (capacity)")
    t0 = time.perf_counter()
    for kid, prm, ins, _ in specs:
        plain(kid, prm, ins)
    plain_wall = time.perf_counter() - t0
    srv = ce.Server(budget, keep_outputs=False, session_timeout_s=30.0)
    tickets = [srv.submit(*s_[:2], *s_[2]) for s_ in specs]
    for t in tickets:
        srv.wait(t, 600.0)
    srv.drain(120.0)
    sat = srv.stats()
    srv.close()
    capacity = sat.completed / sat.wall_s
    plain_capacity = n_jobs / plain_wall

    def replay_server(arrivals):
        srv = ce.Server(budget, keep_outputs=False, session_timeout_s=30.0)
        tks = []

        def client():
            c0 = time.perf_counter()
            for a, s_ in zip(arrivals, specs):
                now = time.perf_counter() - c0
                if now < a:
                    time.sleep(a - now)
                tks.append(srv.submit(*s_[:2], *s_[2]))
        th = threading.Thread(target=client)
        th.start()
        th.join()
        for t in tks:
            srv.wait(t, 600.0)
        srv.drain(120.0)
        r = srv.stats()
        srv.close()
        return {"p50_ms": r.p50_s * 1e3, "p99_ms": r.p99_s * 1e3, "mean_ms": r.mean_s * 1e3, "max_ms": r.max_s * 1e3,
                "items_per_s": r.items_per_s, "jobs_per_s": r.jobs_per_s, "wall_s": r.wall_s,
                "max_inflight": int(r.max_inflight_seen), "peak_hbm_bytes": int(r.peak_hbm)}

    def replay_plain(arrivals):
        lat = []
        t0 = time.perf_counter()
        for a, (kid, prm, ins, _) in zip(arrivals, specs):
            now = time.perf_counter() - t0
            if now < a:
                time.sleep(a - now)
            plain(kid, prm, ins)
            lat.append(time.perf_counter() - t0 - a)
        wall = time.perf_counter() - t0
        return {"p50_ms": pct(lat, 50) * 1e3, "p99_ms": pct(lat, 99) * 1e3, "mean_ms": sum(lat) / len(lat) * 1e3,
                "max_ms": max(lat) * 1e3, "items_per_s": n_items / wall, "jobs_per_s": n_jobs / wall, "wall_s": wall}

    loads = {}
    base_rate = n_jobs / trace[-1].arrival_s  # the trace's own rate
    for rho in (0.5, 0.7, 0.9):
        lam = rho * capacity
        arrivals = [j.arrival_s * base_rate / lam for j in trace]
        log(f"serving: rho {rho}, {lam:.0f} jobs/s over {arrivals[-1]:.1f} s")
        loads[str(rho)] = {"rate_jobs_per_s": lam, "serving": replay_server(arrivals), "plain": replay_plain(arrivals)}
    del scratch
    cpu_base = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        t0 = time.perf_counter()
        done = nj = 0
        for j in trace:
            if j.kind != "escape":
                continue
            p = synth.escape_region(j.size, j.size, *j.region, j.max_iter)
            O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)
            done += p.w * p.h
            nj += 1
            if time.perf_counter() - t0 > 10.0:
                break
        dt = time.perf_counter() - t0
        cpu_base = {"value": done / dt, "unit": "work-items/s", "cores": 1, "kind": "oracle",
                    "sample": f"the first {nj} escape-time jobs of the trace", "seconds": dt}
    res = {
        "metric": METRIC, "value": sat.items_per_s, "unit": "work-items/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": sat.wall_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed (u32 escape, f32 blur and n-body)",
        "data": "synthetic (seeded SplitMix64 trace, paper_1805_02755_amd/synth.py)",
        "config": {"workload": f"serving trace: {n_jobs} jobs, escape side [256,4096] max_iter U[64,4096], "
                               "blur side [1024,16384], n-body [4096,131072] (hardware rsqrt)",
                   "form": "persistent serving kernel, continuous batching"},
        "roofline": None,
        "cpu_baseline": cpu_base,
        "serve": {"capacity_jobs_per_s": capacity, "saturated_items_per_s": sat.items_per_s,
                  "saturated_p50_ms": sat.p50_s * 1e3, "saturated_p99_ms": sat.p99_s * 1e3,
                  "plain_capacity_jobs_per_s": plain_capacity, "plain_items_per_s": n_items / plain_wall,
                  "loads": loads},
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
