#!/usr/bin/env python3
"""Co-execution bench on one MI355X plus the host CPU cores.

Default workload: 5x5 Gaussian blur of an 8192 x 8192 FP32 image (pixels
uniform in [0, 1), seed 0xB1), HGuided scheduler, GPU + every host core. A
step is one ce_engine_run over the whole image. Inputs are resident before
the timed region: in HBM for the GPU and mirrored in host memory for the host
workers; the output ends in HBM (the host's rows copied by the SDMA engines
during the run).

The JSON line reports work-items/s of the co-executed run (value: K runs timed
back to back, nothing else in the loop), the plain single-GPU launch of the
same kernel, the engine's overhead over it, the balance and efficiency of
section 7.3 (from per-run medians, measured alike for the plain launch, the
engine alone and the co-execution), the roofline of the persistent GPU kernel
(timed with HIP events on its stream, in a second, untimed pass of K runs) and
the oracle timed on the host.

Other workloads: --workload escape (1024^2, max_iter 256, Static with 8
packages, GPU + 1 host thread) and --workload nbody (65,536 bodies, Dynamic
256-body packages, GPU + every host core).
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
# Non-packed FP32 VALU issue rate: 256 CUs x 64 lanes per clock x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


DEVICE_SOURCES = ("paper_1805_02755_amd/csrc/kernels.hip", "paper_1805_02755_amd/csrc/device_tiles.hpp",
                  "paper_1805_02755_amd/csrc/device_atomics.hpp", "paper_1805_02755_amd/csrc/device_payloads.hpp",
                  "paper_1805_02755_amd/csrc/common.hpp", "paper_1805_02755_amd/csrc/sched_device.hpp",
                  "paper_1805_02755_amd/csrc/rt_tile.hpp")


def measured_traffic(name):
    """HBM bytes per dispatch from the committed counter summary, or None if
    the device sources changed since the counters were taken."""
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
    return rec.get("traffic_bytes_per_dispatch")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["blur", "escape", "runtime", "nbody", "nbody-step", "binomial", "batch", "serve",
                                           "copy"],
                    default="blur")
    ap.add_argument("--serve-jobs", type=int, default=2000)
    ap.add_argument("--trace-out", default=None, help="write the last co-executed run's package trace (JSON) here")
    ap.add_argument("--mode", choices=["device", "host"], default="device",
                    help="device: inputs and output resident in HBM; host: host buffers, PCIe inside the step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--merge", choices=["dma", "gpu"], default="dma",
                    help="how the host's share reaches the device output: the GPU's copy engines (dma) or "
                         "gather workgroups inside its kernel (gpu)")
    ap.add_argument("--host-threads", type=int, default=0)
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1805_02755_amd as ce
    from paper_1805_02755_amd import synth

    ce.lib()  # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    sync = torch.cuda.synchronize
    host_cores = os.cpu_count() or 1
    if args.workload == "batch":
        return bench_batch(args, ce, synth, torch, np, stream)
    if args.workload == "serve":
        return bench_serve(args, ce, synth, torch, np, stream)
    if args.workload == "copy":
        return bench_copy(args, torch, stream)
    if args.workload == "nbody-step":
        return bench_nbody_step(args, ce, synth, torch, np, stream)
    if args.workload == "binomial":
        return bench_binomial(args, ce, synth, torch, np, stream)

    eng = ce.Engine()
    eng.stream(stream.cuda_stream)
    eng.output_merge(ce.CE_MERGE_DMA if args.merge == "dma" else ce.CE_MERGE_GPU_GATHER)

    # ---------------------------------------------------------------- payload
    wl = args.workload
    if wl == "blur":
        w = h = 8192
        log("generating 8192x8192 image")
        img = synth.blur_image(w, h)
        wt = ce.ce_gauss5_weights(1.0)
        img_d = torch.from_numpy(img).to(dev)
        wt_d = torch.from_numpy(wt).to(dev)
        out_d = torch.empty_like(img_d)
        out_h = np.empty_like(img) if args.mode == "host" else None
        params = ce.ce_blur5_params(w, h)
        kid = ce.CE_KERNEL_BLUR5
        gws, lws = [w, h], None
        ins_host, ins_dev = [img, wt], [img_d, wt_d]
        n_items = w * h
        G = h
        bytes_per_item = 8.0  # 4 B read + 4 B written; halo re-reads are not algorithmic
        host_threads = args.host_threads
        coexec = dict(kind=ce.CE_SCHED_HGUIDED, k=2)
        config = {"workload": "blur5x5 8192x8192 fp32, sigma 1, clamp-to-edge", "scheduler": "hguided",
                  "devices": "gpu+host", "residency": args.mode, "output_merge": args.merge}
        bound = "hbm"
    elif wl in ("escape", "runtime"):
        p = synth.escape_small()
        params = ce.ce_escape_params(p.w, p.h, *p.as_f32(), p.max_iter)
        kid = ce.CE_KERNEL_ESCAPE
        gws, lws = [p.w, p.h], None
        out_d = torch.empty((p.h, p.w), dtype=torch.int32, device=dev)
        out_h = np.empty((p.h, p.w), np.uint32) if args.mode == "host" else None
        ins_host, ins_dev = [], []
        n_items = p.w * p.h
        G = p.h
        host_threads = args.host_threads
        coexec = dict(kind=ce.CE_SCHED_HGUIDED, k=2)
        config = {"workload": "escape-time 1024x1024 over [-2,1]x[-1.5,1.5], max_iter 256", "scheduler": "hguided",
                  "devices": "gpu+host", "residency": args.mode}
        bound = "alu"
        if wl == "runtime":
            if args.mode != "device":
                raise SystemExit("--workload runtime runs with device residency only")
            from paper_1805_02755_amd import rt_examples
            config["workload"] += ", supplied as HIP source at run time (hipRTC) with a C host version"
            # The plain C host version needs about 0.16 ms per 1024-pixel row,
            # more than the GPU's whole run: 64-pixel granules and HGuided let
            # the host take only what it finishes in time.
            rt_lws = 64
            G = n_items // rt_lws
            config["granule"] = "64 pixels"
    else:
        n = 65536
        bodies = synth.nbody_bodies(n)
        b_d = torch.from_numpy(bodies).to(dev)
        out_d = torch.empty_like(b_d)
        out_h = np.empty_like(bodies) if args.mode == "host" else None
        params = ce.ce_nbody_params(n, 1e-6, 1)
        kid = ce.CE_KERNEL_NBODY_ACC
        gws, lws = [n], [256]
        ins_host, ins_dev = [bodies], [b_d]
        n_items = n
        G = n // 256
        host_threads = args.host_threads
        coexec = dict(kind=ce.CE_SCHED_DYNAMIC, package_granules=1)
        config = {"workload": "nbody acceleration 65536 bodies fp32, eps2 1e-6, strict rsqrt",
                  "scheduler": "dynamic 256-body packages", "devices": "gpu+host", "residency": args.mode}
        bound = "alu"
    sync()

    eng.work_items(gws, lws)
    if wl == "runtime":
        eng.work_items([n_items], [rt_lws])
        t_c = time.perf_counter()
        eng.program_source(rt_examples.source("escape.hiprtc"), "escape_item",
                           host=rt_examples.host_fn("escape_host"), n_in=0, n_out=1, out_item_bytes=4,
                           scalars=rt_examples.escape_scalars(p.w, *p.as_f32(), p.max_iter))
        config["compile_s"] = time.perf_counter() - t_c
    else:
        eng.program_kernel(kid, params)
    for slot in range(len(ins_host)):
        if args.mode == "host":
            eng.program_in(slot, host=ins_host[slot])
        else:
            eng.program_in(slot, host=ins_host[slot], dev=ins_dev[slot], nbytes=ins_host[slot].nbytes)
    if args.mode == "host":
        eng.program_out(0, host=out_h)
    else:
        eng.program_out(0, dev=out_d, nbytes=out_d.numel() * out_d.element_size())

    K, W = args.steps, args.warmup

    # ---------------------------------------------- plain single-GPU launch
    log("bare launch")
    def bare_launch(do_sync):
        if wl == "runtime":
            eng.bare_run_source(n_items, rt_lws, [], [out_d], stream=stream.cuda_stream, sync=do_sync)
        else:
            ce.ce_bare_run(kid, params, ins_dev if args.mode != "host" else ins_dev_b, out_d,
                           stream=stream.cuda_stream, sync=do_sync)

    def bare():
        if args.mode == "host":
            for i, a in enumerate(ins_host):
                ins_dev_b[i].copy_(torch.from_numpy(a), non_blocking=False)
            ce.ce_bare_run(kid, params, ins_dev_b, out_d, stream=stream.cuda_stream, sync=True)
            out_h_b[...] = out_d.cpu().numpy().view(out_h_b.dtype).reshape(out_h_b.shape)
        else:
            bare_launch(True)
    if args.mode == "host":
        ins_dev_b = [torch.empty(a.shape, dtype=torch.from_numpy(a).dtype, device=dev) for a in ins_host]
        out_h_b = np.empty_like(out_h)
    t_bare = timed_runs(bare, W, K, sync)
    hev = HipEvents()
    ev_s = [hev.create() for _ in range(K)]
    ev_e = [hev.create() for _ in range(K)]
    # kernel time of the plain launch, from events on its stream
    for i in range(K):
        hev.record(ev_s[i], stream.cuda_stream)
        bare_launch(False)
        hev.record(ev_e[i], stream.cuda_stream)
    sync()
    k_bare_ms = med([hev.elapsed_ms(ev_s[i], ev_e[i]) for i in range(K)])

    # ------------------------------------------------- engine, GPU alone
    log("engine GPU only")
    eng.use(ce.CE_DEV_GPU, 0, 0)
    eng.scheduler(ce.CE_SCHED_STATIC)
    t_gpu = timed_runs(eng.run, W, K, sync)
    k_gpu = []
    for i in range(K):
        eng.kernel_events(ev_s[i], ev_e[i])
        eng.run()
        k_gpu.append(hev.elapsed_ms(ev_s[i], ev_e[i]))
    eng.kernel_events(None, None)
    k_gpu_ms = med(k_gpu)

    # ------------------------------------------------- engine, host alone
    log("engine host only")
    eng.use(ce.CE_DEV_HOST, 0, host_threads)
    eng.scheduler(ce.CE_SCHED_STATIC)
    t_host = timed_runs(eng.run, 1, min(K, 5), sync)
    host_threads_used = eng.stats().host_threads

    # ------------------------------------------------- co-execution
    T_bare, T_gpu, T_host = med(t_bare), med(t_gpu), med(t_host)
    if coexec["kind"] == ce.CE_SCHED_HGUIDED:
        # computing powers from the standalone throughputs, the slower device at 1
        if T_host >= T_gpu:
            coexec["power"] = [max(1, min(1 << 20, int(round(T_host / T_gpu)))), 1]
        else:
            coexec["power"] = [1, max(1, min(1 << 20, int(round(T_gpu / T_host))))]
    elif coexec["kind"] == ce.CE_SCHED_STATIC:
        coexec["props"] = [max(0.0, 1.0 - T_gpu / (T_gpu + T_host))]
    eng.use(ce.CE_DEV_GPU | ce.CE_DEV_HOST, 0, host_threads)
    eng.scheduler(**coexec)
    log(f"co-execution {coexec}")
    for _ in range(W):
        eng.run()
    # the timed steps: nothing but the runs (and a clock read) in the loop
    per_run = []
    sync()
    t0 = time.perf_counter()
    for i in range(K):
        a = time.perf_counter()
        eng.run()
        per_run.append(time.perf_counter() - a)
    sync()
    T_total = time.perf_counter() - t0
    # the same runs again, untimed, for kernel events and per-run statistics
    stats = []
    for i in range(K):
        eng.kernel_events(ev_s[i], ev_e[i])
        eng.run()
        stats.append(eng.stats())
    eng.kernel_events(None, None)
    trace = eng.trace()
    if args.trace_out:
        with open(args.trace_out, "w") as f:
            json.dump({"stats": {"t_device": list(stats[-1].t_device[:2]), "t_run": stats[-1].t_run,
                                 "t_gather": stats[-1].t_gather, "gathered_bytes": stats[-1].gathered_bytes},
                       "packages": [list(r) for r in trace]}, f)

    kern_ms = [hev.elapsed_ms(ev_s[i], ev_e[i]) for i in range(K)]
    for ev in ev_s + ev_e:
        hev.destroy(ev)
    gpu_items = [s.items[0] for s in stats]
    host_items = [s.items[1] for s in stats]
    T_co = T_total / K
    value = n_items * K / T_total
    # speedup and efficiency compare per-run medians, measured the same way
    # for the plain launch, the engine alone and the co-execution
    s_real = T_bare / med(per_run)
    s_max = min(T_bare, T_host) * (1.0 / T_bare + 1.0 / T_host)
    balance = med([s.balance for s in stats])

    # --------------------------------------------------------- roofline
    if wl == "blur":
        achieved = sum(bytes_per_item * g for g in gpu_items) / (sum(kern_ms) * 1e-3) / 1e9
        traffic = measured_traffic("blur5_8192_hbm_traffic.json") if args.mode == "device" else None
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_unit": "bytes per launch",
                "kernel": "k_persistent<Blur5Tile>", "kernel_ms": med(kern_ms),
                "algorithmic_bytes_per_item": bytes_per_item}
    elif wl in ("escape", "runtime"):
        cnt = out_d.cpu().numpy().view(np.uint32).astype(np.int64)
        iters = int(cnt.sum())
        ops = 8.0 * iters * (sum(gpu_items) / (K * n_items))
        achieved = ops / (med(kern_ms) * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s (FP32 VALU lane-ops)",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                "kernel": "k_persistent<RtTile> (hipRTC)" if wl == "runtime" else "k_persistent<EscapeTile>",
                "kernel_ms": med(kern_ms), "iterations": iters}
    else:
        n = n_items
        ops = 24.0 * n * n * (sum(gpu_items) / (K * n_items))
        achieved = ops / (med(kern_ms) * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s (FP32 VALU lane-ops)",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": None, "kernel": "k_persistent<NbodyTile<true>>",
                "kernel_ms": med(kern_ms), "ops_per_interaction": 24}

    # ------------------------------------------------------ CPU baseline
    cpu_base = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        from oracle import oracle as O
        t0 = time.perf_counter()
        done_items = 0
        if wl == "blur":
            wt_o = O.gauss5_weights(1.0)
            passes = 0
            while passes < 4 and (time.perf_counter() - t0 < 10.0):
                O.blur5(img, wt_o)
                passes += 1
                done_items += n_items
            sample = f"{passes} full passes over the 8192x8192 image"
        elif wl in ("escape", "runtime"):
            passes = 0
            while passes < 40 and (time.perf_counter() - t0 < 10.0):
                O.escape(p.w, p.h, *[float(v) for v in p.as_f32()], p.max_iter)
                passes += 1
                done_items += n_items
            sample = f"{passes} full passes over the 1024x1024 grid"
        else:
            i = 0
            while time.perf_counter() - t0 < 10.0:
                O.nbody_acc_body(bodies, 1e-6, i, True)
                i += 1
            done_items = i
            sample = f"{i} bodies (each against all 65536)"
        dt = time.perf_counter() - t0
        cpu_base = {"value": done_items / dt, "unit": "work-items/s", "cores": 1, "kind": "oracle",
                    "sample": sample, "seconds": dt}

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "work-items/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": T_co * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if wl in ("escape", "runtime") else "f32",
        "data": "synthetic (seeded SplitMix64 inputs, paper_1805_02755_amd/synth.py)",
        "config": config,
        "roofline": roof,
        "cpu_baseline": cpu_base,
        "coexec": {
            "plain_gpu_items_per_s": n_items / T_bare,
            "vs_plain_gpu": s_real,
            "balance": balance,
            "s_real": s_real,
            "s_max": s_max,
            "efficiency": s_real / s_max,
            "overhead_pct_gpu_only": (T_gpu - T_bare) / T_bare * 100.0,
            "t_bare_ms": T_bare * 1e3,
            "t_bare_kernel_ms": k_bare_ms,
            "t_engine_gpu_ms": T_gpu * 1e3,
            "t_engine_gpu_kernel_ms": k_gpu_ms,
            "t_engine_host_ms": T_host * 1e3,
            "t_coexec_ms_median": med(per_run) * 1e3,
            "host_threads": host_threads_used,
            "host_cores": host_cores,
            "gpu_share": sum(gpu_items) / (K * n_items),
            "packages_gpu": med([s.packages[0] for s in stats]),
            "packages_host": med([s.packages[1] for s in stats]),
            "scheduler": {k: (list(v) if isinstance(v, (list, tuple)) else v) for k, v in coexec.items()},
            "t_device_ms": [med([s.t_device[0] for s in stats]) * 1e3, med([s.t_device[1] for s in stats]) * 1e3],
            "t_gather_ms": med([s.t_gather for s in stats]) * 1e3,
            "gathered_MiB": med([s.gathered_bytes for s in stats]) / 2**20,
            "trace_packages": len(trace),
        },
    }
    print(json.dumps(res), flush=True)
    eng.close()


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
    s_real = T_bare / med(per_run)
    s_max = min(T_bare, T_host) * (1.0 / T_bare + 1.0 / T_host)
    gpu_share = sum(s_.items[0] for s_ in stats) / (K * n)
    ops = 24.0 * n * n * gpu_share
    achieved = ops / (med(kern_ms) * 1e-3) / 1e12
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s (FP32 VALU lane-ops)", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "kernel": "k_persistent<NbodyStepTile<true>>", "kernel_ms": med(kern_ms),
                     "ops_per_interaction": 24},
        "cpu_baseline": cpu_base,
        "coexec": {
            "plain_gpu_items_per_s": n / T_bare, "vs_plain_gpu": s_real, "s_real": s_real, "s_max": s_max,
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
    s_real = T_bare / med(per_run)
    s_max = min(T_bare, T_host) * (1.0 / T_bare + 1.0 / T_host)
    gpu_share = sum(s_.items[0] for s_ in stats) / (K * items)
    # per call: 255 leaves (mul, sub, max) and steps*(steps+1)/2 node updates (two muls and an add)
    ops = 4.0 * n_groups * (3.0 * (steps + 1) + 3.0 * steps * (steps + 1) / 2) * gpu_share
    achieved = ops / (med(kern_ms) * 1e-3) / 1e12
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s (FP32 VALU lane-ops)", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "kernel": "k_persistent<BinomialTile>", "kernel_ms": med(kern_ms)},
        "cpu_baseline": cpu_base,
        "coexec": {
            "plain_gpu_items_per_s": items / T_bare, "vs_plain_gpu": s_real, "s_real": s_real, "s_max": s_max,
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
    achieved = 8.0 * iters / (med(kern) * 1e-3) / 1e12
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s (FP32 VALU lane-ops)", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "kernel": "k_batch_escape", "kernel_ms": med(kern), "iterations": iters},
        "cpu_baseline": cpu_base,
        "batch": {"separate_launch_ms": med(t_sep) * 1e3, "separate_gpu_ms": med(g_sep),
                  "graph_launch_ms": med(per_run) * 1e3, "graph_gpu_ms": med(kern),
                  "speedup_vs_separate": med(t_sep) / med(per_run), "jobs": len(jobs), "items": n_items},
    }
    print(json.dumps(res), flush=True)
    b.close()


def bench_copy(args, torch, stream):
    """Reference for the HBM counters and the achievable stream rate: a plain
    device copy of 256 MiB (the blur image's size), timed with HIP events."""
    dev = torch.device("cuda:0")
    a = torch.rand(8192 * 8192, device=dev)
    b = torch.empty_like(a)
    hev = HipEvents()
    s0, s1 = hev.create(), hev.create()
    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            b.copy_(a)
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.steps):
            hev.record(s0, stream.cuda_stream)
            b.copy_(a)
            hev.record(s1, stream.cuda_stream)
            ms.append(hev.elapsed_ms(s0, s1))
    nbytes = 2 * a.numel() * 4
    print(json.dumps({"workload": "device copy 256 MiB fp32", "bytes_per_copy": nbytes, "steps": args.steps,
                      "ms_median": med(ms), "GBps": nbytes / (med(ms) * 1e-3) / 1e9}), flush=True)


def bench_serve(args, ce, synth, torch, np, stream):
    """Serving: a Poisson trace of escape, blur and n-body jobs (200 jobs/s,
    sizes log-uniform; seed 0x5E2E) replayed in real time against the
    persistent serving kernel, and against one plain launch per job in
    arrival order. Inputs come from resident pools in HBM (a job of side s
    reads the first s*s pixels of one 16384^2 image; a job of n bodies the
    first n of 131,072); outputs are allocated per job from the HBM budget."""
    import threading
    trace = synth.serve_trace(args.serve_jobs)
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
    torch.cuda.synchronize()

    # --- one plain launch per job, in arrival order (FIFO, no overlap)
    log(f"serving trace: {len(trace)} jobs over {trace[-1].arrival_s:.1f} s; plain launches first")
    scratch = torch.empty(out_bytes, dtype=torch.uint8, device=dev)
    lat_plain = []
    t0 = time.perf_counter()
    for j, (kid, prm, ins, _) in zip(trace, specs):
        now = time.perf_counter() - t0
        if now < j.arrival_s:
            time.sleep(j.arrival_s - now)
        ce.ce_bare_run(kid, prm, ins, scratch, stream=stream.cuda_stream, sync=True)
        lat_plain.append(time.perf_counter() - t0 - j.arrival_s)
    wall_plain = time.perf_counter() - t0
    del scratch
    torch.cuda.synchronize()

    # --- the serving kernel
    log("serving kernel")
    srv = ce.Server(max(4 << 30, 8 * out_bytes), keep_outputs=False, session_timeout_s=600.0)
    warm = [srv.submit(*specs[i][:2], *specs[i][2]) for i in range(min(8, len(specs)))]
    for t in warm:
        srv.wait(t, 120.0)
    srv.drain(120.0)
    srv.close()
    srv = ce.Server(max(4 << 30, 8 * out_bytes), keep_outputs=False, session_timeout_s=600.0)
    tickets = []

    def client():
        c0 = time.perf_counter()
        for j, (kid, prm, ins, _) in zip(trace, specs):
            now = time.perf_counter() - c0
            if now < j.arrival_s:
                time.sleep(j.arrival_s - now)
            tickets.append(srv.submit(kid, prm, *ins))

    th = threading.Thread(target=client)
    th.start()
    th.join()
    for t in tickets:
        srv.wait(t, 600.0)
    srv.drain(120.0)
    r = srv.stats()
    srv.close()
    lat_plain.sort()
    pct = lambda v, q: float(np.percentile(np.asarray(v), q))
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
        "metric": METRIC, "value": r.items_per_s, "unit": "work-items/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": r.wall_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "mixed (u32 escape, f32 blur and n-body)", "data": "synthetic (seeded SplitMix64 trace, paper_1805_02755_amd/synth.py)",
        "config": {"workload": f"serving trace: {len(trace)} Poisson arrivals at 200/s, escape side [256,4096], "
                               "blur side [1024,16384], n-body [4096,131072]", "form": "persistent serving kernel"},
        "roofline": None,
        "cpu_baseline": cpu_base,
        "serve": {"jobs": int(r.completed), "items": int(r.items), "p50_ms": r.p50_s * 1e3, "p99_ms": r.p99_s * 1e3,
                  "mean_ms": r.mean_s * 1e3, "max_ms": r.max_s * 1e3, "wall_s": r.wall_s,
                  "jobs_per_s": r.jobs_per_s, "peak_hbm_bytes": int(r.peak_hbm),
                  "max_inflight": int(r.max_inflight_seen),
                  "plain_p50_ms": pct(lat_plain, 50) * 1e3, "plain_p99_ms": pct(lat_plain, 99) * 1e3,
                  "plain_wall_s": wall_plain, "plain_items_per_s": n_items / wall_plain},
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
