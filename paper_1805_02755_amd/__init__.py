"""Python binding of the MI355X co-execution engine (libcoexec.so).

Argument marshalling only: every step of a run executes inside the native
library (HIP kernels on the GPU, C++ workers on the host cores). The names
follow the C ABI declared in include/coexec.h. There is no fallback: if the
library is not built, loading it raises.

The library is loaded lazily, so ``import paper_1805_02755_amd.synth`` does
not touch it.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoexec.so")

# status codes
CE_OK = 0
CE_E_INVALID = -1
CE_E_STATE = -2
CE_E_NOMEM = -3
CE_E_DEVICE = -4
CE_E_UNSUPPORTED = -5
CE_E_BUDGET = -6
CE_E_TIMEOUT = -7
STATUS_NAMES = {0: "CE_OK", -1: "CE_E_INVALID", -2: "CE_E_STATE", -3: "CE_E_NOMEM", -4: "CE_E_DEVICE",
                -5: "CE_E_UNSUPPORTED", -6: "CE_E_BUDGET", -7: "CE_E_TIMEOUT"}

CE_DEV_GPU = 1
CE_DEV_HOST = 2
CE_MAX_DEVICES = 2

CE_KERNEL_ESCAPE = 1
CE_KERNEL_BLUR5 = 2
CE_KERNEL_NBODY_ACC = 3
CE_KERNEL_NBODY_STEP = 4
CE_KERNEL_BINOMIAL = 5
CE_KERNEL_RUNTIME = 6
CE_RT_MAX_BUFS = 4
CE_RT_SCALAR_BYTES = 128

CE_SCHED_STATIC = 0
CE_SCHED_DYNAMIC = 1
CE_SCHED_HGUIDED = 2
CE_ORDER_HOST_FIRST = 0
CE_ORDER_GPU_FIRST = 1

CE_MERGE_DMA = 0
CE_MERGE_GPU_GATHER = 1

EXPORTED_SYMBOLS = (
    "ce_engine_create", "ce_engine_destroy", "ce_engine_use", "ce_engine_work_items", "ce_engine_scheduler",
    "ce_engine_stream", "ce_engine_output_merge", "ce_engine_gpu_workgroups", "ce_engine_wait_bounds", "ce_engine_kernel_events", "ce_program_kernel", "ce_program_in", "ce_program_out", "ce_program_out_pattern",
    "ce_engine_run", "ce_engine_run_noalloc", "ce_engine_stats", "ce_engine_trace", "ce_engine_has_errors", "ce_engine_error_count",
    "ce_engine_error", "ce_engine_clear_errors", "ce_stream_copy", "ce_bare_run", "ce_bare_run_outs", "ce_sched_static_plan", "ce_sched_hguided_size",
    "ce_gauss5_weights", "ce_binomial_table", "ce_version", "ce_batch_create", "ce_batch_destroy", "ce_batch_add_escape",
    "ce_batch_clear", "ce_batch_set_config", "ce_batch_get_config", "ce_batch_tune", "ce_batch_run",
    "ce_batch_run_separate", "ce_batch_stats", "ce_batch_error", "ce_server_create", "ce_server_destroy",
    "ce_server_submit", "ce_server_job_ticks", "ce_server_poll", "ce_server_wait", "ce_server_output", "ce_server_copy_output",
    "ce_server_release", "ce_server_drain", "ce_server_stats", "ce_server_error", "ce_program_source",
    "ce_rt_compile_check", "ce_rt_code_object", "ce_engine_bare_run_source",
)

CE_JOB_QUEUED = 0
CE_JOB_ADMITTED = 1
CE_JOB_DONE = 2
CE_JOB_FAILED = 3


class ce_escape_params(C.Structure):
    _fields_ = [("w", C.c_uint32), ("h", C.c_uint32), ("x0", C.c_float), ("y0", C.c_float), ("dx", C.c_float),
                ("dy", C.c_float), ("max_iter", C.c_uint32)]


class ce_blur5_params(C.Structure):
    _fields_ = [("w", C.c_uint32), ("h", C.c_uint32)]


class ce_nbody_params(C.Structure):
    _fields_ = [("n", C.c_uint32), ("eps2", C.c_float), ("strict", C.c_uint32)]


class ce_nbody_step_params(C.Structure):
    _fields_ = [("n", C.c_uint32), ("eps2", C.c_float), ("dt", C.c_float), ("strict", C.c_uint32)]


class ce_binomial_params(C.Structure):
    _fields_ = [("n_groups", C.c_uint32), ("steps", C.c_uint32), ("strike", C.c_float), ("pu", C.c_float),
                ("pd", C.c_float)]


class ce_rt_args(C.Structure):
    _fields_ = [("buf", C.c_void_p * CE_RT_MAX_BUFS), ("scalars", C.c_ubyte * CE_RT_SCALAR_BYTES)]


# host version of a runtime payload: (i0, i1, const ce_rt_args*)
CE_RT_HOST_FN = C.CFUNCTYPE(C.c_int32, C.c_uint64, C.c_uint64, C.POINTER(ce_rt_args))


class ce_rt_desc(C.Structure):
    _fields_ = [("source", C.c_char_p), ("entry", C.c_char_p), ("host", C.c_void_p), ("n_in", C.c_uint32),
                ("n_out", C.c_uint32), ("in_bytes", C.c_uint64 * 2), ("out_item_bytes", C.c_uint32),
                ("scalar_bytes", C.c_uint32), ("scalars", C.c_void_p)]


class ce_sched_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("order", C.c_int32), ("n_packages", C.c_uint32), ("k", C.c_uint32),
                ("package_granules", C.c_uint64), ("props", C.c_double * CE_MAX_DEVICES),
                ("power", C.c_uint64 * CE_MAX_DEVICES), ("min_granules", C.c_uint64 * CE_MAX_DEVICES)]


class ce_run_stats(C.Structure):
    _fields_ = [("t_run", C.c_double), ("t_device", C.c_double * CE_MAX_DEVICES), ("t_gpu_kernel", C.c_double),
                ("granules", C.c_uint64 * CE_MAX_DEVICES), ("items", C.c_uint64 * CE_MAX_DEVICES),
                ("packages", C.c_uint64 * CE_MAX_DEVICES), ("n_devices", C.c_uint32),
                ("device_kind", C.c_uint32 * CE_MAX_DEVICES), ("balance", C.c_double),
                ("total_granules", C.c_uint64), ("total_items", C.c_uint64), ("gpu_workgroups", C.c_uint32),
                ("host_threads", C.c_uint32), ("t_gather", C.c_double), ("gathered_bytes", C.c_uint64),
                ("t_launched", C.c_double), ("t_host_done", C.c_double), ("t_gpu_seen", C.c_double),
                ("t_synced", C.c_double), ("t_copies_done", C.c_double)]


class ce_batch_config(C.Structure):
    _fields_ = [("tile_rows", C.c_uint32), ("tile_cols", C.c_uint32), ("package_tiles", C.c_uint32)]


class ce_batch_report(C.Structure):
    _fields_ = [("jobs", C.c_uint32), ("workgroups", C.c_uint32), ("items", C.c_uint64),
                ("total_tiles", C.c_uint64), ("tile_rows", C.c_uint32), ("tile_cols", C.c_uint32),
                ("package_tiles", C.c_uint32), ("pad", C.c_uint32), ("t_run", C.c_double),
                ("t_gpu_ms", C.c_double), ("launches", C.c_uint64)]


class ce_server_config(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_inflight", C.c_uint32), ("keep_outputs", C.c_uint32),
                ("max_jobs", C.c_uint32), ("workgroups_per_cu", C.c_uint32), ("session_timeout_s", C.c_double)]


class ce_job(C.Structure):
    _fields_ = [("kernel_id", C.c_int32), ("pad", C.c_uint32), ("esc", ce_escape_params), ("blur", ce_blur5_params),
                ("nb", ce_nbody_params), ("in0_dev", C.c_void_p), ("in1_dev", C.c_void_p),
                ("in0_host", C.c_void_p), ("in1_host", C.c_void_p)]


class ce_server_report(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("items", C.c_uint64),
                ("p50_s", C.c_double), ("p99_s", C.c_double), ("mean_s", C.c_double), ("max_s", C.c_double),
                ("wall_s", C.c_double), ("items_per_s", C.c_double), ("jobs_per_s", C.c_double),
                ("peak_hbm", C.c_uint64), ("max_inflight_seen", C.c_uint64)]


class ce_package_rec(C.Structure):
    _fields_ = [("device", C.c_uint32), ("pad", C.c_uint32), ("begin", C.c_uint64), ("end", C.c_uint64),
                ("t_claim", C.c_double), ("t_end", C.c_double)]


_lib = None


def lib():
    """Loads libcoexec.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python -m paper_1805_02755_amd._build")
    _lib = load(LIB_PATH)
    return _lib


def load(path: str):
    """Opens a library exporting the C ABI and declares its signatures."""
    L = C.CDLL(path)
    vp, sz, u32, u64, i32 = C.c_void_p, C.c_size_t, C.c_uint32, C.c_uint64, C.c_int32
    sigs = {
        "ce_engine_create": (i32, [C.POINTER(vp)]),
        "ce_engine_destroy": (None, [vp]),
        "ce_engine_use": (i32, [vp, u32, C.c_int, C.c_int]),
        "ce_engine_work_items": (i32, [vp, u32, C.POINTER(u64), C.POINTER(u32)]),
        "ce_engine_scheduler": (i32, [vp, C.POINTER(ce_sched_desc)]),
        "ce_engine_stream": (i32, [vp, vp]),
        "ce_engine_kernel_events": (i32, [vp, vp, vp]),
        "ce_engine_output_merge": (i32, [vp, C.c_int]),
        "ce_engine_gpu_workgroups": (i32, [vp, u32]),
        "ce_engine_wait_bounds": (i32, [vp, C.c_double, C.c_double]),
        "ce_program_kernel": (i32, [vp, C.c_int, vp, sz]),
        "ce_program_in": (i32, [vp, u32, vp, vp, sz]),
        "ce_program_out": (i32, [vp, u32, vp, vp, sz]),
        "ce_program_out_pattern": (i32, [vp, u32, u32]),
        "ce_engine_run": (i32, [vp]),
        "ce_engine_run_noalloc": (i32, [vp]),
        "ce_engine_stats": (i32, [vp, C.POINTER(ce_run_stats)]),
        "ce_engine_trace": (sz, [vp, C.POINTER(ce_package_rec), sz]),
        "ce_engine_has_errors": (C.c_int, [vp]),
        "ce_engine_error_count": (C.c_int, [vp]),
        "ce_engine_error": (C.c_char_p, [vp, C.c_int]),
        "ce_engine_clear_errors": (None, [vp]),
        "ce_bare_run": (i32, [C.c_int, vp, sz, C.POINTER(vp), vp, vp, C.c_int]),
        "ce_stream_copy": (i32, [vp, vp, sz, vp, C.c_int]),
        "ce_bare_run_outs": (i32, [C.c_int, vp, sz, C.POINTER(vp), C.POINTER(vp), C.c_uint32, vp, C.c_int]),
        "ce_program_source": (i32, [vp, C.POINTER(ce_rt_desc), C.c_char_p, sz]),
        "ce_rt_compile_check": (i32, [C.c_char_p, C.c_char_p, C.c_char_p, sz]),
        "ce_rt_code_object": (i32, [C.c_char_p, C.c_char_p, vp, sz, C.POINTER(sz), C.c_char_p, sz]),
        "ce_engine_bare_run_source": (i32, [vp, u64, u32, C.POINTER(vp), C.POINTER(vp), vp, C.c_int]),
        "ce_sched_static_plan": (i32, [u64, u32, C.POINTER(C.c_double), C.POINTER(u32), u32, C.POINTER(u64),
                                       C.POINTER(u64)]),
        "ce_sched_hguided_size": (u64, [u64, C.POINTER(u64), u32, u32, u32, u64]),
        "ce_gauss5_weights": (i32, [C.c_double, C.POINTER(C.c_float)]),
        "ce_binomial_table": (i32, [C.c_uint32, C.c_double, C.c_double, C.c_double, C.POINTER(C.c_float),
                                    C.POINTER(C.c_float), C.POINTER(C.c_float)]),
        "ce_version": (C.c_char_p, []),
        "ce_batch_create": (i32, [C.POINTER(vp), vp]),
        "ce_batch_destroy": (None, [vp]),
        "ce_batch_add_escape": (i32, [vp, C.POINTER(ce_escape_params), vp, C.POINTER(u32)]),
        "ce_batch_clear": (i32, [vp]),
        "ce_batch_set_config": (i32, [vp, C.POINTER(ce_batch_config)]),
        "ce_batch_get_config": (i32, [vp, C.POINTER(ce_batch_config)]),
        "ce_batch_tune": (i32, [vp, u32, C.POINTER(ce_batch_config)]),
        "ce_batch_run": (i32, [vp]),
        "ce_batch_run_separate": (i32, [vp]),
        "ce_batch_stats": (i32, [vp, C.POINTER(ce_batch_report)]),
        "ce_batch_error": (C.c_char_p, [vp]),
        "ce_server_create": (i32, [C.POINTER(ce_server_config), vp, C.POINTER(vp)]),
        "ce_server_destroy": (None, [vp]),
        "ce_server_submit": (i32, [vp, C.POINTER(ce_job), C.POINTER(u64)]),
        "ce_server_job_ticks": (i32, [vp, u64, C.POINTER(u64), C.POINTER(u64)]),
        "ce_server_poll": (i32, [vp, u64, C.POINTER(i32)]),
        "ce_server_wait": (i32, [vp, u64, C.c_double]),
        "ce_server_output": (i32, [vp, u64, C.POINTER(vp), C.POINTER(sz)]),
        "ce_server_copy_output": (i32, [vp, u64, vp, sz]),
        "ce_server_release": (i32, [vp, u64]),
        "ce_server_drain": (i32, [vp, C.c_double]),
        "ce_server_stats": (i32, [vp, C.POINTER(ce_server_report)]),
        "ce_server_error": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sigs.items():
        try:
            f = getattr(L, name)
        except AttributeError:
            if path == LIB_PATH:
                raise
            continue  # a test build with part of the ABI
        f.restype = res
        f.argtypes = args
    return L


class CoexecError(RuntimeError):
    def __init__(self, status: int, where: str, messages=()):
        self.status = status
        self.messages = list(messages)
        msg = f"{where}: {STATUS_NAMES.get(status, status)}"
        if self.messages:
            msg += " -- " + " | ".join(self.messages)
        super().__init__(msg)


def _ptr(x) -> Optional[int]:
    """Address of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _nbytes(x) -> int:
    if hasattr(x, "nbytes"):
        return int(x.nbytes)
    if hasattr(x, "element_size"):
        return int(x.numel() * x.element_size())
    raise TypeError(f"cannot size {type(x)}")


# ---------------------------------------------------------------- free functions
def ce_version() -> str:
    return lib().ce_version().decode()


def ce_binomial_table(steps: int, sigma: float, rate: float, T: float):
    """Leaf factors (steps+1 float32), pu and pd of CE_KERNEL_BINOMIAL's tree."""
    import numpy as np
    f = np.empty(steps + 1, dtype=np.float32)
    pu, pd = C.c_float(), C.c_float()
    st = lib().ce_binomial_table(steps, sigma, rate, T, f.ctypes.data_as(C.POINTER(C.c_float)), C.byref(pu),
                                 C.byref(pd))
    if st != CE_OK:
        raise CoexecError(st, "ce_binomial_table")
    return f, np.float32(pu.value), np.float32(pd.value)


def ce_gauss5_weights(sigma: float = 1.0):
    import numpy as np
    w = np.empty(25, dtype=np.float32)
    st = lib().ce_gauss5_weights(sigma, w.ctypes.data_as(C.POINTER(C.c_float)))
    if st != CE_OK:
        raise CoexecError(st, "ce_gauss5_weights")
    return w


def ce_sched_static_plan(G: int, props, order, n_bands: int = 0):
    n = len(order)
    p = (C.c_double * max(1, n - 1))(*(list(props)[: n - 1] or [0.0]))
    o = (C.c_uint32 * n)(*order)
    b = (C.c_uint64 * n)()
    e = (C.c_uint64 * n)()
    st = lib().ce_sched_static_plan(G, n, p, o, n_bands, b, e)
    if st != CE_OK:
        return None
    return [(int(b[d]), int(e[d])) for d in range(n)]


def ce_sched_hguided_size(G_r: int, power, k: int, i: int, min_i: int) -> int:
    P = (C.c_uint64 * len(power))(*power)
    return int(lib().ce_sched_hguided_size(G_r, P, len(power), k, i, min_i))


def _params(kernel_id: int, params):
    return params, C.sizeof(params)


def ce_bare_run(kernel_id: int, params, ins, out, stream=None, sync: bool = True) -> None:
    """One plain grid launch of the payload over the whole space (device pointers)."""
    arr = (C.c_void_p * max(1, len(ins)))(*[_ptr(x) for x in ins]) if ins else None
    st = lib().ce_bare_run(kernel_id, C.byref(params), C.sizeof(params), arr, _ptr(out),
                           _ptr(stream) if stream is not None else None, int(sync))
    if st != CE_OK:
        raise CoexecError(st, "ce_bare_run")


def ce_stream_copy(dst, src, nbytes: int, stream=None, sync: bool = True) -> None:
    """The streaming-copy bandwidth reference (device pointers)."""
    st = lib().ce_stream_copy(_ptr(dst), _ptr(src), nbytes, _ptr(stream) if stream is not None else None, int(sync))
    if st != CE_OK:
        raise CoexecError(st, "ce_stream_copy")


def ce_bare_run_outs(kernel_id: int, params, ins, outs, stream=None, sync: bool = True) -> None:
    """As ce_bare_run for payloads with several outputs (device pointers)."""
    arr = (C.c_void_p * max(1, len(ins)))(*[_ptr(x) for x in ins]) if ins else None
    oarr = (C.c_void_p * len(outs))(*[_ptr(x) for x in outs])
    st = lib().ce_bare_run_outs(kernel_id, C.byref(params), C.sizeof(params), arr, oarr, len(outs),
                                _ptr(stream) if stream is not None else None, int(sync))
    if st != CE_OK:
        raise CoexecError(st, "ce_bare_run_outs")


def ce_rt_compile_check(source: str, entry: str):
    """Compiles a runtime payload's source for gfx950 (no GPU needed).
    Returns (status, compiler log)."""
    buf = C.create_string_buffer(1 << 16)
    st = lib().ce_rt_compile_check(source.encode(), entry.encode(), buf, len(buf))
    return st, buf.value.decode(errors="replace")


def ce_rt_code_object(source: str, entry: str) -> bytes:
    """The gfx950 code object hipRTC builds for a runtime payload."""
    n = C.c_size_t(0)
    log = C.create_string_buffer(1 << 16)
    st = lib().ce_rt_code_object(source.encode(), entry.encode(), None, 0, C.byref(n), log, len(log))
    if st != CE_OK:
        raise CoexecError(st, "ce_rt_code_object", [log.value.decode(errors="replace")])
    buf = C.create_string_buffer(n.value)
    st = lib().ce_rt_code_object(source.encode(), entry.encode(), buf, n.value, C.byref(n), log, len(log))
    if st != CE_OK:
        raise CoexecError(st, "ce_rt_code_object", [log.value.decode(errors="replace")])
    return buf.raw[:n.value]


def stream_handle(stream) -> Optional[int]:
    """hipStream_t of a torch.cuda.Stream (or None)."""
    if stream is None:
        return None
    return int(stream.cuda_stream)


# ---------------------------------------------------------------- engine
class Engine:
    """Owns one ce_engine; methods mirror the C calls one to one."""

    def __init__(self, library=None):
        self._L = library if library is not None else lib()
        h = C.c_void_p()
        st = self._L.ce_engine_create(C.byref(h))
        if st != CE_OK:
            raise CoexecError(st, "ce_engine_create")
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            self._L.ce_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def errors(self):
        L = self._L
        return [L.ce_engine_error(self._h, i).decode() for i in range(L.ce_engine_error_count(self._h))]

    def clear_errors(self):
        self._L.ce_engine_clear_errors(self._h)

    def _check(self, st, where):
        if st != CE_OK:
            raise CoexecError(st, where, self.errors()[-3:])
        return st

    def use(self, dev_mask: int, gpu_ordinal: int = 0, host_threads: int = 0):
        return self._check(self._L.ce_engine_use(self._h, dev_mask, gpu_ordinal, host_threads), "ce_engine_use")

    def work_items(self, gws, lws=None):
        g = (C.c_uint64 * len(gws))(*gws)
        l = (C.c_uint32 * len(lws))(*lws) if lws else None
        return self._check(self._L.ce_engine_work_items(self._h, len(gws), g, l), "ce_engine_work_items")

    def scheduler(self, kind: int, order: int = CE_ORDER_HOST_FIRST, n_packages: int = 0, k: int = 2,
                  package_granules: int = 0, props=(), power=(), min_granules=()):
        d = ce_sched_desc()
        d.kind, d.order, d.n_packages, d.k, d.package_granules = kind, order, n_packages, k, package_granules
        for i, v in enumerate(props):
            d.props[i] = v
        for i, v in enumerate(power):
            d.power[i] = v
        for i, v in enumerate(min_granules):
            d.min_granules[i] = v
        return self._check(self._L.ce_engine_scheduler(self._h, C.byref(d)), "ce_engine_scheduler")

    def stream(self, hip_stream):
        return self._check(self._L.ce_engine_stream(self._h, hip_stream), "ce_engine_stream")

    def output_merge(self, mode: int):
        return self._check(self._L.ce_engine_output_merge(self._h, mode), "ce_engine_output_merge")

    def wait_bounds(self, dispenser_s: float = 0.0, gather_s: float = 0.0):
        return self._check(self._L.ce_engine_wait_bounds(self._h, dispenser_s, gather_s), "ce_engine_wait_bounds")

    def gpu_workgroups(self, workgroups: int):
        return self._check(self._L.ce_engine_gpu_workgroups(self._h, workgroups), "ce_engine_gpu_workgroups")

    def kernel_events(self, start=None, stop=None):
        """Records torch.cuda.Event objects (or raw hipEvent_t) around the GPU kernel."""
        a = None if start is None else int(getattr(start, "cuda_event", start))
        b = None if stop is None else int(getattr(stop, "cuda_event", stop))
        return self._check(self._L.ce_engine_kernel_events(self._h, a, b), "ce_engine_kernel_events")

    def program_kernel(self, kernel_id: int, params):
        self._params = params
        return self._check(self._L.ce_program_kernel(self._h, kernel_id, C.byref(params), C.sizeof(params)),
                           "ce_program_kernel")

    def program_in(self, slot: int, host=None, dev=None, nbytes: Optional[int] = None):
        nb = nbytes if nbytes is not None else _nbytes(host if host is not None else dev)
        self._keep += [host, dev]
        return self._check(self._L.ce_program_in(self._h, slot, _ptr(host), _ptr(dev), nb), "ce_program_in")

    def program_out(self, slot: int, host=None, dev=None, nbytes: Optional[int] = None):
        nb = nbytes if nbytes is not None else _nbytes(host if host is not None else dev)
        self._keep += [host, dev]
        return self._check(self._L.ce_program_out(self._h, slot, _ptr(host), _ptr(dev), nb), "ce_program_out")

    def program_out_pattern(self, outs: int, items: int):
        return self._check(self._L.ce_program_out_pattern(self._h, outs, items), "ce_program_out_pattern")

    def program_source(self, source: str, entry: str, host=None, n_in: int = 0, n_out: int = 1, in_bytes=(),
                       out_item_bytes: int = 4, scalars: bytes = b""):
        """Binds a payload given as HIP source (compiled for gfx950 now) and,
        for the host workers, `host`: a CE_RT_HOST_FN or a raw C function
        address. Returns the compiler's log; raises CoexecError on failure."""
        d = ce_rt_desc()
        src, ent = source.encode(), entry.encode()
        d.source, d.entry = src, ent
        if host is None:
            d.host = None
        elif isinstance(host, int):
            d.host = host
        else:
            d.host = C.cast(host, C.c_void_p).value
        d.n_in, d.n_out = n_in, n_out
        for k, b in enumerate(in_bytes):
            d.in_bytes[k] = b
        d.out_item_bytes = out_item_bytes
        sc = C.create_string_buffer(bytes(scalars), max(1, len(scalars)))
        d.scalar_bytes, d.scalars = len(scalars), C.cast(sc, C.c_void_p).value if scalars else None
        self._keep += [src, ent, host, sc]
        log = C.create_string_buffer(1 << 16)
        st = self._L.ce_program_source(self._h, C.byref(d), log, len(log))
        text = log.value.decode(errors="replace")
        if st != CE_OK:
            raise CoexecError(st, "ce_program_source", self.errors()[-3:] + ([text] if text else []))
        return text

    def bare_run_source(self, gws: int, lws: int, ins, outs, stream=None, sync: bool = True):
        """Plain single launch of the bound runtime payload (device pointers)."""
        arr = (C.c_void_p * max(1, len(ins)))(*[_ptr(x) for x in ins]) if ins else None
        oarr = (C.c_void_p * len(outs))(*[_ptr(x) for x in outs])
        return self._check(self._L.ce_engine_bare_run_source(self._h, gws, lws, arr, oarr,
                                                             _ptr(stream) if stream is not None else None,
                                                             int(sync)), "ce_engine_bare_run_source")

    def run(self):
        return self._check(self._L.ce_engine_run(self._h), "ce_engine_run")

    def run_status(self) -> int:
        return int(self._L.ce_engine_run(self._h))

    def run_noalloc(self):
        return self._check(self._L.ce_engine_run_noalloc(self._h), "ce_engine_run_noalloc")

    def run_noalloc_status(self) -> int:
        return int(self._L.ce_engine_run_noalloc(self._h))

    def stats(self) -> ce_run_stats:
        s = ce_run_stats()
        self._check(self._L.ce_engine_stats(self._h, C.byref(s)), "ce_engine_stats")
        return s

    def trace(self):
        n = self._L.ce_engine_trace(self._h, None, 0)
        buf = (ce_package_rec * max(1, n))()
        n = self._L.ce_engine_trace(self._h, buf, n)
        return [(r.device, r.begin, r.end, r.t_claim, r.t_end) for r in buf[:n]]


class Batch:
    """Owns one ce_batch (the batched form); methods mirror the C calls."""

    def __init__(self, stream=None, library=None):
        self._L = library if library is not None else lib()
        h = C.c_void_p()
        st = self._L.ce_batch_create(C.byref(h), stream)
        if st != CE_OK:
            raise CoexecError(st, "ce_batch_create")
        self._h = h
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            self._L.ce_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, where):
        if st != CE_OK:
            msg = self._L.ce_batch_error(self._h)
            raise CoexecError(st, where, [msg.decode()] if msg else [])
        return st

    def add_escape(self, params, dev_out) -> int:
        idx = C.c_uint32()
        self._keep.append(dev_out)
        self._check(self._L.ce_batch_add_escape(self._h, C.byref(params), _ptr(dev_out), C.byref(idx)),
                    "ce_batch_add_escape")
        return int(idx.value)

    def clear(self):
        self._keep = []
        return self._check(self._L.ce_batch_clear(self._h), "ce_batch_clear")

    def set_config(self, tile_rows: int, package_tiles: int):
        c = ce_batch_config(tile_rows, 0, package_tiles)
        return self._check(self._L.ce_batch_set_config(self._h, C.byref(c)), "ce_batch_set_config")

    def get_config(self):
        c = ce_batch_config()
        self._check(self._L.ce_batch_get_config(self._h, C.byref(c)), "ce_batch_get_config")
        return (c.tile_rows, c.tile_cols, c.package_tiles)

    def tune(self, reps: int = 3):
        c = ce_batch_config()
        self._check(self._L.ce_batch_tune(self._h, reps, C.byref(c)), "ce_batch_tune")
        return (c.tile_rows, c.tile_cols, c.package_tiles)

    def run(self):
        return self._check(self._L.ce_batch_run(self._h), "ce_batch_run")

    def run_separate(self):
        return self._check(self._L.ce_batch_run_separate(self._h), "ce_batch_run_separate")

    def stats(self) -> ce_batch_report:
        s = ce_batch_report()
        self._check(self._L.ce_batch_stats(self._h, C.byref(s)), "ce_batch_stats")
        return s


class Server:
    """Owns one ce_server (the serving form); methods mirror the C calls.

    Host inputs passed to ``submit`` are kept alive until the job finishes.
    """

    def __init__(self, hbm_budget: int, max_inflight: int = 0, keep_outputs: bool = False, max_jobs: int = 0,
                 workgroups_per_cu: int = 0, session_timeout_s: float = 0.0, stream=None, library=None):
        self._L = library if library is not None else lib()
        cfg = ce_server_config(hbm_budget, max_inflight, 1 if keep_outputs else 0, max_jobs, workgroups_per_cu,
                               session_timeout_s)
        h = C.c_void_p()
        st = self._L.ce_server_create(C.byref(cfg), stream, C.byref(h))
        if st != CE_OK:
            raise CoexecError(st, "ce_server_create")
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            self._L.ce_server_destroy(self._h)
            self._h = None
            self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, where):
        if st != CE_OK:
            msg = self._L.ce_server_error(self._h)
            raise CoexecError(st, where, [msg.decode()] if msg else [])
        return st

    def submit(self, kernel_id: int, params, in0=None, in1=None) -> int:
        """Submits one job. Inputs that are device tensors stay resident and
        are read in place; numpy arrays are copied into HBM at admission."""
        j = ce_job()
        j.kernel_id = kernel_id
        if kernel_id == CE_KERNEL_ESCAPE:
            j.esc = params
        elif kernel_id == CE_KERNEL_BLUR5:
            j.blur = params
        elif kernel_id == CE_KERNEL_NBODY_ACC:
            j.nb = params
        keep = []
        for slot, x in ((0, in0), (1, in1)):
            if x is None:
                continue
            keep.append(x)
            is_dev = hasattr(x, "is_cuda") and x.is_cuda
            if is_dev:
                setattr(j, f"in{slot}_dev", _ptr(x))
            else:
                setattr(j, f"in{slot}_host", _ptr(x))
        t = C.c_uint64()
        self._check(self._L.ce_server_submit(self._h, C.byref(j), C.byref(t)), "ce_server_submit")
        if keep:
            self._keep[int(t.value)] = keep
        return int(t.value)

    def job_ticks(self, ticket: int):
        """(first tile start, last tile end) of a finished job, in GPU ticks."""
        a, b = C.c_uint64(), C.c_uint64()
        self._check(self._L.ce_server_job_ticks(self._h, ticket, C.byref(a), C.byref(b)), "ce_server_job_ticks")
        return int(a.value), int(b.value)

    def poll(self, ticket: int) -> int:
        v = C.c_int32()
        self._check(self._L.ce_server_poll(self._h, ticket, C.byref(v)), "ce_server_poll")
        return int(v.value)

    def wait(self, ticket: int, timeout_s: float = 60.0):
        try:
            return self._check(self._L.ce_server_wait(self._h, ticket, timeout_s), "ce_server_wait")
        finally:
            if self.poll(ticket) in (CE_JOB_DONE, CE_JOB_FAILED):
                self._keep.pop(ticket, None)

    def output(self, ticket: int):
        p, n = C.c_void_p(), C.c_size_t()
        self._check(self._L.ce_server_output(self._h, ticket, C.byref(p), C.byref(n)), "ce_server_output")
        return p.value, int(n.value)

    def copy_output(self, ticket: int, dst):
        """Copies a finished job's output into the numpy array ``dst``."""
        self._check(self._L.ce_server_copy_output(self._h, ticket, _ptr(dst), _nbytes(dst)), "ce_server_copy_output")
        return dst

    def release(self, ticket: int):
        self._keep.pop(ticket, None)
        return self._check(self._L.ce_server_release(self._h, ticket), "ce_server_release")

    def drain(self, timeout_s: float = 120.0):
        try:
            return self._check(self._L.ce_server_drain(self._h, timeout_s), "ce_server_drain")
        finally:
            self._keep = {}

    def stats(self) -> ce_server_report:
        r = ce_server_report()
        self._check(self._L.ce_server_stats(self._h, C.byref(r)), "ce_server_stats")
        return r
