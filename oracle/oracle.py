"""Oracle for the co-execution hot path -- TEST INFRASTRUCTURE ONLY.

Thin numpy wrappers over ``liboracle.so`` (plain sequential C, see oracle.c)
plus plain-Python definitions of the scheduler sequences and of the metrics of
section 7.3. Only the tests, the smoke check and the bench's CPU-baseline leg
import this module; the engine never does, and this module imports nothing
from the engine package.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def lib():
    """Loads liboracle.so, building it with gcc if it is not there yet."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_escape_pixel.restype = C.c_uint32
        L.orc_escape_pixel.argtypes = [C.c_uint32, C.c_uint32, C.c_float, C.c_float, C.c_float,
                                       C.c_float, C.c_uint32]
        L.orc_escape.restype = None
        L.orc_escape.argtypes = [C.c_uint32, C.c_uint32, C.c_float, C.c_float, C.c_float, C.c_float,
                                 C.c_uint32, _u32p]
        L.orc_gauss5_weights.restype = None
        L.orc_gauss5_weights.argtypes = [C.c_double, _f32p]
        L.orc_blur5_pixel.restype = C.c_float
        L.orc_blur5_pixel.argtypes = [_f32p, C.c_uint32, C.c_uint32, _f32p, C.c_uint32, C.c_uint32]
        L.orc_blur5.restype = None
        L.orc_blur5.argtypes = [_f32p, C.c_uint32, C.c_uint32, _f32p, _f32p]
        L.orc_rsqrt_lomont.restype = C.c_float
        L.orc_rsqrt_lomont.argtypes = [C.c_float]
        L.orc_rsqrt_lomont_estimate.restype = C.c_float
        L.orc_rsqrt_lomont_estimate.argtypes = [C.c_float]
        L.orc_rsqrt_newton.restype = C.c_float
        L.orc_rsqrt_newton.argtypes = [C.c_float, C.c_float]
        L.orc_nbody_acc_body.restype = None
        L.orc_nbody_acc_body.argtypes = [_f32p, C.c_uint32, C.c_float, C.c_int, C.c_uint32, _f32p]
        L.orc_nbody_acc.restype = None
        L.orc_nbody_acc.argtypes = [_f32p, C.c_uint32, C.c_float, C.c_int, _f32p]
        L.orc_nbody_acc_f64.restype = None
        L.orc_nbody_acc_f64.argtypes = [_f32p, C.c_uint32, C.c_double, C.c_uint32, C.c_uint32, _f64p]
        L.orc_nbody_step_body.restype = None
        L.orc_nbody_step_body.argtypes = [_f32p, _f32p, C.c_uint32, C.c_float, C.c_float, C.c_int, C.c_uint32,
                                          _f32p, _f32p]
        L.orc_nbody_step.restype = None
        L.orc_nbody_step.argtypes = [_f32p, _f32p, C.c_uint32, C.c_float, C.c_float, C.c_int, _f32p, _f32p]
        L.orc_binomial_table.restype = None
        L.orc_binomial_table.argtypes = [C.c_uint32, C.c_double, C.c_double, C.c_double, _f32p,
                                         C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.orc_binomial_price.restype = C.c_float
        L.orc_binomial_price.argtypes = [C.c_float, C.c_float, C.c_uint32, _f32p, C.c_float, C.c_float]
        L.orc_static_plan.restype = C.c_int
        L.orc_static_plan.argtypes = [C.c_uint64, C.c_uint32, _f64p, _u32p, C.c_uint32, _u64p, _u64p]
        L.orc_hguided_size.restype = C.c_uint64
        L.orc_hguided_size.argtypes = [C.c_uint64, _u64p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64]
        _lib = L
    return _lib


# --------------------------------------------------------------------------
# payloads
# --------------------------------------------------------------------------
def escape_pixel(r, c, x0, y0, dx, dy, max_iter) -> int:
    return int(lib().orc_escape_pixel(r, c, x0, y0, dx, dy, max_iter))


def escape(w, h, x0, y0, dx, dy, max_iter) -> np.ndarray:
    out = np.empty((h, w), dtype=np.uint32)
    lib().orc_escape(w, h, x0, y0, dx, dy, max_iter, out)
    return out


def gauss5_weights(sigma: float = 1.0) -> np.ndarray:
    w = np.empty(25, dtype=np.float32)
    lib().orc_gauss5_weights(sigma, w)
    return w


def blur5(img: np.ndarray, wt: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.float32)
    h, w = img.shape
    out = np.empty_like(img)
    lib().orc_blur5(img, w, h, np.ascontiguousarray(wt, dtype=np.float32), out)
    return out


def blur5_pixel(img: np.ndarray, wt: np.ndarray, y: int, x: int) -> np.float32:
    img = np.ascontiguousarray(img, dtype=np.float32)
    h, w = img.shape
    return np.float32(lib().orc_blur5_pixel(img, w, h, np.ascontiguousarray(wt, dtype=np.float32), y, x))


def rsqrt_lomont(x: float) -> np.float32:
    return np.float32(lib().orc_rsqrt_lomont(x))


def rsqrt_lomont_estimate(x: float) -> np.float32:
    """Lomont's integer first estimate alone (no Newton step)."""
    return np.float32(lib().orc_rsqrt_lomont_estimate(x))


def rsqrt_newton(hx: float, y: float) -> np.float32:
    """One Newton step for 1/sqrt(x) from y, given hx = x/2."""
    return np.float32(lib().orc_rsqrt_newton(hx, y))


def nbody_acc(pos4: np.ndarray, eps2: float, strict: bool = True) -> np.ndarray:
    pos4 = np.ascontiguousarray(pos4, dtype=np.float32)
    out = np.empty_like(pos4)
    lib().orc_nbody_acc(pos4, pos4.shape[0], eps2, int(strict), out)
    return out


def nbody_acc_body(pos4: np.ndarray, eps2: float, i: int, strict: bool = True) -> np.ndarray:
    pos4 = np.ascontiguousarray(pos4, dtype=np.float32)
    out = np.empty(4, dtype=np.float32)
    lib().orc_nbody_acc_body(pos4, pos4.shape[0], eps2, int(strict), i, out)
    return out


def nbody_step(pos4: np.ndarray, vel4: np.ndarray, eps2: float, dt: float, strict: bool = True):
    """One integration step of every body: returns (positions, velocities)."""
    pos4 = np.ascontiguousarray(pos4, dtype=np.float32)
    vel4 = np.ascontiguousarray(vel4, dtype=np.float32)
    assert pos4.shape == vel4.shape and pos4.shape[1] == 4
    po, vo = np.empty_like(pos4), np.empty_like(vel4)
    lib().orc_nbody_step(pos4, vel4, pos4.shape[0], eps2, dt, int(strict), po, vo)
    return po, vo


def nbody_step_body(pos4: np.ndarray, vel4: np.ndarray, eps2: float, dt: float, i: int, strict: bool = True):
    pos4 = np.ascontiguousarray(pos4, dtype=np.float32)
    vel4 = np.ascontiguousarray(vel4, dtype=np.float32)
    po, vo = np.empty(4, np.float32), np.empty(4, np.float32)
    lib().orc_nbody_step_body(pos4, vel4, pos4.shape[0], eps2, dt, int(strict), i, po, vo)
    return po, vo


def binomial_table(steps: int, sigma: float, rate: float, T: float):
    """(leaf factors f_0..f_N as float32, pu, pd) of the Cox-Ross-Rubinstein tree."""
    f = np.empty(steps + 1, np.float32)
    pu, pd = C.c_float(), C.c_float()
    lib().orc_binomial_table(steps, sigma, rate, T, f, C.byref(pu), C.byref(pd))
    return f, np.float32(pu.value), np.float32(pd.value)


def binomial_price(S: float, X: float, steps: int, factors: np.ndarray, pu, pd) -> np.float32:
    f = np.ascontiguousarray(factors, dtype=np.float32)
    return np.float32(lib().orc_binomial_price(S, X, steps, f, float(pu), float(pd)))


def binomial(spots: np.ndarray, X: float, steps: int, factors: np.ndarray, pu, pd) -> np.ndarray:
    """Prices of every spot (any shape, float32), one call each."""
    s = np.ascontiguousarray(spots, dtype=np.float32)
    out = np.empty_like(s)
    flat, of = s.reshape(-1), out.reshape(-1)
    for k in range(flat.size):
        of[k] = binomial_price(float(flat[k]), X, steps, factors, pu, pd)
    return out


def nbody_acc_f64(pos4: np.ndarray, eps2: float, i0: int = 0, i1: int | None = None) -> np.ndarray:
    pos4 = np.ascontiguousarray(pos4, dtype=np.float32)
    n = pos4.shape[0]
    i1 = n if i1 is None else i1
    out = np.empty((i1 - i0, 3), dtype=np.float64)
    lib().orc_nbody_acc_f64(pos4, n, eps2, i0, i1, out)
    return out


# --------------------------------------------------------------------------
# schedulers (section 5.3)
# --------------------------------------------------------------------------
def static_plan(G: int, props, order, n_bands: int = 0):
    """Returns [(begin, end)] per device (device order), or None if invalid."""
    n = len(order)
    p = np.ascontiguousarray(np.asarray(list(props) + [0.0] * (max(n - 1, 0) - len(props)),
                                        dtype=np.float64)[: max(n - 1, 1)])
    if p.size == 0:
        p = np.zeros(1)
    o = np.ascontiguousarray(np.asarray(order, dtype=np.uint32))
    b = np.zeros(n, dtype=np.uint64)
    e = np.zeros(n, dtype=np.uint64)
    rc = lib().orc_static_plan(G, n, p, o, n_bands, b, e)
    if rc != 0:
        return None
    return [(int(b[d]), int(e[d])) for d in range(n)]


def hguided_size(G_r: int, P, k: int, i: int, min_i: int) -> int:
    Pa = np.ascontiguousarray(np.asarray(P, dtype=np.uint64))
    return int(lib().orc_hguided_size(G_r, Pa, len(P), k, i, min_i))


def hguided_sequence(G: int, P, k: int, mins, requests) -> list[tuple[int, int, int]]:
    """Packages (device, begin, size) when devices ask in the order given by
    the iterable ``requests`` until nothing is pending."""
    nxt = 0
    out = []
    for dev in requests:
        if nxt >= G:
            break
        s = hguided_size(G - nxt, P, k, dev, mins[dev])
        out.append((dev, nxt, s))
        nxt += s
    return out


def dynamic_sequence(G: int, package: int, requests) -> list[tuple[int, int, int]]:
    """Dynamic (section 5.3): equal packages of ``package`` granules handed in
    index order to whichever device asks; the last one may be short."""
    nxt = 0
    out = []
    for dev in requests:
        if nxt >= G:
            break
        s = min(package, G - nxt)
        out.append((dev, nxt, s))
        nxt += s
    return out


def dynamic_package_for_count(G: int, n_packages: int) -> int:
    """Package size when Dynamic is given a package count: ceil(G / count)."""
    return -(-G // n_packages)


# --------------------------------------------------------------------------
# metrics (section 7.3)
# --------------------------------------------------------------------------
def overhead_pct(t_engine: float, t_native: float) -> float:
    """Overhead = (T_engine - T_native) / T_native * 100."""
    return (t_engine - t_native) / t_native * 100.0


def balance(t_devices) -> float:
    """Balance = T_first_finisher / T_last_finisher."""
    t = list(t_devices)
    return min(t) / max(t)


def s_max(t_standalone) -> float:
    """Maximum achievable speedup over the fastest device: T_min * sum 1/T_i
    (throughput reading of the formula of section 7.3)."""
    t = list(t_standalone)
    return min(t) * sum(1.0 / x for x in t)


def efficiency(s_real: float, s_max_value: float) -> float:
    return s_real / s_max_value


@dataclass
class Coverage:
    ok: bool
    missing: int
    duplicated: int


def coverage(G: int, packages) -> Coverage:
    """Counts how often each granule is covered by packages (begin, size)."""
    cnt = np.zeros(G, dtype=np.int64)
    for b, s in packages:
        cnt[b:b + s] += 1
    return Coverage(bool(np.all(cnt == 1)), int(np.sum(cnt == 0)), int(np.sum(cnt > 1)))
