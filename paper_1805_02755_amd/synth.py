"""Seeded synthetic workloads shared by the tests, the bench and the oracle checks.

This module generates inputs only: it holds none of the payload arithmetic,
scheduling or metric code. Every random draw comes from SplitMix64 (Steele,
Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014),
used as a counter-based generator: draw ``i`` of stream ``s`` under seed ``k``
is ``mix64(base(k, s) + (i + 1) * GOLDEN)``. A float in [0, 1) is the top 24
bits of a draw times 2**-24, so it is exactly representable in FP32.

The workloads stand in for the paper's benchmark programs (section 7.2,
Table 2), which are not available; shapes and distributions follow the
configurations the co-execution engine is measured on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Seeds of the measured configurations.
SEED_BLUR = 0xB1
SEED_NBODY = 0x4B0D1
SEED_BATCH = 0xBA7C4
SEED_SERVE = 0x5E2E


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _base(seed: int, stream: int) -> np.uint64:
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        b = mix64(np.array([s + np.uint64(stream) * GOLDEN], dtype=np.uint64))[0]
    return np.uint64(b)


def draws_u64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Draws ``start .. start+n-1`` of a stream as uint64."""
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(_base(seed, stream) + idx * GOLDEN)


def uniform_f32(seed: int, stream: int, n: int, lo: float = 0.0, hi: float = 1.0,
                start: int = 0) -> np.ndarray:
    """FP32 uniform draws on [lo, hi): top 24 bits of each draw scaled."""
    u = (draws_u64(seed, stream, n, start) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)
    return (lo + (hi - lo) * u).astype(np.float32)


def uniform_f64(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """FP64 uniform draws on [0, 1) from the top 53 bits of each draw."""
    return (draws_u64(seed, stream, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# --------------------------------------------------------------------------
# Escape-time fractal parameters
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class EscapeParams:
    """Pixel (r, c) maps to c = (x0 + c*dx) + i (y0 + r*dy); output is uint32."""
    w: int
    h: int
    x0: float
    y0: float
    dx: float
    dy: float
    max_iter: int

    def as_f32(self):
        return (np.float32(self.x0), np.float32(self.y0), np.float32(self.dx), np.float32(self.dy))


def escape_region(w: int, h: int, xa: float, xb: float, ya: float, yb: float,
                  max_iter: int) -> EscapeParams:
    """Region [xa, xb] x [ya, yb] on a w x h grid; steps computed in FP64 then
    rounded once to FP32, origin rounded once to FP32."""
    return EscapeParams(w, h, float(np.float32(xa)), float(np.float32(ya)),
                        float(np.float32((xb - xa) / w)), float(np.float32((yb - ya) / h)),
                        int(max_iter))


def escape_small() -> EscapeParams:
    """1024 x 1024 over [-2, 1] x [-1.5, 1.5], max_iter 256 (all coordinates exact in FP32)."""
    return escape_region(1024, 1024, -2.0, 1.0, -1.5, 1.5, 256)


# --------------------------------------------------------------------------
# 5x5 blur image
# --------------------------------------------------------------------------
def blur_image(w: int = 8192, h: int = 8192, seed: int = SEED_BLUR) -> np.ndarray:
    """FP32 image with pixels uniform in [0, 1), row-major (h, w)."""
    return uniform_f32(seed, 1, w * h).reshape(h, w)


# --------------------------------------------------------------------------
# N-body bodies
# --------------------------------------------------------------------------
def nbody_bodies(n: int = 65536, seed: int = SEED_NBODY) -> np.ndarray:
    """(n, 4) FP32 array of (x, y, z, m): positions uniform in the unit cube,
    masses uniform in [0.5, 1.5)."""
    out = np.empty((n, 4), dtype=np.float32)
    out[:, 0] = uniform_f32(seed, 1, n)
    out[:, 1] = uniform_f32(seed, 2, n)
    out[:, 2] = uniform_f32(seed, 3, n)
    out[:, 3] = uniform_f32(seed, 4, n, 0.5, 1.5)
    return out


def nbody_velocities(n: int = 65536, seed: int = SEED_NBODY) -> np.ndarray:
    """(n, 4) FP32 array of (vx, vy, vz, 0): components uniform in [-0.5, 0.5)."""
    out = np.zeros((n, 4), dtype=np.float32)
    out[:, 0] = uniform_f32(seed, 5, n, -0.5, 0.5)
    out[:, 1] = uniform_f32(seed, 6, n, -0.5, 0.5)
    out[:, 2] = uniform_f32(seed, 7, n, -0.5, 0.5)
    return out


# --------------------------------------------------------------------------
# Binomial option spots
# --------------------------------------------------------------------------
SEED_BINOMIAL = 0xB10A


def binomial_spots(n_groups: int, seed: int = SEED_BINOMIAL) -> np.ndarray:
    """(n_groups, 4) FP32 spot prices uniform in [50, 150): four options per group."""
    return uniform_f32(seed, 1, n_groups * 4, 50.0, 150.0).reshape(n_groups, 4)


# --------------------------------------------------------------------------
# Batched escape-time jobs
# --------------------------------------------------------------------------
def batch_jobs(n_jobs: int = 256, seed: int = SEED_BATCH, side_lo: int = 64, side_hi: int = 2048,
               iter_lo: int = 64, iter_hi: int = 4096) -> list[EscapeParams]:
    """Square escape-time jobs: side log-uniform in [side_lo, side_hi] (rounded),
    max_iter integer-uniform in [iter_lo, iter_hi], region centre jittered
    around (-0.5, 0) by U(-0.25, 0.25) per axis, half-width 1.5 * 2**U(-1, 0)."""
    u_side = uniform_f64(seed, 1, n_jobs)
    u_iter = draws_u64(seed, 2, n_jobs)
    u_cx = uniform_f64(seed, 3, n_jobs)
    u_cy = uniform_f64(seed, 4, n_jobs)
    u_hw = uniform_f64(seed, 5, n_jobs)
    jobs = []
    for i in range(n_jobs):
        side = int(round(math.exp(math.log(side_lo) + u_side[i] * (math.log(side_hi) - math.log(side_lo)))))
        side = max(side_lo, min(side_hi, side))
        mi = iter_lo + int(u_iter[i] % np.uint64(iter_hi - iter_lo + 1))
        cx = -0.5 + (u_cx[i] * 0.5 - 0.25)
        cy = u_cy[i] * 0.5 - 0.25
        hw = 1.5 * 2.0 ** (u_hw[i] - 1.0)
        jobs.append(escape_region(side, side, cx - hw, cx + hw, cy - hw, cy + hw, mi))
    return jobs


# --------------------------------------------------------------------------
# Serving trace
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class ServeJob:
    kind: str          # "escape" | "blur" | "nbody"
    arrival_s: float   # arrival time in seconds from the start of the trace
    size: int          # side (escape, blur) or body count (nbody)
    max_iter: int      # escape only
    seed: int          # seed of the job's own input (blur image, bodies)
    region: tuple      # escape only: (xa, xb, ya, yb)


def serve_trace(n_jobs: int = 2000, seed: int = SEED_SERVE, rate_hz: float = 200.0,
                escape_side=(256, 4096), blur_side=(1024, 16384), nbody_n=(4096, 131072),
                iter_lo: int = 64, iter_hi: int = 4096) -> list[ServeJob]:
    """Poisson arrivals (exponential gaps at ``rate_hz``) of a job mix drawn
    uniformly over the three payload kinds; sizes log-uniform in the ranges."""
    u_gap = uniform_f64(seed, 1, n_jobs)
    u_kind = draws_u64(seed, 2, n_jobs)
    u_size = uniform_f64(seed, 3, n_jobs)
    u_iter = draws_u64(seed, 4, n_jobs)
    u_cx = uniform_f64(seed, 5, n_jobs)
    u_cy = uniform_f64(seed, 6, n_jobs)
    u_hw = uniform_f64(seed, 7, n_jobs)
    t = 0.0
    jobs = []
    kinds = ("escape", "blur", "nbody")
    for i in range(n_jobs):
        t += -math.log(1.0 - u_gap[i]) / rate_hz
        kind = kinds[int(u_kind[i] % np.uint64(3))]
        lo, hi = {"escape": escape_side, "blur": blur_side, "nbody": nbody_n}[kind]
        size = int(round(math.exp(math.log(lo) + u_size[i] * (math.log(hi) - math.log(lo)))))
        size = max(lo, min(hi, size))
        mi = iter_lo + int(u_iter[i] % np.uint64(iter_hi - iter_lo + 1))
        cx = -0.5 + (u_cx[i] * 0.5 - 0.25)
        cy = u_cy[i] * 0.5 - 0.25
        hw = 1.5 * 2.0 ** (u_hw[i] - 1.0)
        jobs.append(ServeJob(kind, t, size, mi if kind == "escape" else 0,
                             (seed * 1000003 + i) & 0xFFFFFFFF, (cx - hw, cx + hw, cy - hw, cy + hw)))
    return jobs
