// Per-work-item payload arithmetic on the GPU, shared by the persistent,
// plain and batched kernels. Each function fixes one FP32 operation sequence
// (compiled with -ffp-contract=off) that the host workers repeat exactly.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ce {

// Escape-time count (Mandelbrot program, section 7.2): z <- z^2 + c from 0,
// first n >= 1 with |z_n|^2 > 4, capped at max_iter.
__device__ __forceinline__ uint32_t escape_count(float cr, float ci, uint32_t max_iter) {
  float zr = 0.0f, zi = 0.0f;
  uint32_t n = 0;
  // Four iterations per loop test: each iteration's escape test is computed
  // from its own z exactly as below, and the first that fires gives the
  // count, so the result is that of the one-step loop. Before the escape
  // |z| <= 2, so nothing overflows; after it at most three more steps are
  // taken from |z| > 2, whose tests are not looked at.
  while (n + 4 <= max_iter) {
    const float a2 = zr * zr, b2 = zi * zi;
    const float s0 = a2 + b2;
    const float zi1 = __builtin_fmaf(zr + zr, zi, ci);
    const float zr1 = (a2 - b2) + cr;
    const float c2 = zr1 * zr1, d2 = zi1 * zi1;
    const float s1 = c2 + d2;
    const float zi2 = __builtin_fmaf(zr1 + zr1, zi1, ci);
    const float zr2 = (c2 - d2) + cr;
    const float e2 = zr2 * zr2, f2 = zi2 * zi2;
    const float s2 = e2 + f2;
    const float zi3 = __builtin_fmaf(zr2 + zr2, zi2, ci);
    const float zr3 = (e2 - f2) + cr;
    const float g2 = zr3 * zr3, h2 = zi3 * zi3;
    const float s3 = g2 + h2;
    if ((s0 > 4.0f) | (s1 > 4.0f) | (s2 > 4.0f) | (s3 > 4.0f))
      return n + (s0 > 4.0f ? 0u : (s1 > 4.0f ? 1u : (s2 > 4.0f ? 2u : 3u)));
    zi = __builtin_fmaf(zr3 + zr3, zi3, ci);
    zr = (g2 - h2) + cr;
    n += 4;
  }
  while (n < max_iter) {
    const float x2 = zr * zr;
    const float y2 = zi * zi;
    if (x2 + y2 > 4.0f) break;
    const float t = zr + zr;
    zi = __builtin_fmaf(t, zi, ci);
    zr = (x2 - y2) + cr;
    ++n;
  }
  return n;
}

}  // namespace ce
