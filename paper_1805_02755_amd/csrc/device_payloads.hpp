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
