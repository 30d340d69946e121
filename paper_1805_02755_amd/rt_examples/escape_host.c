/* Host version of escape.hiprtc for the engine's host workers (a
 * separate implementation of the same work-item function; built by the
 * tests with -ffp-contract=off). */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef struct {
  void* buf[4];
  unsigned char scalars[128];
} rt_args;

int32_t escape_host(uint64_t i0, uint64_t i1, const rt_args* a) {
  float f[4];
  uint32_t u[2];
  memcpy(f, a->scalars, sizeof f);
  memcpy(u, a->scalars + 16, sizeof u);
  uint32_t* out = (uint32_t*)a->buf[0];
  for (uint64_t i = i0; i < i1; ++i) {
    const uint32_t r = (uint32_t)(i / u[0]), c = (uint32_t)(i % u[0]);
    const float cr = f[0] + (float)c * f[2];
    const float ci = f[1] + (float)r * f[3];
    float zr = 0.0f, zi = 0.0f;
    uint32_t n = 0;
    while (n < u[1]) {
      const float x2 = zr * zr, y2 = zi * zi;
      if (x2 + y2 > 4.0f) break;
      const float t = zr + zr;
      zi = fmaf(t, zi, ci);
      zr = (x2 - y2) + cr;
      ++n;
    }
    out[i] = n;
  }
  return 0;
}

/* Two inputs, two outputs: z0 = alpha * x + y and z1 = x - y (float32). */
int32_t axpy2_host(uint64_t i0, uint64_t i1, const rt_args* a) {
  float alpha;
  memcpy(&alpha, a->scalars, sizeof alpha);
  const float* x = (const float*)a->buf[0];
  const float* y = (const float*)a->buf[1];
  float* z0 = (float*)a->buf[2];
  float* z1 = (float*)a->buf[3];
  for (uint64_t i = i0; i < i1; ++i) {
    const float p = alpha * x[i];
    z0[i] = p + y[i];
    z1[i] = x[i] - y[i];
  }
  return 0;
}
