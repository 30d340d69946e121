// Host payload workers: scalar FMA versions and AVX-512 versions. Vector
// lanes are independent work-items, so every lane performs exactly the scalar
// operation sequence (one IEEE operation per step, fma only where written).
// Compiled with -ffp-contract=off; fast-math is never used.
#include "host_payloads.hpp"

#include <immintrin.h>
#include <string.h>

namespace ce {
namespace {

#define T_FMA __attribute__((target("avx2,fma")))
#define T_512 __attribute__((target("avx512f,avx512dq,avx512bw,avx512vl,avx2,fma")))

// ------------------------------------------------------------ escape-time
T_FMA inline uint32_t escape_scalar(float cr, float ci, uint32_t max_iter) {
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

T_FMA void escape_rows_fma(const ce_escape_params& p, uint64_t r0, uint64_t r1, uint32_t* out) {
  for (uint64_t r = r0; r < r1; ++r) {
    const float ci = p.y0 + (float)r * p.dy;
    uint32_t* row = out + r * p.w;
    for (uint32_t c = 0; c < p.w; ++c) {
      const float cr = p.x0 + (float)c * p.dx;
      row[c] = escape_scalar(cr, ci, p.max_iter);
    }
  }
}

T_512 void escape_rows_512(const ce_escape_params& p, uint64_t r0, uint64_t r1, uint32_t* out) {
  const __m512 four = _mm512_set1_ps(4.0f);
  const __m512 vx0 = _mm512_set1_ps(p.x0), vdx = _mm512_set1_ps(p.dx);
  const __m512i lane = _mm512_setr_epi32(0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15);
  const __m512i one = _mm512_set1_epi32(1);
  for (uint64_t r = r0; r < r1; ++r) {
    const __m512 ci = _mm512_set1_ps(p.y0 + (float)r * p.dy);
    uint32_t* row = out + r * p.w;
    for (uint32_t c0 = 0; c0 < p.w; c0 += 16) {
      const __m512i cidx = _mm512_add_epi32(_mm512_set1_epi32((int)c0), lane);
      const uint32_t left = p.w - c0;
      __mmask16 active = left >= 16 ? (__mmask16)0xFFFF : (__mmask16)((1u << left) - 1u);
      const __mmask16 valid = active;
      const __m512 cr = _mm512_add_ps(vx0, _mm512_mul_ps(_mm512_cvtepu32_ps(cidx), vdx));
      __m512 zr = _mm512_setzero_ps(), zi = _mm512_setzero_ps();
      __m512i n = _mm512_setzero_si512();
      for (uint32_t it = 0; it < p.max_iter && active; ++it) {
        const __m512 x2 = _mm512_mul_ps(zr, zr);
        const __m512 y2 = _mm512_mul_ps(zi, zi);
        const __mmask16 esc = _mm512_cmp_ps_mask(_mm512_add_ps(x2, y2), four, _CMP_GT_OQ);
        active = (__mmask16)(active & ~esc);
        const __m512 t = _mm512_add_ps(zr, zr);
        const __m512 zin = _mm512_fmadd_ps(t, zi, ci);
        const __m512 zrn = _mm512_add_ps(_mm512_sub_ps(x2, y2), cr);
        zr = _mm512_mask_mov_ps(zr, active, zrn);
        zi = _mm512_mask_mov_ps(zi, active, zin);
        n = _mm512_mask_add_epi32(n, active, n, one);
      }
      _mm512_mask_storeu_epi32(row + c0, valid, n);
    }
  }
}

// ------------------------------------------------------------------ blur
inline uint32_t clampu(int64_t v, uint32_t n) { return (uint32_t)(v < 0 ? 0 : (v >= (int64_t)n ? n - 1 : v)); }

T_FMA inline float blur_px(const float* in, uint32_t w, uint32_t h, const float* wt, uint64_t y, uint32_t x) {
  float acc = 0.0f;
  for (int dy = 0; dy < 5; ++dy) {
    const float* row = in + (size_t)clampu((int64_t)y + dy - 2, h) * w;
    for (int dx = 0; dx < 5; ++dx) acc = __builtin_fmaf(wt[dy * 5 + dx], row[clampu((int64_t)x + dx - 2, w)], acc);
  }
  return acc;
}

T_FMA void blur5_rows_fma(const float* in, uint32_t w, uint32_t h, const float* wt, uint64_t r0, uint64_t r1,
                          float* out) {
  for (uint64_t y = r0; y < r1; ++y)
    for (uint32_t x = 0; x < w; ++x) out[y * w + x] = blur_px(in, w, h, wt, y, x);
}

T_512 void blur5_rows_512(const float* in, uint32_t w, uint32_t h, const float* wt, uint64_t r0, uint64_t r1,
                          float* out) {
  __m512 vw[25];
  for (int k = 0; k < 25; ++k) vw[k] = _mm512_set1_ps(wt[k]);
  for (uint64_t y = r0; y < r1; ++y) {
    const float* rows[5];
    for (int dy = 0; dy < 5; ++dy) rows[dy] = in + (size_t)clampu((int64_t)y + dy - 2, h) * w;
    float* orow = out + y * w;
    // interior columns [2, w-2) need no clamping in x
    uint32_t x = 2;
    if (w >= 4) {
      for (; x + 16 <= w - 2; x += 16) {
        __m512 acc = _mm512_setzero_ps();
        for (int dy = 0; dy < 5; ++dy)
          for (int dx = 0; dx < 5; ++dx)
            acc = _mm512_fmadd_ps(vw[dy * 5 + dx], _mm512_loadu_ps(rows[dy] + x + dx - 2), acc);
        _mm512_storeu_ps(orow + x, acc);
      }
    }
    for (uint32_t c = 0; c < w; ++c) {
      if (c >= 2 && c < x) continue;
      orow[c] = blur_px(in, w, h, wt, y, c);
    }
  }
}

// ---------------------------------------------------------------- n-body
// Lomont, "Fast Inverse Square Root" (2003): integer estimate, then three
// Newton-Raphson steps t = y*y; u = fma(-(x/2), t, 1.5); y = y*u.
T_FMA inline float rsqrt_lomont(float x) {
  uint32_t b;
  memcpy(&b, &x, 4);
  b = 0x5f375a86u - (b >> 1);
  float y;
  memcpy(&y, &b, 4);
  const float hx = 0.5f * x;
  for (int s = 0; s < 3; ++s) {
    const float t = y * y;
    const float u = __builtin_fmaf(-hx, t, 1.5f);
    y = y * u;
  }
  return y;
}

T_512 inline __m512 rsqrt_lomont_512(__m512 x) {
  const __m512i b = _mm512_sub_epi32(_mm512_set1_epi32(0x5f375a86), _mm512_srli_epi32(_mm512_castps_si512(x), 1));
  __m512 y = _mm512_castsi512_ps(b);
  const __m512 hx = _mm512_mul_ps(_mm512_set1_ps(0.5f), x);
  const __m512 c15 = _mm512_set1_ps(1.5f);
  for (int s = 0; s < 3; ++s) {
    const __m512 t = _mm512_mul_ps(y, y);
    const __m512 u = _mm512_fnmadd_ps(hx, t, c15);  // -(hx*t) + 1.5, one rounding
    y = _mm512_mul_ps(y, u);
  }
  return y;
}

T_FMA void nbody_body(const float* pos4, uint32_t n, float eps2, int strict, uint64_t i, float* o) {
  const float xi = pos4[4 * i], yi = pos4[4 * i + 1], zi = pos4[4 * i + 2];
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
  for (uint32_t j = 0; j < n; ++j) {
    const float* pj = pos4 + 4 * (size_t)j;
    const float dx = pj[0] - xi, dy = pj[1] - yi, dz = pj[2] - zi;
    const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
    const float rinv = strict ? rsqrt_lomont(r2) : 1.0f / __builtin_sqrtf(r2);
    const float s = (rinv * rinv) * rinv;
    const float f = pj[3] * s;
    ax = __builtin_fmaf(f, dx, ax);
    ay = __builtin_fmaf(f, dy, ay);
    az = __builtin_fmaf(f, dz, az);
  }
  o[0] = ax;
  o[1] = ay;
  o[2] = az;
  o[3] = 0.0f;
}

T_FMA void nbody_bodies_fma(const float* pos4, uint32_t n, float eps2, int strict, uint64_t i0, uint64_t i1,
                            float* out4) {
  for (uint64_t i = i0; i < i1; ++i) nbody_body(pos4, n, eps2, strict, i, out4 + 4 * i);
}

template <bool STRICT>
T_512 void nbody_block16(const float* pos4, uint32_t n, float eps2, uint64_t i0, float* out4) {
  alignas(64) float xs[16], ys[16], zs[16];
  for (int l = 0; l < 16; ++l) {
    xs[l] = pos4[4 * (i0 + l)];
    ys[l] = pos4[4 * (i0 + l) + 1];
    zs[l] = pos4[4 * (i0 + l) + 2];
  }
  const __m512 xi = _mm512_load_ps(xs), yi = _mm512_load_ps(ys), zi = _mm512_load_ps(zs);
  const __m512 e2 = _mm512_set1_ps(eps2);
  const __m512 one = _mm512_set1_ps(1.0f);
  __m512 ax = _mm512_setzero_ps(), ay = _mm512_setzero_ps(), az = _mm512_setzero_ps();
  for (uint32_t j = 0; j < n; ++j) {
    const float* pj = pos4 + 4 * (size_t)j;
    const __m512 dx = _mm512_sub_ps(_mm512_set1_ps(pj[0]), xi);
    const __m512 dy = _mm512_sub_ps(_mm512_set1_ps(pj[1]), yi);
    const __m512 dz = _mm512_sub_ps(_mm512_set1_ps(pj[2]), zi);
    const __m512 r2 = _mm512_fmadd_ps(dz, dz, _mm512_fmadd_ps(dy, dy, _mm512_fmadd_ps(dx, dx, e2)));
    const __m512 rinv = STRICT ? rsqrt_lomont_512(r2) : _mm512_div_ps(one, _mm512_sqrt_ps(r2));
    const __m512 s = _mm512_mul_ps(_mm512_mul_ps(rinv, rinv), rinv);
    const __m512 f = _mm512_mul_ps(_mm512_set1_ps(pj[3]), s);
    ax = _mm512_fmadd_ps(f, dx, ax);
    ay = _mm512_fmadd_ps(f, dy, ay);
    az = _mm512_fmadd_ps(f, dz, az);
  }
  alignas(64) float oa[16], ob[16], oc[16];
  _mm512_store_ps(oa, ax);
  _mm512_store_ps(ob, ay);
  _mm512_store_ps(oc, az);
  for (int l = 0; l < 16; ++l) {
    float* o = out4 + 4 * (i0 + l);
    o[0] = oa[l];
    o[1] = ob[l];
    o[2] = oc[l];
    o[3] = 0.0f;
  }
}

T_512 void nbody_bodies_512(const float* pos4, uint32_t n, float eps2, int strict, uint64_t i0, uint64_t i1,
                            float* out4) {
  uint64_t i = i0;
  for (; i + 16 <= i1; i += 16) {
    if (strict)
      nbody_block16<true>(pos4, n, eps2, i, out4);
    else
      nbody_block16<false>(pos4, n, eps2, i, out4);
  }
  for (; i < i1; ++i) nbody_body(pos4, n, eps2, strict, i, out4 + 4 * i);
}

const HostPayloadFns kFma = {escape_rows_fma, blur5_rows_fma, nbody_bodies_fma, "avx2+fma"};
const HostPayloadFns k512 = {escape_rows_512, blur5_rows_512, nbody_bodies_512, "avx512"};

}  // namespace

void nbody_step_update(const float* pos4, const float* vel4, float dt, uint64_t i0, uint64_t i1, float* pos_out4,
                       float* vel_out4) {
  const float h = (dt * dt) * 0.5f;
  for (uint64_t i = i0; i < i1; ++i) {
    const float* x = pos4 + 4 * i;
    const float* v = vel4 + 4 * i;
    float* xo = pos_out4 + 4 * i;
    float* vo = vel_out4 + 4 * i;
    const float a[3] = {vo[0], vo[1], vo[2]};
    for (int c = 0; c < 3; ++c) {
      xo[c] = (x[c] + v[c] * dt) + a[c] * h;
      vo[c] = v[c] + a[c] * dt;
    }
    xo[3] = x[3];
    vo[3] = v[3];
  }
}

void binomial_groups(const float* spots4, const float* factors, uint32_t steps, float strike, float pu, float pd,
                     uint64_t g0, uint64_t g1, float* out4) {
  float v[256];
  for (uint64_t g = g0; g < g1; ++g) {
    for (int c = 0; c < 4; ++c) {
      const float S = spots4[4 * g + c];
      for (uint32_t j = 0; j <= steps; ++j) {
        const float t = S * factors[j] - strike;
        v[j] = t > 0.0f ? t : 0.0f;
      }
      for (uint32_t L = steps; L-- > 0;)
        for (uint32_t j = 0; j <= L; ++j) {
          const float up = pu * v[j + 1];
          const float dn = pd * v[j];
          v[j] = up + dn;
        }
      out4[4 * g + c] = v[0];
    }
  }
}

const HostPayloadFns* host_payloads() {
  __builtin_cpu_init();
  if (__builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512dq") &&
      __builtin_cpu_supports("avx512bw") && __builtin_cpu_supports("avx512vl"))
    return &k512;
  if (__builtin_cpu_supports("fma") && __builtin_cpu_supports("avx2")) return &kFma;
  return nullptr;
}

}  // namespace ce
