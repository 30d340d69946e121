/*
 * Oracle for the co-execution hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain sequential definitions of the three benchmark payloads and of the
 * package schedulers of section 5.3. Nothing here is blocked, fused or
 * reordered; each function follows the definition it cites. The engine does
 * not link, load or include this file. Only tests, the smoke check and the
 * bench's CPU-baseline leg call it.
 *
 * Compiled with -O2 -ffp-contract=off and without fast-math, so every FP32
 * expression below is one correctly rounded IEEE operation per operator and
 * a fused multiply-add happens only where fmaf() is written.
 */
#include "oracle.h"

#include <math.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Escape-time fractal. The paper runs the Mandelbrot program of its suite
 * (section 7.2; Table 2: no inputs, one output buffer, irregular cost per
 * item). Its arithmetic is the textbook escape-time iteration z <- z^2 + c
 * from z = 0, stopped at the first |z|^2 > 4 or after max_iter steps. The FP32
 * evaluation order is fixed as: x2 = zr*zr, y2 = zi*zi, test x2 + y2 > 4,
 * zi <- fma(zr + zr, zi, ci), zr <- (x2 - y2) + cr. */
uint32_t orc_escape_pixel(uint32_t r, uint32_t c, float x0, float y0, float dx, float dy,
                          uint32_t max_iter) {
  const float cr = x0 + (float)c * dx;
  const float ci = y0 + (float)r * dy;
  float zr = 0.0f, zi = 0.0f;
  uint32_t n = 0;
  while (n < max_iter) {
    const float x2 = zr * zr;
    const float y2 = zi * zi;
    if (x2 + y2 > 4.0f) break;
    const float t = zr + zr;
    zi = fmaf(t, zi, ci);
    zr = (x2 - y2) + cr;
    n = n + 1;
  }
  return n;
}

void orc_escape(uint32_t w, uint32_t h, float x0, float y0, float dx, float dy, uint32_t max_iter,
                uint32_t* out) {
  for (uint32_t r = 0; r < h; ++r)
    for (uint32_t c = 0; c < w; ++c)
      out[(size_t)r * w + c] = orc_escape_pixel(r, c, x0, y0, dx, dy, max_iter);
}

/* ------------------------------------------------------------------------ */
/* 5x5 Gaussian blur. The paper's Gaussian program (section 7.2; Table 2: an
 * image and a weight buffer in, one image out, one output per work-item).
 * Weights: w(dx,dy) = exp(-(dx^2+dy^2) / (2 sigma^2)) / sum over the 5x5
 * window, evaluated in double and rounded once to float. */
void orc_gauss5_weights(double sigma, float w[25]) {
  double e[25];
  double sum = 0.0;
  for (int dy = -2; dy <= 2; ++dy)
    for (int dx = -2; dx <= 2; ++dx) {
      const double v = exp(-(double)(dx * dx + dy * dy) / (2.0 * sigma * sigma));
      e[(dy + 2) * 5 + (dx + 2)] = v;
      sum += v;
    }
  for (int k = 0; k < 25; ++k) w[k] = (float)(e[k] / sum);
}

static uint32_t clampi(int64_t v, int64_t lo, int64_t hi) {
  return (uint32_t)(v < lo ? lo : (v > hi ? hi : v));
}

/* out(y,x) = sum_{dy=-2..2} sum_{dx=-2..2} w(dy,dx) * in(clamp(y+dy), clamp(x+dx)),
 * clamp-to-edge, accumulated in FP32 by fmaf with dy outer and dx inner, both
 * ascending, starting from +0. */
float orc_blur5_pixel(const float* in, uint32_t w, uint32_t h, const float wt[25], uint32_t y,
                      uint32_t x) {
  float acc = 0.0f;
  for (int dy = -2; dy <= 2; ++dy) {
    const uint32_t yy = clampi((int64_t)y + dy, 0, (int64_t)h - 1);
    for (int dx = -2; dx <= 2; ++dx) {
      const uint32_t xx = clampi((int64_t)x + dx, 0, (int64_t)w - 1);
      acc = fmaf(wt[(dy + 2) * 5 + (dx + 2)], in[(size_t)yy * w + xx], acc);
    }
  }
  return acc;
}

void orc_blur5(const float* in, uint32_t w, uint32_t h, const float wt[25], float* out) {
  for (uint32_t y = 0; y < h; ++y)
    for (uint32_t x = 0; x < w; ++x) out[(size_t)y * w + x] = orc_blur5_pixel(in, w, h, wt, y, x);
}

/* ------------------------------------------------------------------------ */
/* N-body acceleration. The paper's NBody program (section 6.2 listing, Table 2)
 * integrates positions and velocities under softened all-pairs gravity; the
 * hot path here is its force part:
 *   a_i = sum_j m_j (p_j - p_i) / (|p_j - p_i|^2 + eps2)^(3/2),
 * with j = i included (it contributes exactly zero).
 *
 * Strict mode evaluates 1/sqrt by the published approximation of Lomont,
 * "Fast Inverse Square Root" (2003): the integer estimate 0x5f375a86 - (bits
 * >> 1) followed by three Newton-Raphson steps y <- y * (1.5 - (x/2) y^2), each
 * written as t = y*y; u = fma(-(x/2), t, 1.5); y = y*u. Fast mode uses the
 * correctly rounded 1/sqrtf. */
/* Lomont's integer first estimate of 1/sqrt(x), before any Newton step. */
float orc_rsqrt_lomont_estimate(float x) {
  uint32_t bits;
  memcpy(&bits, &x, sizeof bits);
  bits = 0x5f375a86u - (bits >> 1);
  float y;
  memcpy(&y, &bits, sizeof y);
  return y;
}

/* One Newton-Raphson step for 1/sqrt(x) from the estimate y, with hx = x/2. */
float orc_rsqrt_newton(float hx, float y) {
  const float t = y * y;
  const float u = fmaf(-hx, t, 1.5f);
  return y * u;
}

float orc_rsqrt_lomont(float x) {
  float y = orc_rsqrt_lomont_estimate(x);
  const float hx = 0.5f * x;
  for (int step = 0; step < 3; ++step) y = orc_rsqrt_newton(hx, y);
  return y;
}

void orc_nbody_acc_body(const float* pos4, uint32_t n, float eps2, int strict, uint32_t i,
                        float out4[4]) {
  const float xi = pos4[4 * (size_t)i + 0];
  const float yi = pos4[4 * (size_t)i + 1];
  const float zi = pos4[4 * (size_t)i + 2];
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
  for (uint32_t j = 0; j < n; ++j) {
    const float dx = pos4[4 * (size_t)j + 0] - xi;
    const float dy = pos4[4 * (size_t)j + 1] - yi;
    const float dz = pos4[4 * (size_t)j + 2] - zi;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
    const float rinv = strict ? orc_rsqrt_lomont(r2) : 1.0f / sqrtf(r2);
    const float s = (rinv * rinv) * rinv;
    const float f = pos4[4 * (size_t)j + 3] * s;
    ax = fmaf(f, dx, ax);
    ay = fmaf(f, dy, ay);
    az = fmaf(f, dz, az);
  }
  out4[0] = ax;
  out4[1] = ay;
  out4[2] = az;
  out4[3] = 0.0f;
}

void orc_nbody_acc(const float* pos4, uint32_t n, float eps2, int strict, float* out4) {
  for (uint32_t i = 0; i < n; ++i) orc_nbody_acc_body(pos4, n, eps2, strict, i, out4 + 4 * (size_t)i);
}

/* N-body integration step (the NBody program of section 6.2: positions and
 * velocities in, positions and velocities out, a time step and a squared
 * softening). The paper shows the program's buffers and arguments, not its
 * update; the update here is the constant-acceleration step of elementary
 * kinematics over dt, with a_i the acceleration of orc_nbody_acc_body:
 *   v' = v + a dt,   x' = x + v dt + a dt^2 / 2,
 * evaluated per component in FP32 as h = (dt * dt) * 0.5, x' = (x + v*dt) + a*h,
 * v' = v + a*dt. The mass (w of the position) and w of the velocity are copied. */
void orc_nbody_step_body(const float* pos4, const float* vel4, uint32_t n, float eps2, float dt, int strict,
                         uint32_t i, float pos_out[4], float vel_out[4]) {
  float a[4];
  orc_nbody_acc_body(pos4, n, eps2, strict, i, a);
  const float h = (dt * dt) * 0.5f;
  for (int c = 0; c < 3; ++c) {
    const float x = pos4[4 * (size_t)i + c];
    const float v = vel4[4 * (size_t)i + c];
    const float vdt = v * dt;
    const float ah = a[c] * h;
    pos_out[c] = (x + vdt) + ah;
    const float adt = a[c] * dt;
    vel_out[c] = v + adt;
  }
  pos_out[3] = pos4[4 * (size_t)i + 3];
  vel_out[3] = vel4[4 * (size_t)i + 3];
}

void orc_nbody_step(const float* pos4, const float* vel4, uint32_t n, float eps2, float dt, int strict,
                    float* pos_out4, float* vel_out4) {
  for (uint32_t i = 0; i < n; ++i)
    orc_nbody_step_body(pos4, vel4, n, eps2, dt, strict, i, pos_out4 + 4 * (size_t)i, vel_out4 + 4 * (size_t)i);
}

/* The same sum in double for bodies [i0, i1): error reference for FP32. */
void orc_nbody_acc_f64(const float* pos4, uint32_t n, double eps2, uint32_t i0, uint32_t i1,
                       double* out3) {
  for (uint32_t i = i0; i < i1; ++i) {
    double a[3] = {0.0, 0.0, 0.0};
    for (uint32_t j = 0; j < n; ++j) {
      double d[3];
      for (int c = 0; c < 3; ++c) d[c] = (double)pos4[4 * (size_t)j + c] - (double)pos4[4 * (size_t)i + c];
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
      const double s = (double)pos4[4 * (size_t)j + 3] / (r2 * sqrt(r2));
      for (int c = 0; c < 3; ++c) a[c] += s * d[c];
    }
    for (int c = 0; c < 3; ++c) out3[3 * (size_t)(i - i0) + c] = a[c];
  }
}

/* ------------------------------------------------------------------------ */
/* Binomial option pricing (the Binomial Options program of sections 6.1 and
 * 7.2: one output per work-group of steps+1 work-items, an out pattern of
 * 1:255 for 254 steps). The paper gives the program's shape, not its
 * arithmetic; this is the textbook Cox-Ross-Rubinstein tree for a European
 * call. Per step dt = T/N, up factor u = exp(sigma sqrt(dt)), down d = 1/u,
 * risk-neutral p = (exp(r dt) - d)/(u - d), discount exp(-r dt). The tree's
 * constants are computed in double and rounded once to FP32: pu = disc*p,
 * pd = disc*(1-p), and the leaf factors f_j = u^(2j-N) for j = 0..N. */
void orc_binomial_table(uint32_t steps, double sigma, double rate, double T, float* factors, float* pu,
                        float* pd) {
  const double dt = T / (double)steps;
  const double lu = sigma * sqrt(dt);
  const double u = exp(lu);
  const double d = 1.0 / u;
  const double p = (exp(rate * dt) - d) / (u - d);
  const double disc = exp(-rate * dt);
  *pu = (float)(disc * p);
  *pd = (float)(disc * (1.0 - p));
  for (uint32_t j = 0; j <= steps; ++j) factors[j] = (float)exp(lu * ((double)(2 * (int64_t)j) - (double)steps));
}

/* Price of one call with spot S and strike X, in FP32: leaves
 * V_j = max(S*f_j - X, 0), then for each level L = N-1 .. 0 and j = 0..L,
 * V_j = pu*V_{j+1} + pd*V_j (two products, then their sum); the price is V_0. */
float orc_binomial_price(float S, float X, uint32_t steps, const float* factors, float pu, float pd) {
  float v[1024];
  if (steps >= 1024) return -1.0f;
  for (uint32_t j = 0; j <= steps; ++j) {
    const float t = S * factors[j] - X;
    v[j] = t > 0.0f ? t : 0.0f;
  }
  for (uint32_t L = steps; L-- > 0;)
    for (uint32_t j = 0; j <= L; ++j) {
      const float up = pu * v[j + 1];
      const float dn = pd * v[j];
      v[j] = up + dn;
    }
  return v[0];
}

/* ------------------------------------------------------------------------ */
/* Static scheduler (section 5.3): before the run the index space is cut into
 * one contiguous part per device, sized by the given proportions. The API
 * listing of section 6.2 passes n-1 proportions for n devices; the last device
 * takes the remainder. The delivery order decides which device's part comes
 * first along the index space (section 7.3: "Static" vs "Static rev").
 * Boundaries are floors of the cumulative proportion times G. With n_bands > 0
 * the space is first cut into n_bands equal bands (band b ends at
 * floor((b+1) G / n_bands)) and device d receives max(1, round(p_d * n_bands))
 * bands, capped so that every later device keeps at least one band; the last
 * device receives the remaining bands. */
int orc_static_plan(uint64_t G, uint32_t n, const double* props, const uint32_t* order,
                    uint32_t n_bands, uint64_t* begin, uint64_t* end) {
  if (n == 0 || n > 64) return -1;
  double share[64];
  double rest = 1.0;
  for (uint32_t d = 0; d + 1 < n; ++d) {
    if (!(props[d] >= 0.0) || props[d] > 1.0) return -1;
    share[d] = props[d];
    rest -= props[d];
  }
  if (rest < -1e-12) return -1;
  share[n - 1] = rest < 0.0 ? 0.0 : rest;
  uint32_t seen[64] = {0};
  for (uint32_t k = 0; k < n; ++k) {
    if (order[k] >= n || seen[order[k]]) return -1;
    seen[order[k]] = 1;
  }
  if (n_bands == 0) {
    double cum = 0.0;
    uint64_t prev = 0;
    for (uint32_t k = 0; k < n; ++k) {
      const uint32_t d = order[k];
      cum += share[d];
      uint64_t b = (k + 1 == n) ? G : (uint64_t)floor(cum * (double)G);
      if (b > G) b = G;
      if (b < prev) b = prev;
      begin[d] = prev;
      end[d] = b;
      prev = b;
    }
    return 0;
  }
  if (n_bands < n || (uint64_t)n_bands > G) return -1;
  uint64_t nb[64];
  uint64_t used = 0;
  for (uint32_t d = 0; d + 1 < n; ++d) {
    const double r = floor(share[d] * (double)n_bands + 0.5);
    uint64_t want = r < 1.0 ? 1 : (uint64_t)r;
    const uint64_t cap = n_bands - used - (n - 1 - d); /* leave one band per later device */
    nb[d] = want > cap ? cap : want;
    used += nb[d];
  }
  nb[n - 1] = n_bands - used;
  uint64_t band = 0;
  for (uint32_t k = 0; k < n; ++k) {
    const uint32_t d = order[k];
    begin[d] = band * G / n_bands;
    band += nb[d];
    end[d] = band * G / n_bands;
  }
  return 0;
}

/* HGuided (section 5.3): packet_size_i = floor(G_r P_i / (k n sum_j P_j)),
 * bounded below by the device's minimum package size and above by the
 * pending granules G_r. */
uint64_t orc_hguided_size(uint64_t G_r, const uint64_t* P, uint32_t n, uint32_t k, uint32_t i,
                          uint64_t min_i) {
  unsigned __int128 sumP = 0;
  for (uint32_t j = 0; j < n; ++j) sumP += P[j];
  const unsigned __int128 num = (unsigned __int128)G_r * P[i];
  const unsigned __int128 den = (unsigned __int128)k * n * sumP;
  uint64_t s = den ? (uint64_t)(num / den) : G_r;
  if (s < min_i) s = min_i;
  if (s > G_r) s = G_r;
  return s;
}
