/*
 * Oracle for the co-execution hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, single-threaded definitions of what the engine computes,
 * written from the paper and from the textbook definitions of its benchmark
 * payloads. Only the test suite, the smoke check and the bench's CPU-baseline
 * leg may call into this library; the engine never links or loads it, and it
 * shares no source with the engine.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC.
 * FP32 arithmetic is written one operation at a time; fused multiply-adds occur
 * only where fmaf() is called (C99 fmaf is correctly rounded).
 */
#ifndef ORACLE_H
#define ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- payload 1: escape-time fractal (Mandelbrot benchmark, section 7.2 and
 * Table 2). Pixel (r, c) has c = (x0 + c*dx) + i(y0 + r*dy); the count is the
 * first n >= 1 with |z_n|^2 > 4 under z_{n+1} = z_n^2 + c, z_0 = 0, capped at
 * max_iter. */
uint32_t orc_escape_pixel(uint32_t r, uint32_t c, float x0, float y0, float dx, float dy,
                          uint32_t max_iter);
void orc_escape(uint32_t w, uint32_t h, float x0, float y0, float dx, float dy, uint32_t max_iter,
                uint32_t* out);

/* ---- payload 2: 5x5 Gaussian blur (Gaussian benchmark, section 7.2, Table 2:
 * image and weights in, image out). */
void orc_gauss5_weights(double sigma, float w[25]);
float orc_blur5_pixel(const float* in, uint32_t w, uint32_t h, const float wt[25], uint32_t y,
                      uint32_t x);
void orc_blur5(const float* in, uint32_t w, uint32_t h, const float wt[25], float* out);

/* ---- payload 3: all-pairs N-body acceleration (NBody benchmark, section 6.2
 * and Table 2), force part only. Bodies are float4 (x, y, z, m). */
float orc_rsqrt_lomont_estimate(float x);
float orc_rsqrt_newton(float hx, float y);
float orc_rsqrt_lomont(float x);
void orc_nbody_acc_body(const float* pos4, uint32_t n, float eps2, int strict, uint32_t i,
                        float out4[4]);
void orc_nbody_acc(const float* pos4, uint32_t n, float eps2, int strict, float* out4);
void orc_nbody_acc_f64(const float* pos4, uint32_t n, double eps2, uint32_t i0, uint32_t i1,
                       double* out3);
/* ---- N-body integration step (NBody program of section 6.2: pos and vel
 * in, pos and vel out, dt, eps2): v' = v + a dt, x' = x + v dt + a dt^2/2 with
 * a from orc_nbody_acc_body; mass and vel w copied. */
void orc_nbody_step_body(const float* pos4, const float* vel4, uint32_t n, float eps2, float dt, int strict,
                         uint32_t i, float pos_out[4], float vel_out[4]);
void orc_nbody_step(const float* pos4, const float* vel4, uint32_t n, float eps2, float dt, int strict,
                    float* pos_out4, float* vel_out4);

/* ---- Binomial option pricing (Binomial Options program, sections 6.1 and 7.2):
 * Cox-Ross-Rubinstein tree of `steps` steps for a European call; the tree's
 * constants rounded once from double; the backward induction in FP32. */
void orc_binomial_table(uint32_t steps, double sigma, double rate, double T, float* factors, float* pu,
                        float* pd);
float orc_binomial_price(float S, float X, uint32_t steps, const float* factors, float pu, float pd);

/* ---- schedulers (section 5.3) */
/* Static: n devices, props[0..n-2] fractions in device order, last gets the
 * rest; order[k] = device placed k-th along the index space. With n_bands > 0
 * the boundaries snap to a grid of n_bands equal bands and every device gets
 * at least one band. Writes begin[d], end[d] (granules). Returns 0 or -1. */
int orc_static_plan(uint64_t G, uint32_t n, const double* props, const uint32_t* order,
                    uint32_t n_bands, uint64_t* begin, uint64_t* end);
/* HGuided package size for device i (section 5.3 equation). */
uint64_t orc_hguided_size(uint64_t G_r, const uint64_t* P, uint32_t n, uint32_t k, uint32_t i,
                          uint64_t min_i);

#ifdef __cplusplus
}
#endif
#endif
