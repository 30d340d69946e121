// Tile payloads for gfx950: how a workgroup of 256 threads computes one tile
// of each payload. Shared by the persistent, plain and serving kernels so
// every form runs the same per-item FP32 operation sequence.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/coexec.h"
#include "common.hpp"
#include "device_payloads.hpp"

namespace ce {

struct EscapeTile {
  // workgroups per CU the persistent kernel is compiled for: eight, the
  // residency of the plain launch, so that the 2048 tiles of a 1024 x 1024
  // grid run in one round
  static constexpr int kMinBlocksPerCu = 8;
  ce_escape_params p;
  uint32_t* out;
  __device__ void load_constants() {}
  __host__ __device__ uint32_t ncb() const { return (uint32_t)ceil_div(p.w, kEscapeTileCols); }
  __host__ __device__ uint64_t granules() const { return p.h; }
  __host__ __device__ uint32_t ntiles(uint64_t g0, uint64_t g1) const {
    return (uint32_t)(ceil_div(g1 - g0, kEscapeTileRows) * ncb());
  }
  // A tile is kEscapeTileRows x kEscapeTileCols pixels walked as strips of 64
  // consecutive pixels of one row: thread j takes pixels j, j + 256, ... of
  // the tile in row-major order.
  __device__ void run(uint64_t g0, uint64_t g1, uint32_t t) const {
    const uint32_t nc = ncb();
    const uint64_t rb = g0 + (uint64_t)(t / nc) * kEscapeTileRows;
    const uint32_t cb = (t % nc) * kEscapeTileCols;
#pragma unroll 1
    for (uint32_t q = threadIdx.x; q < kEscapeTileRows * kEscapeTileCols; q += kBlockThreads) {
      const uint64_t r = rb + q / kEscapeTileCols;
      const uint32_t c = cb + q % kEscapeTileCols;
      if (r < g1 && c < p.w) {
        const float cr = p.x0 + (float)c * p.dx;
        const float ci = p.y0 + (float)r * p.dy;
        out[r * p.w + c] = escape_count(cr, ci, p.max_iter);
      }
    }
  }
};

// 5x5 blur (Gaussian program, section 7.2): out(y,x) = sum over dy, dx of
// w(dy,dx) in(clamp(y+dy), clamp(x+dx)), accumulated by fma with dy outer,
// dx inner, ascending. Each thread owns 4 adjacent columns and walks down the
// tile's rows with a 5-row window of 8 columns (x-2 .. x+5) in registers.
// DPP controls (GFX9 data-parallel primitives): whole-wave shift by one lane.
constexpr int kDppWaveShl1 = 0x130;  // lane i reads lane i+1
constexpr int kDppWaveShr1 = 0x138;  // lane i reads lane i-1
__device__ __forceinline__ float dpp_from_left(float edge, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), kDppWaveShr1, 0xF, 0xF,
                                                    false));
}
__device__ __forceinline__ float dpp_from_right(float edge, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), kDppWaveShl1, 0xF, 0xF,
                                                    false));
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// kFresh: the input may have been written after the launch began (the
// serving kernel reuses memory while it runs), so wave-uniform reads, which
// the compiler would serve from the scalar cache, use coherent vector loads.
template <bool kFresh>
struct Blur5TileT {
  // five resident workgroups per CU keep enough loads in flight for HBM
  static constexpr int kMinBlocksPerCu = 5;
  ce_blur5_params p;
  const float* in;
  const float* wt;
  float* out;
  float w[25];
  __device__ __forceinline__ float uniform_load(const float* a) const {
    if constexpr (kFresh) {
      const uint32_t v = __hip_atomic_load(const_cast<uint32_t*>(reinterpret_cast<const uint32_t*>(a)),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return __uint_as_float(__builtin_amdgcn_readfirstlane(v));
    } else {
      return *a;
    }
  }
  // Weights are read once per workgroup in uniform control flow, so they
  // live in scalar registers and feed the FMAs as scalar operands.
  __device__ void load_constants() {
#pragma unroll
    for (int k = 0; k < 25; ++k) w[k] = uniform_load(wt + k);
  }
  __host__ __device__ uint32_t ncb() const { return (uint32_t)ceil_div(p.w, kBlurTileCols); }
  __host__ __device__ uint64_t granules() const { return p.h; }
  __host__ __device__ uint32_t ntiles(uint64_t g0, uint64_t g1) const {
    return (uint32_t)(ceil_div(g1 - g0, kBlurTileRows) * ncb());
  }
  __device__ __forceinline__ const float* row_ptr(int64_t yy) const {
    yy = yy < 0 ? 0 : (yy >= (int64_t)p.h ? (int64_t)p.h - 1 : yy);
    return in + (size_t)yy * p.w;
  }
  // One output row for this lane's 4 columns from a 5-row window of the 8
  // input columns x-2 .. x+5, in the fixed tap order.
  __device__ __forceinline__ void out4(const float* r0, const float* r1, const float* r2, const float* r3,
                                       const float* r4, float o[4]) const {
    const float* r[5] = {r0, r1, r2, r3, r4};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float acc = 0.0f;
#pragma unroll
      for (int dy = 0; dy < 5; ++dy)
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) acc = __builtin_fmaf(w[dy * 5 + dx], r[dy][q + dx], acc);
      o[q] = acc;
    }
  }

  // Fast path: the wave's 256 columns lie inside the image and rows are
  // 16-byte aligned. Each lane loads its float4; the two columns on either
  // side come from the neighbouring lanes by DPP, and the wave's outer halo
  // from four uniform (scalar) loads clamped to the image.
  struct Raw {
    float4 c;
    float l0, l1, r0, r1;
  };
  __device__ __forceinline__ void load_raw(int64_t yy, uint32_t x, uint32_t xw, Raw& a) const {
    const float* row = row_ptr(yy);
    a.c = *reinterpret_cast<const float4*>(row + x);
    a.l0 = uniform_load(row + (xw >= 2 ? xw - 2 : 0));
    a.l1 = uniform_load(row + (xw >= 1 ? xw - 1 : 0));
    a.r0 = uniform_load(row + (xw + 256 < p.w ? xw + 256 : p.w - 1));
    a.r1 = uniform_load(row + (xw + 257 < p.w ? xw + 257 : p.w - 1));
  }
  __device__ __forceinline__ void expand(const Raw& a, float v[8]) const {
    v[0] = dpp_from_left(a.l0, a.c.z);
    v[1] = dpp_from_left(a.l1, a.c.w);
    v[2] = a.c.x;
    v[3] = a.c.y;
    v[4] = a.c.z;
    v[5] = a.c.w;
    v[6] = dpp_from_right(a.r0, a.c.x);
    v[7] = dpp_from_right(a.r1, a.c.y);
  }
  __device__ void run_fast(uint64_t r0, uint64_t r1, uint32_t x, uint32_t xw) const {
    // Rotating window of 6 rows: row y lives in slot (y - r0 + 2) mod 6; the
    // row two below the current one is requested one step ahead.
    float v[6][8];
    Raw pend;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Raw a;
      load_raw((int64_t)r0 - 2 + j, x, xw, a);
      expand(a, v[j]);
    }
    load_raw((int64_t)r0 + 2, x, xw, pend);
    for (uint64_t yb = r0; yb < r1; yb += 6) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const uint64_t y = yb + k;
        if (y >= r1) break;
        expand(pend, v[(k + 4) % 6]);  // row y + 2
        if (y + 1 < r1) load_raw((int64_t)y + 3, x, xw, pend);
        float o[4];
        out4(v[k % 6], v[(k + 1) % 6], v[(k + 2) % 6], v[(k + 3) % 6], v[(k + 4) % 6], o);
        // Streaming store: the output is not read again by this kernel, so
        // it should not push the input rows (reused as halo) out of L2.
        const f32x4 ov = {o[0], o[1], o[2], o[3]};
        __builtin_nontemporal_store(ov, reinterpret_cast<f32x4*>(out + (size_t)y * p.w + x));
      }
    }
  }

  // General path (ragged widths, the wave holding the image's right edge when
  // the width is not a multiple of 4): per-element clamped loads.
  __device__ void load8(int64_t yy, uint32_t x, float v[8]) const {
    const float* row = row_ptr(yy);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int64_t xx = (int64_t)x - 2 + k;
      xx = xx < 0 ? 0 : (xx >= (int64_t)p.w ? (int64_t)p.w - 1 : xx);
      v[k] = row[xx];
    }
  }
  __device__ void run_general(uint64_t r0, uint64_t r1, uint32_t x) const {
    if (x >= p.w) return;
    float win[5][8];
#pragma unroll
    for (int j = 0; j < 4; ++j) load8((int64_t)r0 - 2 + j, x, win[j + 1]);
    for (uint64_t y = r0; y < r1; ++y) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < 8; ++k) win[j][k] = win[j + 1][k];
      load8((int64_t)y + 2, x, win[4]);
      float o[4];
      out4(win[0], win[1], win[2], win[3], win[4], o);
      float* orow = out + (size_t)y * p.w;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (x + q < p.w) __builtin_nontemporal_store(o[q], orow + x + q);
    }
  }

  __device__ void run(uint64_t g0, uint64_t g1, uint32_t t) const {
    const uint32_t nc = ncb();
    const uint64_t r0 = g0 + (uint64_t)(t / nc) * kBlurTileRows;
    const uint64_t r1 = (r0 + kBlurTileRows < g1) ? r0 + kBlurTileRows : g1;
    // first column of this wave (uniform) and of this lane
    const uint32_t xw = (t % nc) * kBlurTileCols + (__builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u) * 4u;
    const uint32_t x = xw + (threadIdx.x & 63u) * 4u;
    if (xw >= p.w) return;
    if ((p.w & 3u) == 0 && xw + 256 <= p.w)
      run_fast(r0, r1, x, xw);
    else
      run_general(r0, r1, x);
  }
};

using Blur5Tile = Blur5TileT<false>;
using Blur5TileFresh = Blur5TileT<true>;

// Lomont, "Fast Inverse Square Root" (2003): integer estimate then three
// Newton-Raphson steps y <- y (1.5 - (x/2) y^2) written as t = y*y,
// u = fma(-(x/2), t, 1.5), y = y*u. Same operation sequence as the host.
__device__ __forceinline__ float rsqrt_lomont(float x) {
  const uint32_t b = 0x5f375a86u - (__float_as_uint(x) >> 1);
  float y = __uint_as_float(b);
  const float hx = 0.5f * x;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const float t = y * y;
    const float u = __builtin_fmaf(-hx, t, 1.5f);
    y = y * u;
  }
  return y;
}

// All-pairs acceleration of body i (NBody program, force part): the sum of
// m_j d_ij / (|d_ij|^2 + eps2)^(3/2) over j ascending, one FP32 sum per
// component. Positions of the j bodies are staged through LDS 256 at a time;
// every thread of the workgroup takes part in the staging, and loads its
// part of the next stage while the current one is computed (at 65,536
// bodies a workgroup is one wave per SIMD, so no other wave hides that
// load). Eight bodies per step: measured against 4 and 16, and against
// reading the next eight from LDS during the current eight, it is fastest.
template <bool STRICT>
__device__ __forceinline__ void nbody_accumulate(const float4* pos, uint32_t n, float eps2, const float4 pi,
                                                 float4* sh, float& ax, float& ay, float& az) {
  ax = 0.0f;
  ay = 0.0f;
  az = 0.0f;
  float4 stage = make_float4(0.f, 0.f, 0.f, 0.f);
  if (threadIdx.x < n) stage = pos[threadIdx.x];
  for (uint32_t j0 = 0; j0 < n; j0 += kNbodyGranule) {
    __syncthreads();
    sh[threadIdx.x] = stage;
    __syncthreads();
    if (j0 + kNbodyGranule + threadIdx.x < n) stage = pos[j0 + kNbodyGranule + threadIdx.x];
    const uint32_t m = (n - j0 < kNbodyGranule) ? n - j0 : kNbodyGranule;
    const auto body = [&](const float4 pj) {
      const float dx = pj.x - pi.x;
      const float dy = pj.y - pi.y;
      const float dz = pj.z - pi.z;
      const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
      const float rinv = STRICT ? rsqrt_lomont(r2) : __builtin_amdgcn_rsqf(r2);
      const float s = (rinv * rinv) * rinv;
      const float f = pj.w * s;
      ax = __builtin_fmaf(f, dx, ax);
      ay = __builtin_fmaf(f, dy, ay);
      az = __builtin_fmaf(f, dz, az);
    };
    // Two batches of eight bodies in registers: the next batch is read from
    // LDS while the current one is computed, so the reads' latency never
    // waits on the arithmetic (with one wave per SIMD nothing else would
    // hide it, and how much of it a plain unrolled loop hides depends on the
    // compiler's schedule). Scheduling fences keep each batch's reads a
    // phase ahead of its arithmetic; the bodies of a batch still interleave.
    // The bodies are taken in index order.
    uint32_t jj = 0;
    if (m >= 8) {
      float4 a[8], b[8];
#pragma unroll
      for (uint32_t k = 0; k < 8; ++k) a[k] = sh[k];
      for (; jj + 16 <= m; jj += 16) {
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) b[k] = sh[jj + 8 + k];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) body(a[k]);
        __builtin_amdgcn_sched_barrier(0);
        // the batch after (read within the stage; unused past its end)
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) a[k] = sh[(jj + 16 + k) & (kNbodyGranule - 1)];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) body(b[k]);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (jj + 8 <= m) {
#pragma unroll
        for (uint32_t k = 0; k < 8; ++k) body(a[k]);
        jj += 8;
      }
    }
    for (; jj < m; ++jj) body(sh[jj]);
  }
}

// Accelerations: a granule is 256 bodies, one per thread.
template <bool STRICT>
struct NbodyTile {
  static constexpr int kMinBlocksPerCu = 1;  // one granule per workgroup: no bound
  ce_nbody_params p;
  const float4* pos;
  float4* out;
  __device__ void load_constants() {}
  __host__ __device__ uint64_t granules() const { return ceil_div(p.n, kNbodyGranule); }
  __host__ __device__ uint32_t ntiles(uint64_t g0, uint64_t g1) const { return (uint32_t)(g1 - g0); }
  __device__ void run(uint64_t g0, uint64_t, uint32_t t) const {
    __shared__ float4 sh[kNbodyGranule];
    const uint64_t i = (g0 + t) * kNbodyGranule + threadIdx.x;
    const bool active = i < p.n;
    const float4 pi = active ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    float ax, ay, az;
    nbody_accumulate<STRICT>(pos, p.n, p.eps2, pi, sh, ax, ay, az);
    if (active) out[i] = make_float4(ax, ay, az, 0.0f);
  }
};

// Integration step (NBody program: positions and velocities in and out):
// with the acceleration above, v' = v + a dt and x' = x + v dt + a dt^2/2,
// per component as h = (dt dt) 0.5, x' = (x + v dt) + a h, v' = v + a dt;
// the mass and the velocity's w are copied.
template <bool STRICT>
struct NbodyStepTile {
  static constexpr int kMinBlocksPerCu = 1;
  ce_nbody_step_params p;
  const float4* pos;
  const float4* vel;
  float4* pos_out;
  float4* vel_out;
  __device__ void load_constants() {}
  __host__ __device__ uint64_t granules() const { return ceil_div(p.n, kNbodyGranule); }
  __host__ __device__ uint32_t ntiles(uint64_t g0, uint64_t g1) const { return (uint32_t)(g1 - g0); }
  __device__ void run(uint64_t g0, uint64_t, uint32_t t) const {
    __shared__ float4 sh[kNbodyGranule];
    const uint64_t i = (g0 + t) * kNbodyGranule + threadIdx.x;
    const bool active = i < p.n;
    const float4 pi = active ? pos[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    float ax, ay, az;
    nbody_accumulate<STRICT>(pos, p.n, p.eps2, pi, sh, ax, ay, az);
    if (!active) return;
    const float4 vi = vel[i];
    const float dt = p.dt;
    const float h = (dt * dt) * 0.5f;
    float4 xo, vo;
    xo.x = (pi.x + vi.x * dt) + ax * h;
    xo.y = (pi.y + vi.y * dt) + ay * h;
    xo.z = (pi.z + vi.z * dt) + az * h;
    xo.w = pi.w;
    vo.x = vi.x + ax * dt;
    vo.y = vi.y + ay * dt;
    vo.z = vi.z + az * dt;
    vo.w = vi.w;
    pos_out[i] = xo;
    vel_out[i] = vo;
  }
};

// Binomial option pricing: a granule is one work-group pricing four calls
// (one float4 of spots). Thread j holds leaf j of all four trees. At each
// level of the backward induction a node needs its upper neighbour, held by
// the next lane: inside a wave it arrives by a DPP wave shift, and only the
// first lane of each wave goes through LDS, to the last lane of the wave
// below, after one barrier per level. Waves whose nodes all lie above the
// level skip the arithmetic; inside a working wave every lane computes, and
// lanes above the level produce values that no later level reads. The loop
// is bound by barrier latency and issue, so the persistent kernel is asked
// for eight resident workgroups per CU, as many as a plain launch reaches.
struct BinomialTile {
  static constexpr int kMinBlocksPerCu = 8;
  static constexpr uint32_t kWaves = kBlockThreads / 64;
  ce_binomial_params p;
  const float4* spots;
  const float* factors;
  float4* out;
  __device__ void load_constants() {}
  __host__ __device__ uint64_t granules() const { return p.n_groups; }
  // A tile is two consecutive groups (the last tile of a package may hold
  // one): both trees advance together, so each barrier serves twice the work.
  static constexpr uint32_t kGroupsPerTile = 2;
  __host__ __device__ uint32_t ntiles(uint64_t g0, uint64_t g1) const {
    return (uint32_t)((g1 - g0 + kGroupsPerTile - 1) / kGroupsPerTile);
  }
  // Lane i receives lane i + 1's value (DPP wave_shl:1); the last lane,
  // which has no source, keeps `top`.
  static __device__ float from_next_lane(float x, float top) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(top), __float_as_int(x), 0x130, 0xf, 0xf, false));
  }
  __device__ float4 leaves(float4 S, float f, float X) const {
    const float a = S.x * f - X, b = S.y * f - X, c = S.z * f - X, d = S.w * f - X;
    return make_float4(a > 0.0f ? a : 0.0f, b > 0.0f ? b : 0.0f, c > 0.0f ? c : 0.0f, d > 0.0f ? d : 0.0f);
  }
  __device__ void level(float4& v, const float4& top, float pu, float pd) const {
    const float ux = from_next_lane(v.x, top.x), uy = from_next_lane(v.y, top.y);
    const float uz = from_next_lane(v.z, top.z), uw = from_next_lane(v.w, top.w);
    v.x = pu * ux + pd * v.x;
    v.y = pu * uy + pd * v.y;
    v.z = pu * uz + pd * v.z;
    v.w = pu * uw + pd * v.w;
  }
  __device__ void run(uint64_t g0, uint64_t g1, uint32_t t) const {
    // edge[L & 1][k][w] holds the level-L value of the first lane of wave w
    // for the tile's group k; slot kWaves is never written and feeds only
    // the unused last leaf.
    __shared__ float4 edge[2][kGroupsPerTile][kWaves + 1];
    const uint64_t grp = g0 + (uint64_t)t * kGroupsPerTile;
    const bool two = grp + 1 < g1;  // uniform across the workgroup
    const uint32_t j = threadIdx.x;
    const uint32_t w = __builtin_amdgcn_readfirstlane(j >> 6);
    const uint32_t n = p.steps;
    const float4 S0 = spots[grp];
    const float4 S1 = two ? spots[grp + 1] : S0;
    const float X = p.strike, pu = p.pu, pd = p.pd;
    float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
    if (j <= n) {
      const float f = factors[j];
      v0 = leaves(S0, f, X);
      v1 = leaves(S1, f, X);
    }
    // Level L's copy of edge is rewritten at level L - 2, after the barrier of
    // level L - 1 that follows every read of it, so one barrier per level suffices.
    for (uint32_t L = n; L-- > 0;) {
      float4(*e)[kWaves + 1] = edge[L & 1];
      if ((j & 63) == 0) {
        e[0][w] = v0;
        e[1][w] = v1;
      }
      __syncthreads();
      if (w * 64 <= L) {
        const float4 top0 = e[0][w + 1], top1 = e[1][w + 1];
        level(v0, top0, pu, pd);
        level(v1, top1, pu, pd);
      }
    }
    if (j == 0) {
      out[grp] = v0;
      if (two) out[grp + 1] = v1;
    }
  }
};

}  // namespace ce
