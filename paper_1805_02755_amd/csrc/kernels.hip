// GPU side of the co-execution engine for gfx950 (CDNA4).
//
// One persistent kernel per payload pulls packages of the index space from a
// two-level dispenser (section 5.3 schedulers, section 4.2 architecture):
//  - level 1 lives in host-coherent pinned memory and is shared with the host
//    worker pool; the GPU reaches it with system-scope atomics over PCIe;
//  - level 2 lives in HBM: a ticket counter hands the tiles of the GPU's
//    current package to its workgroups with device-scope atomics.
// The workgroup whose ticket is the first one past the published tiles is the
// only one that claims the next level-1 package, so the GPU acts as a single
// device towards the scheduler while all its workgroups share each package.
//
// Payload arithmetic is written one FP32 operation at a time and compiled
// with -ffp-contract=off, so every work-item gets the same bits as on the
// host workers.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

namespace ce {

// ---------------------------------------------------------------- utilities
__device__ __forceinline__ uint64_t now_tick() { return __builtin_amdgcn_s_memrealtime(); }

// Memory ordering. On gfx950 each XCD has its own L2, so an agent-scope
// acquire or release invalidates or writes back the L2; doing that per tile
// would throttle the streaming payloads. The dispenser therefore uses relaxed
// atomics on its hot path (agent- and system-scope atomics are performed at
// the coherent memory side, so every access sees the latest value of its
// location) and publishes package descriptors as single 64-bit words that
// readers spin on. Acquire/release is used only for the claim lock (once
// per package) and when a workgroup leaves (once per run).
__device__ __forceinline__ uint64_t sys_load(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void sys_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void sys_store_release(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t sys_fetch_add(uint64_t* p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ bool sys_cas(uint64_t* p, uint64_t* expected, uint64_t desired) {
  return __hip_atomic_compare_exchange_strong(p, expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_SYSTEM);
}
template <class U>
__device__ __forceinline__ U dev_load(U* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class U>
__device__ __forceinline__ void dev_store(U* p, U v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class U>
__device__ __forceinline__ U dev_add(U* p, U v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------------------- payloads
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

struct EscapeTile {
  ce_escape_params p;
  uint32_t* out;
  __device__ void load_constants() {}
  __host__ __device__ uint32_t ncb() const { return (uint32_t)ceil_div(p.w, kEscapeTileCols); }
  __host__ __device__ uint64_t granules() const { return p.h; }
  __host__ __device__ uint32_t ntiles(uint64_t g0, uint64_t g1) const {
    return (uint32_t)(ceil_div(g1 - g0, kEscapeTileRows) * ncb());
  }
  // A tile is 16 rows x 64 columns; each wave covers four 8 x 8 blocks so
  // the lanes of a wave iterate over neighbouring pixels.
  __device__ void run(uint64_t g0, uint64_t g1, uint32_t t) const {
    const uint32_t nc = ncb();
    const uint64_t rb = g0 + (uint64_t)(t / nc) * kEscapeTileRows;
    const uint32_t cb = (t % nc) * kEscapeTileCols;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
#pragma unroll 1
    for (uint32_t i = 0; i < 4; ++i) {
      const uint32_t b = wave * 4u + i;
      const uint64_t r = rb + (b >> 3) * 8u + (lane >> 3);
      const uint32_t c = cb + (b & 7u) * 8u + (lane & 7u);
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

struct Blur5Tile {
  ce_blur5_params p;
  const float* in;
  const float* wt;
  float* out;
  float w[25];
  // Weights are read once per workgroup in uniform control flow, so they
  // live in scalar registers and feed the FMAs as scalar operands.
  __device__ void load_constants() {
#pragma unroll
    for (int k = 0; k < 25; ++k) w[k] = wt[k];
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
    a.l0 = row[xw >= 2 ? xw - 2 : 0];
    a.l1 = row[xw >= 1 ? xw - 1 : 0];
    a.r0 = row[xw + 256 < p.w ? xw + 256 : p.w - 1];
    a.r1 = row[xw + 257 < p.w ? xw + 257 : p.w - 1];
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
        *reinterpret_cast<float4*>(out + (size_t)y * p.w + x) = make_float4(o[0], o[1], o[2], o[3]);
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
        if (x + q < p.w) orow[x + q] = o[q];
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

// All-pairs acceleration (NBody program, force part): body i accumulates
// m_j d_ij / (|d_ij|^2 + eps2)^(3/2) over j ascending in one FP32 sum per
// component. A granule is 256 bodies, one per thread; positions of the j
// bodies are staged through LDS 256 at a time.
template <bool STRICT>
struct NbodyTile {
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
    const float eps2 = p.eps2;
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    for (uint32_t j0 = 0; j0 < p.n; j0 += kNbodyGranule) {
      __syncthreads();
      if (j0 + threadIdx.x < p.n) sh[threadIdx.x] = pos[j0 + threadIdx.x];
      __syncthreads();
      const uint32_t m = (p.n - j0 < kNbodyGranule) ? p.n - j0 : kNbodyGranule;
#pragma unroll 8
      for (uint32_t jj = 0; jj < m; ++jj) {
        const float4 pj = sh[jj];
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
      }
    }
    if (active) out[i] = make_float4(ax, ay, az, 0.0f);
  }
};

// ---------------------------------------------------------------- dispenser
// Claims the next level-1 package for the GPU. Only the holder of the claim
// lock runs this.
__device__ bool claim_package(const SchedArgs& s, uint64_t* g0, uint64_t* g1, bool* timed_out) {
  L2State* q = s.l2;
  if (s.kind == kStatic) {
    const uint32_t b = dev_load(&q->st_next);
    if (s.st_nbands == 0) {
      // one package per device, cut only if it exceeds the descriptor's size field
      const uint64_t a = s.st_begin + (uint64_t)b * kPubMaxSize;
      if (a >= s.st_end) return false;
      *g0 = a;
      *g1 = (s.st_end - a > kPubMaxSize) ? a + kPubMaxSize : s.st_end;
    } else {
      const uint64_t b0 = s.st_begin + b;  // st_begin/st_end hold band indices here
      if (b0 >= s.st_end) return false;
      *g0 = band_edge(b0, s.G, s.st_nbands);
      *g1 = band_edge(b0 + 1, s.G, s.st_nbands);
    }
    dev_store(&q->st_next, b + 1);
    return true;
  }
  if (s.kind == kDynamic) {
    const uint64_t a = sys_fetch_add(&s.l1->next, s.pkg);
    if (a >= s.G) return false;
    *g0 = a;
    *g1 = (a + s.pkg < s.G) ? a + s.pkg : s.G;
    return true;
  }
  // HGuided: the size follows the pending granules at the moment of the claim.
  uint64_t cur = sys_load(&s.l1->next);
  for (uint64_t tries = 0;; ++tries) {
    if (cur >= s.G) return false;
    uint64_t sz = hguided_size(s.G - cur, s.P_self, s.sumP, s.n_dev, s.k, s.min_self);
    if (sz > kPubMaxSize) sz = kPubMaxSize;
    if (sys_cas(&s.l1->next, &cur, cur + sz)) {
      *g0 = cur;
      *g1 = cur + sz;
      return true;
    }
    if (tries > s.spin_limit) {
      *timed_out = true;
      return false;
    }
  }
}

// Publishes one package at the end of the GPU's tile sequence (lock held).
template <class T>
__device__ void publish(const T& pay, const SchedArgs& s, uint64_t tot, uint64_t g0, uint64_t g1, uint64_t tc) {
  L2State* q = s.l2;
  const uint32_t n = dev_load(&q->n_pkgs);
  const uint32_t nt = pay.ntiles(g0, g1);
  PkgSlot* ps = &s.pkgs[n];  // trace record, read by the host after the run;
  ps->g0 = g0;               // its tile counter was cleared at the end of the last run
  ps->g1 = g1;
  ps->base = tot;
  ps->ntiles = nt;
  ps->t_claim = tc;
  ps->t_end = 0;
  if (n == 0) dev_store(&q->t_first, tc);
  dev_store(&q->n_pkgs, n + 1);
  dev_store(&q->granules, dev_load(&q->granules) + (g1 - g0));
  dev_store(&s.pub[n], pub_word(g0, g1 - g0));
  dev_store(&q->total, tot + nt);
}

// Ticket chain with lookahead. A workgroup takes the next tile ticket; when
// it is within `lookahead` tiles of the end of the published tiles it tries
// to take the claim lock and append the next level-1 package, so the PCIe
// round trip of the claim overlaps the last round of tiles. The GPU thus
// acts as one device towards the scheduler while its workgroups share each
// package. Returns false when this workgroup should leave.
template <class T>
__device__ bool next_tile(const T& pay, const SchedArgs& s, uint32_t* p_cache, uint64_t* base_cache, uint32_t* p_out,
                          uint32_t* ti_out, uint64_t* g0_out, uint64_t* g1_out, uint32_t* nt_out) {
  L2State* q = s.l2;
  const uint64_t t = dev_add(&q->ticket, (uint64_t)1);
  uint64_t spins = 0;
  for (;;) {
    const uint64_t tot = dev_load(&q->total);
    if (t + s.lookahead < tot) break;
    if (dev_load(&q->done)) {
      if (t < tot) break;
      return false;
    }
    uint32_t unlocked = 0;
    if (__hip_atomic_compare_exchange_strong(&q->lock, &unlocked, 1u, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) {
      const uint64_t tot2 = dev_load(&q->total);
      if (!dev_load(&q->done) && t + s.lookahead >= tot2) {
        uint64_t g0 = 0, g1 = 0;
        bool timed_out = false;
        const uint64_t tc = now_tick();
        if (dev_load(&q->n_pkgs) >= s.max_pkgs || !claim_package(s, &g0, &g1, &timed_out)) {
          if (timed_out || dev_load(&q->n_pkgs) >= s.max_pkgs) sys_store(&s.l1->gpu_flags, 1);
          dev_store(&q->done, 1u);
        } else {
          publish(pay, s, tot2, g0, g1, tc);
        }
      }
      __hip_atomic_store(&q->lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }
    if (t < tot) break;
    if (++spins > s.spin_limit) {
      sys_store(&s.l1->gpu_flags, 1);
      dev_store(&q->done, 1u);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  // Locate the package holding ticket t: walk the publication words from the
  // last package this workgroup used, accumulating tile bases.
  uint32_t p = *p_cache;
  uint64_t base = *base_cache;
  for (uint64_t spins2 = 0;;) {
    const uint64_t w = dev_load(&s.pub[p]);
    if (w == 0) {  // published by the claimer but not visible here yet
      if (++spins2 > s.spin_limit) {
        sys_store(&s.l1->gpu_flags, 1);
        return false;
      }
      continue;
    }
    const uint64_t g0 = pub_g0(w), g1 = g0 + pub_size(w);
    const uint32_t nt = pay.ntiles(g0, g1);
    if (t < base + nt) {
      *p_cache = p;
      *base_cache = base;
      *p_out = p;
      *ti_out = (uint32_t)(t - base);
      *g0_out = g0;
      *g1_out = g1;
      *nt_out = nt;
      return true;
    }
    base += nt;
    ++p;
  }
}

__device__ __forceinline__ void tile_done(const SchedArgs& s, uint32_t p, uint32_t nt) {
  PkgSlot* ps = &s.pkgs[p];
  const uint32_t d = dev_add(&ps->tiles_done, 1u);
  if (d + 1 == nt) {
    const uint64_t te = now_tick();
    ps->t_end = te;
    __hip_atomic_fetch_max(&s.l2->t_last, te, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The last workgroup out publishes the GPU's summary to the host, clears the
// publication words and resets the level-2 state for the next run.
__device__ void leave(const SchedArgs& s) {
  L2State* q = s.l2;
  const uint32_t ex = __hip_atomic_fetch_add(&q->exit_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
  if (ex + 1 != gridDim.x) return;
  const uint64_t tf = dev_load(&q->t_first);
  const uint64_t tl = dev_load(&q->t_last);
  const uint64_t gr = dev_load(&q->granules);
  const uint32_t np = dev_load(&q->n_pkgs);
  for (uint32_t i = 0; i < np && i < s.max_pkgs; ++i) {
    dev_store(&s.pub[i], (uint64_t)0);
    dev_store(&s.pkgs[i].tiles_done, 0u);
  }
  sys_store(&s.l1->gpu_t_first, tf);
  sys_store(&s.l1->gpu_t_last, tl);
  sys_store(&s.l1->gpu_granules, gr);
  sys_store(&s.l1->gpu_packages, np);
  dev_store(&q->ticket, (uint64_t)0);
  dev_store(&q->total, (uint64_t)0);
  dev_store(&q->n_pkgs, 0u);
  dev_store(&q->done, 0u);
  dev_store(&q->st_next, 0u);
  dev_store(&q->granules, (uint64_t)0);
  dev_store(&q->t_first, (uint64_t)0);
  dev_store(&q->t_last, (uint64_t)0);
  dev_store(&q->lock, 0u);
  dev_store(&q->gather_next, (uint64_t)0);
  dev_store(&q->exit_count, 0u);
  sys_store_release(&s.l1->gpu_run_id, s.run_id);
}

// Direct claim (Dynamic with single-tile packages): the workgroup takes its
// own package from level 1. Returns false when the dispenser is exhausted.
__device__ bool direct_claim(const SchedArgs& s, uint32_t* slot_out, uint64_t* g0, uint64_t* g1) {
  const uint64_t tc = now_tick();
  const uint64_t a = sys_fetch_add(&s.l1->next, s.pkg);
  if (a >= s.G) return false;
  const uint64_t b = (a + s.pkg < s.G) ? a + s.pkg : s.G;
  const uint32_t slot = dev_add(&s.l2->n_pkgs, 1u);
  if (slot >= s.max_pkgs) {  // the host sizes the table so this cannot happen
    sys_store(&s.l1->gpu_flags, 1);
    return false;
  }
  PkgSlot* ps = &s.pkgs[slot];
  ps->g0 = a;
  ps->g1 = b;
  ps->base = 0;
  ps->ntiles = 1;
  ps->t_claim = tc;
  ps->t_end = 0;
  uint64_t zero = 0;
  __hip_atomic_compare_exchange_strong(&s.l2->t_first, &zero, tc, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  dev_add(&s.l2->granules, b - a);
  *slot_out = slot;
  *g0 = a;
  *g1 = b;
  return true;
}

// Gather (device-resident output with the host in the device set): the host
// workers publish each finished host tile as a byte range of their output
// buffer in a ring in host-coherent memory; workgroups 0 .. gather_wgs-1 read
// those ranges over PCIe and write them into the device output while the
// other workgroups compute, so no copy is left for after the kernel.
__device__ bool gather_entry(const SchedArgs& s, uint64_t* off, uint32_t* len) {
  const uint64_t j = dev_add(&s.l2->gather_next, (uint64_t)1);
  const uint64_t t0 = now_tick();
  const uint64_t want = host_final_word(s.run_id, 0) >> 40;
  for (;;) {
    if (j < s.ring_cap) {
      const uint64_t w = __hip_atomic_load(const_cast<uint64_t*>(&s.ring[j]), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
      if (w != 0) {
        *off = ring_off(w);
        *len = (uint32_t)ring_len(w);
        return true;
      }
    }
    const uint64_t f = sys_load(&s.l1->host_final);
    if ((f >> 40) == want && j >= (f & ((1ull << 40) - 1))) return false;
    if (now_tick() - t0 > s.wait_ticks) {
      sys_store(&s.l1->gpu_flags, 2);
      return false;
    }
    __builtin_amdgcn_s_sleep(8);
  }
}

__device__ void gather_copy(const SchedArgs& s, uint64_t off, uint32_t len) {
  const char* src = s.gsrc + off;
  char* dst = s.gdst + off;
  if (((off | len) & 15u) == 0) {
    const uint4* a = reinterpret_cast<const uint4*>(src);
    uint4* b = reinterpret_cast<uint4*>(dst);
    const uint32_t n = len / 16;
#pragma unroll 8
    for (uint32_t i = threadIdx.x; i < n; i += kBlockThreads) b[i] = a[i];
  } else {
    const uint32_t* a = reinterpret_cast<const uint32_t*>(src);
    uint32_t* b = reinterpret_cast<uint32_t*>(dst);
    const uint32_t n = len / 4;
#pragma unroll 8
    for (uint32_t i = threadIdx.x; i < n; i += kBlockThreads) b[i] = a[i];
  }
}

// Persistent workgroup loop. Every branch around the barriers is uniform
// across the workgroup: the claim block is entered by the whole first wave
// (readfirstlane of the thread id) and only its lane 0 touches the
// dispenser; the loop exit reads the shared flag through readfirstlane.
// With a per-lane "thread 0 only" condition instead, the compiler may
// rotate the loop so that lane 0 leaves an inner loop through an exec-mask
// update while the other lanes keep passing the barriers, which never ends.
template <class T>
__global__ __launch_bounds__(kBlockThreads) void k_persistent(T pay, SchedArgs s) {
  __shared__ uint32_t sh_go, sh_p, sh_ti, sh_nt;
  __shared__ uint64_t sh_g0, sh_g1;
  const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) == 0;
  const bool lane0 = threadIdx.x == 0;
  pay.load_constants();
  uint32_t p_cache = 0;
  uint64_t base_cache = 0;
  uint32_t prev_p = 0xFFFFFFFFu, prev_nt = 0;
  if (blockIdx.x < s.gather_wgs) {
    __shared__ uint64_t sh_off;
    __shared__ uint32_t sh_len;
    for (;;) {
      if (wave0) {
        if (lane0) {
          uint64_t off = 0;
          uint32_t len = 0;
          sh_go = gather_entry(s, &off, &len) ? 1u : 0u;
          sh_off = off;
          sh_len = len;
        }
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(sh_go) == 0) break;
      const uint64_t off = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(sh_off >> 32)) << 32) |
                           __builtin_amdgcn_readfirstlane((uint32_t)sh_off);
      gather_copy(s, off, __builtin_amdgcn_readfirstlane(sh_len));
      __syncthreads();
    }
    if (wave0) {
      if (lane0) leave(s);
    }
    return;
  }
  for (;;) {
    if (wave0) {
      if (lane0) {
        if (prev_p != 0xFFFFFFFFu) tile_done(s, prev_p, prev_nt);
        uint32_t p = 0, ti = 0, nt = 1;
        uint64_t g0 = 0, g1 = 0;
        bool go;
        if (s.direct)
          go = direct_claim(s, &p, &g0, &g1);
        else
          go = next_tile(pay, s, &p_cache, &base_cache, &p, &ti, &g0, &g1, &nt);
        sh_go = go ? 1u : 0u;
        sh_p = p;
        sh_ti = ti;
        sh_nt = nt;
        sh_g0 = g0;
        sh_g1 = g1;
      }
    }
    __syncthreads();
    const uint32_t go = __builtin_amdgcn_readfirstlane(sh_go);
    if (go == 0) break;
    const uint32_t p = __builtin_amdgcn_readfirstlane(sh_p);
    const uint32_t ti = __builtin_amdgcn_readfirstlane(sh_ti);
    const uint32_t nt = __builtin_amdgcn_readfirstlane(sh_nt);
    const uint64_t g0 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(sh_g0 >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)sh_g0);
    const uint64_t g1 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(sh_g1 >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)sh_g1);
    pay.run(g0, g1, ti);
    prev_p = p;
    prev_nt = nt;
    __syncthreads();  // the tile is complete and the shared slots may be reused
  }
  if (wave0) {
    if (lane0) leave(s);
  }
}

template <class T>
__global__ __launch_bounds__(kBlockThreads) void k_bare(T pay, uint64_t G) {
  pay.load_constants();
  pay.run(0, G, blockIdx.x);
}

__global__ void k_calibrate(L1State* l1, uint32_t rounds, uint64_t spin_limit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (uint32_t i = 1; i <= rounds; ++i) {
    uint64_t spins = 0;
    while (sys_load(&l1->ping) != i) {
      if (++spins > spin_limit) return;
      __builtin_amdgcn_s_sleep(1);
    }
    const uint64_t t = now_tick();
    sys_store(&l1->tick, t);
    sys_store(&l1->pong, i);
  }
}

// ------------------------------------------------------------ host helpers
namespace {
EscapeTile make_escape(const KernelArgs& a) { return EscapeTile{a.esc, (uint32_t*)a.out}; }
Blur5Tile make_blur(const KernelArgs& a) {
  return Blur5Tile{a.blur, (const float*)a.in0, (const float*)a.in1, (float*)a.out, {}};
}
template <bool S>
NbodyTile<S> make_nbody(const KernelArgs& a) {
  return NbodyTile<S>{a.nb, (const float4*)a.in0, (float4*)a.out};
}
}  // namespace

uint64_t gpu_granules(const KernelArgs& a) {
  switch (a.kernel_id) {
    case CE_KERNEL_ESCAPE: return make_escape(a).granules();
    case CE_KERNEL_BLUR5: return make_blur(a).granules();
    case CE_KERNEL_NBODY_ACC: return make_nbody<true>(a).granules();
  }
  return 0;
}

uint32_t gpu_tiles(const KernelArgs& a, uint64_t g0, uint64_t g1) {
  switch (a.kernel_id) {
    case CE_KERNEL_ESCAPE: return make_escape(a).ntiles(g0, g1);
    case CE_KERNEL_BLUR5: return make_blur(a).ntiles(g0, g1);
    case CE_KERNEL_NBODY_ACC: return make_nbody<true>(a).ntiles(g0, g1);
  }
  return 0;
}

hipError_t persistent_blocks_per_cu(const KernelArgs& a, int* blocks) {
  switch (a.kernel_id) {
    case CE_KERNEL_ESCAPE:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_persistent<EscapeTile>, kBlockThreads, 0);
    case CE_KERNEL_BLUR5:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_persistent<Blur5Tile>, kBlockThreads, 0);
    case CE_KERNEL_NBODY_ACC:
      return a.strict ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_persistent<NbodyTile<true>>,
                                                                     kBlockThreads, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_persistent<NbodyTile<false>>,
                                                                     kBlockThreads, 0);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_persistent(const KernelArgs& a, const SchedArgs& s, uint32_t grid, hipStream_t st) {
  const dim3 g(grid), b(kBlockThreads);
  switch (a.kernel_id) {
    case CE_KERNEL_ESCAPE: hipLaunchKernelGGL(k_persistent<EscapeTile>, g, b, 0, st, make_escape(a), s); break;
    case CE_KERNEL_BLUR5: hipLaunchKernelGGL(k_persistent<Blur5Tile>, g, b, 0, st, make_blur(a), s); break;
    case CE_KERNEL_NBODY_ACC:
      if (a.strict)
        hipLaunchKernelGGL(k_persistent<NbodyTile<true>>, g, b, 0, st, make_nbody<true>(a), s);
      else
        hipLaunchKernelGGL(k_persistent<NbodyTile<false>>, g, b, 0, st, make_nbody<false>(a), s);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bare(const KernelArgs& a, hipStream_t st) {
  const uint64_t G = gpu_granules(a);
  const uint32_t tiles = gpu_tiles(a, 0, G);
  if (tiles == 0) return hipSuccess;
  const dim3 g(tiles), b(kBlockThreads);
  switch (a.kernel_id) {
    case CE_KERNEL_ESCAPE: hipLaunchKernelGGL(k_bare<EscapeTile>, g, b, 0, st, make_escape(a), G); break;
    case CE_KERNEL_BLUR5: hipLaunchKernelGGL(k_bare<Blur5Tile>, g, b, 0, st, make_blur(a), G); break;
    case CE_KERNEL_NBODY_ACC:
      if (a.strict)
        hipLaunchKernelGGL(k_bare<NbodyTile<true>>, g, b, 0, st, make_nbody<true>(a), G);
      else
        hipLaunchKernelGGL(k_bare<NbodyTile<false>>, g, b, 0, st, make_nbody<false>(a), G);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_calibrate(L1State* l1, uint32_t rounds, uint64_t spin_limit, hipStream_t st) {
  hipLaunchKernelGGL(k_calibrate, dim3(1), dim3(64), 0, st, l1, rounds, spin_limit);
  return hipGetLastError();
}

}  // namespace ce
