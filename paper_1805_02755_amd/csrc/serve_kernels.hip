// Serving kernel for gfx950: one persistent launch per serving session runs
// every job the host admits during the session. Jobs are published by the
// host in a ring in host-coherent memory; the kernel appends each new job's
// tiles to one growing ticket space (the same ticket chain as the
// co-execution kernel, with a job in place of a package), so tiles of jobs
// admitted while others are running interleave on the device. The workgroup
// whose ticket is the first one past the published tiles is the only one
// that reads the host ring. When a job's last tile finishes, that workgroup
// writes the job's completion word in host memory.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "device_atomics.hpp"
#include "device_tiles.hpp"
#include "serve.hpp"

namespace ce {

namespace {

constexpr uint32_t kDescWords = sizeof(ServeDesc) / 8;

__device__ __forceinline__ uint64_t sys_load_c(const uint64_t* p) { return sys_load(const_cast<uint64_t*>(p)); }

// Takes the next tile ticket; returns false when the session is over (the
// host said stop, the ring is full, or no job came for idle_ticks).
__device__ bool serve_next(const ServeArgs& a, uint64_t t_start, uint32_t* p_cache, uint64_t* base_cache,
                           uint32_t* job, uint32_t* ti, uint32_t* nt) {
  ServeState* q = a.q;
  const uint64_t t = dev_add(&q->ticket, (uint64_t)1);
  for (;;) {
    // consumed jobs and their tiles are one word, so they are read together
    // the flag, the job count and the tile count are one word, read together
    const uint64_t ct = dev_load(&q->ct);
    const uint64_t tot = ct & kServeTotalMask, c = (ct & ~kServeDone) >> kServeTotalBits;
    if (t < tot) break;
    if (ct & kServeDone) return false;
    if (t == tot) {
      // this workgroup appends the next admitted job, if there is one
      uint64_t h = sys_load(&a.ctl->head);
      bool stop = false;
      if (c >= h && sys_load(&a.ctl->stop)) {
        // the host set stop after its last head update: read head again, ordered after stop
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        h = sys_load(&a.ctl->head);
        stop = c >= h;
      }
      if (c < h && c < a.cap) {
        const uint64_t* src = reinterpret_cast<const uint64_t*>(&a.ring[c]);
        uint64_t* dst = reinterpret_cast<uint64_t*>(&a.table[c]);
        uint64_t w[kDescWords];
#pragma unroll
        for (uint32_t k = 0; k < kDescWords; ++k) w[k] = sys_load_c(src + k);
#pragma unroll
        for (uint32_t k = 0; k < kDescWords; ++k) dev_store(dst + k, w[k]);
        const uint32_t ntl = (uint32_t)w[1];  // ntiles: low half of the second word
        __hip_atomic_store(&a.pub[c], (uint64_t)ntl, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        dev_store(&q->t_active, now_tick());
        dev_store(&q->ct, ((c + 1) << kServeTotalBits) | (tot + ntl));
        continue;
      }
      // Idle: no job appended for idle_ticks, a normal end of the session
      // (the host publishes a job that comes too late in the next one). Only
      // this workgroup appends jobs and writes ct, so the two decisions
      // cannot cross. The tick of the last append may be later than this
      // workgroup's clock read: compare, never subtract blindly.
      const uint64_t now = now_tick();
      uint64_t ta = dev_load(&q->t_active);
      if (ta < t_start) ta = t_start;
      if (stop || c >= a.cap || (now > ta && now - ta > a.idle_ticks)) {
        dev_store(&q->ct, ct | kServeDone);  // only this workgroup writes ct now
        return false;
      }
    }
    if (t == tot)
      __builtin_amdgcn_s_sleep(2);
    else
      __builtin_amdgcn_s_sleep(16);
  }
  uint32_t p = *p_cache;
  uint64_t base = *base_cache;
  for (uint64_t t1 = 0;;) {
    const uint64_t n = dev_load(&a.pub[p]);
    if (n == 0) {  // published but not visible here yet
      if (t1 == 0) t1 = now_tick();
      if (now_tick() - t1 > a.idle_ticks) {
        dev_store(&q->flags, 1u);
        return false;
      }
      continue;
    }
    if (t < base + n) {
      *p_cache = p;
      *base_cache = base;
      *job = p;
      *ti = (uint32_t)(t - base);
      *nt = (uint32_t)n;
      return true;
    }
    base += n;
    ++p;
  }
}

// Runs tile ti of the job described in LDS (uniform across the workgroup).
__device__ void serve_tile(const ServeDesc& d, uint32_t ti) {
  const uint32_t kind = __builtin_amdgcn_readfirstlane(d.kind);
  if (kind == CE_KERNEL_ESCAPE) {
    EscapeTile e{d.esc, (uint32_t*)d.out};
    e.run(0, d.granules, ti);
  } else if (kind == CE_KERNEL_BLUR5) {
    Blur5TileFresh b{d.blur, (const float*)d.in0, (const float*)d.in1, (float*)d.out, {}};
    b.load_constants();
    b.run(0, d.granules, ti);
  } else if (__builtin_amdgcn_readfirstlane(d.strict)) {
    NbodyTile<true> nbt{d.nb, (const float4*)d.in0, (float4*)d.out};
    nbt.run(0, d.granules, ti);
  } else {
    NbodyTile<false> nbt{d.nb, (const float4*)d.in0, (float4*)d.out};
    nbt.run(0, d.granules, ti);
  }
}

}  // namespace

__global__ __launch_bounds__(kBlockThreads) void k_serve(ServeArgs a) {
  __shared__ ServeDesc sh_desc;
  __shared__ uint32_t sh_go, sh_job, sh_ti, sh_nt;
  const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) == 0;
  const bool lane0 = threadIdx.x == 0;
  const uint64_t t_start = now_tick();
  uint32_t p_cache = 0, cur_job = 0xFFFFFFFFu, prev_job = 0xFFFFFFFFu, prev_nt = 0;
  uint64_t base_cache = 0;
  for (;;) {
    if (wave0) {
      if (lane0) {
        if (prev_job != 0xFFFFFFFFu) {
          // release: this tile's output is written back before it is counted
          const uint32_t old = __hip_atomic_fetch_add(&a.tiles_done[prev_job], 1u, __ATOMIC_RELEASE,
                                                      __HIP_MEMORY_SCOPE_AGENT);
          if (old + 1 == prev_nt) {
            __atomic_thread_fence(__ATOMIC_ACQUIRE);
            const uint64_t seq = dev_load(reinterpret_cast<uint64_t*>(&a.table[prev_job].seq));
            sys_store_release(&a.done_words[seq], now_tick() | 1ull);
          }
        }
        uint32_t job = 0, ti = 0, nt = 0;
        const bool go = serve_next(a, t_start, &p_cache, &base_cache, &job, &ti, &nt);
        // the job's first tile: its start is when the job reached the device
        if (go && ti == 0) sys_store(&a.first_words[job], now_tick());
        if (go && job != cur_job) {
          // descriptor of a new job: coherent loads from its table entry
          const uint64_t* src = reinterpret_cast<const uint64_t*>(&a.table[job]);
          uint64_t* dst = reinterpret_cast<uint64_t*>(&sh_desc);
#pragma unroll
          for (uint32_t k = 0; k < kDescWords; ++k) dst[k] = dev_load(const_cast<uint64_t*>(src + k));
          cur_job = job;
          // The job's inputs may have been copied in (into memory an earlier
          // job used) after this launch began: drop cached lines before reading.
          if (sh_desc.kind != CE_KERNEL_ESCAPE) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        }
        sh_go = go ? 1u : 0u;
        sh_job = job;
        sh_ti = ti;
        sh_nt = nt;
      }
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(sh_go) == 0) break;
    serve_tile(sh_desc, __builtin_amdgcn_readfirstlane(sh_ti));
    prev_job = __builtin_amdgcn_readfirstlane(sh_job);
    prev_nt = __builtin_amdgcn_readfirstlane(sh_nt);
    __syncthreads();
  }
  if (wave0) {
    if (lane0) {
      __builtin_amdgcn_s_waitcnt(0);  // this workgroup's atomics are done before it counts itself out
      const uint32_t ex = dev_add(&a.q->exit_count, 1u);
      if (ex + 1 == gridDim.x) {
        if (dev_load(&a.q->flags)) sys_store(&a.ctl->flags, 1);
        // jobs taken from the ring: the host publishes any later one again
        sys_store(&a.ctl->consumed, (dev_load(&a.q->ct) & ~kServeDone) >> kServeTotalBits);
        sys_store_release(&a.ctl->exited, a.session);
      }
    }
  }
}

uint32_t serve_tiles(const ServeDesc& d) {
  switch (d.kind) {
    case CE_KERNEL_ESCAPE: return EscapeTile{d.esc, nullptr}.ntiles(0, d.esc.h);
    case CE_KERNEL_BLUR5: return Blur5Tile{d.blur, nullptr, nullptr, nullptr, {}}.ntiles(0, d.blur.h);
    case CE_KERNEL_NBODY_ACC: return (uint32_t)ceil_div(d.nb.n, kNbodyGranule);
  }
  return 0;
}

uint64_t serve_granules(const ServeDesc& d) {
  switch (d.kind) {
    case CE_KERNEL_ESCAPE: return d.esc.h;
    case CE_KERNEL_BLUR5: return d.blur.h;
    case CE_KERNEL_NBODY_ACC: return ceil_div(d.nb.n, kNbodyGranule);
  }
  return 0;
}

hipError_t serve_blocks_per_cu(int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_serve, kBlockThreads, 0);
}

hipError_t launch_serve(const ServeArgs& a, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(k_serve, dim3(grid), dim3(kBlockThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace ce
