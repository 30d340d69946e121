// Batched escape-time kernel for gfx950: one persistent launch runs every job
// of a batch. The jobs' tiles are concatenated in job order; workgroups take
// packages of `pkg_tiles` consecutive tiles from an HBM counter (a Dynamic
// schedule inside the GPU) and find each tile's job by binary search over the
// jobs' first tiles, kept in LDS. The per-pixel arithmetic is the same
// escape_count as the single-job kernels.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "common.hpp"
#include "device_payloads.hpp"

namespace ce {

template <uint32_t TR>
__global__ __launch_bounds__(kBlockThreads) void k_batch_escape(BatchArgs a) {
  constexpr uint32_t TC = kBlockThreads / TR;
  extern __shared__ uint64_t sh_base[];  // first tile of each job (n_jobs entries)
  __shared__ uint64_t sh_tile;
  for (uint32_t j = threadIdx.x; j < a.n_jobs; j += kBlockThreads) sh_base[j] = a.jobs[j].tile_base;
  const bool lane0 = threadIdx.x == 0;
  const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) == 0;
  uint32_t job = 0;  // largest job whose first tile is <= the current tile (tiles only increase)
  for (;;) {
    __syncthreads();  // table loaded / previous package finished reading sh_tile
    if (wave0) {
      if (lane0)
        sh_tile = __hip_atomic_fetch_add(&a.counter[0], (uint64_t)a.pkg_tiles, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint64_t t0 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(sh_tile >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)sh_tile);
    if (t0 >= a.total_tiles) break;
    const uint64_t t1 = (t0 + a.pkg_tiles < a.total_tiles) ? t0 + a.pkg_tiles : a.total_tiles;
    for (uint64_t t = t0; t < t1; ++t) {
      uint32_t l = job, h = a.n_jobs;  // sh_base[l] <= t < sh_base[h] (sh_base[n_jobs] = end)
      while (h - l > 1) {
        const uint32_t m = (l + h) >> 1;
        if (sh_base[m] <= t) l = m; else h = m;
      }
      job = __builtin_amdgcn_readfirstlane(l);
      const BatchJob& J = a.jobs[job];
      const uint64_t local = t - sh_base[job];
      const uint32_t ty = (uint32_t)(local / J.tiles_x), tx = (uint32_t)(local % J.tiles_x);
      const uint32_t r = ty * TR + threadIdx.x / TC;
      const uint32_t c = tx * TC + threadIdx.x % TC;
      if (r < J.p.h && c < J.p.w) {
        const float cr = J.p.x0 + (float)c * J.p.dx;
        const float ci = J.p.y0 + (float)r * J.p.dy;
        J.out[(size_t)r * J.p.w + c] = escape_count(cr, ci, J.p.max_iter);
      }
    }
  }
  // the last workgroup out re-arms the counter for the next launch (no memset
  // node is needed when the launch is replayed from a graph)
  if (wave0) {
    if (lane0) {
      const uint64_t ex = __hip_atomic_fetch_add(&a.counter[1], (uint64_t)1, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
      if (ex + 1 == gridDim.x) {
        __hip_atomic_store(&a.counter[0], (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.counter[1], (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

uint32_t batch_shape_cols(int shape) { return kBlockThreads / kBatchShapeRows[shape]; }

hipError_t batch_blocks_per_cu(int shape, size_t lds, int* blocks) {
  switch (shape) {
    case 0: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_escape<1>, kBlockThreads, lds);
    case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_escape<2>, kBlockThreads, lds);
    case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_escape<4>, kBlockThreads, lds);
    case 3: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_escape<8>, kBlockThreads, lds);
    case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_escape<16>, kBlockThreads, lds);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch(int shape, const BatchArgs& a, uint32_t grid, hipStream_t st) {
  const dim3 g(grid), b(kBlockThreads);
  const size_t lds = (size_t)a.n_jobs * sizeof(uint64_t);
  switch (shape) {
    case 0: hipLaunchKernelGGL(k_batch_escape<1>, g, b, lds, st, a); break;
    case 1: hipLaunchKernelGGL(k_batch_escape<2>, g, b, lds, st, a); break;
    case 2: hipLaunchKernelGGL(k_batch_escape<4>, g, b, lds, st, a); break;
    case 3: hipLaunchKernelGGL(k_batch_escape<8>, g, b, lds, st, a); break;
    case 4: hipLaunchKernelGGL(k_batch_escape<16>, g, b, lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ce
