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
#include "device_payloads.hpp"
#include "device_atomics.hpp"
#include "device_tiles.hpp"
#include "kernels.hpp"
#include "rt_tile.hpp"
#include "sched_device.hpp"

namespace ce {

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
BinomialTile make_binomial(const KernelArgs& a) {
  return BinomialTile{a.bin, (const float4*)a.in0, (const float*)a.in1, (float4*)a.out};
}
template <bool S>
NbodyStepTile<S> make_nbody_step(const KernelArgs& a) {
  return NbodyStepTile<S>{a.nbs, (const float4*)a.in0, (const float4*)a.in1, (float4*)a.out, (float4*)a.out1};
}
RtTile make_rt(const KernelArgs& a) { return RtTile{a.rt, a.rt_items, a.rt_lws, rt_tile_items(a.rt_items)}; }
}  // namespace

uint64_t gpu_granules(const KernelArgs& a) {
  switch (a.kernel_id) {
    case CE_KERNEL_ESCAPE: return make_escape(a).granules();
    case CE_KERNEL_BLUR5: return make_blur(a).granules();
    case CE_KERNEL_NBODY_ACC: return make_nbody<true>(a).granules();
    case CE_KERNEL_NBODY_STEP: return make_nbody_step<true>(a).granules();
    case CE_KERNEL_BINOMIAL: return make_binomial(a).granules();
    case CE_KERNEL_RUNTIME: return make_rt(a).granules();
  }
  return 0;
}

uint32_t gpu_tiles(const KernelArgs& a, uint64_t g0, uint64_t g1) {
  switch (a.kernel_id) {
    case CE_KERNEL_ESCAPE: return make_escape(a).ntiles(g0, g1);
    case CE_KERNEL_BLUR5: return make_blur(a).ntiles(g0, g1);
    case CE_KERNEL_NBODY_ACC: return make_nbody<true>(a).ntiles(g0, g1);
    case CE_KERNEL_NBODY_STEP: return make_nbody_step<true>(a).ntiles(g0, g1);
    case CE_KERNEL_BINOMIAL: return make_binomial(a).ntiles(g0, g1);
    case CE_KERNEL_RUNTIME: return make_rt(a).ntiles(g0, g1);
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
    case CE_KERNEL_NBODY_STEP:
      return a.strict ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_persistent<NbodyStepTile<true>>,
                                                                     kBlockThreads, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_persistent<NbodyStepTile<false>>,
                                                                     kBlockThreads, 0);
    case CE_KERNEL_BINOMIAL:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_persistent<BinomialTile>, kBlockThreads, 0);
    case CE_KERNEL_RUNTIME:
      if (!a.rt_fn_persistent) return hipErrorInvalidValue;
      return hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (hipFunction_t)a.rt_fn_persistent,
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
    case CE_KERNEL_NBODY_STEP:
      if (a.strict)
        hipLaunchKernelGGL(k_persistent<NbodyStepTile<true>>, g, b, 0, st, make_nbody_step<true>(a), s);
      else
        hipLaunchKernelGGL(k_persistent<NbodyStepTile<false>>, g, b, 0, st, make_nbody_step<false>(a), s);
      break;
    case CE_KERNEL_BINOMIAL: hipLaunchKernelGGL(k_persistent<BinomialTile>, g, b, 0, st, make_binomial(a), s); break;
    case CE_KERNEL_RUNTIME: {
      if (!a.rt_fn_persistent) return hipErrorInvalidValue;
      RtTile pay = make_rt(a);
      SchedArgs sa = s;
      void* params[] = {&pay, &sa};
      return hipModuleLaunchKernel((hipFunction_t)a.rt_fn_persistent, grid, 1, 1, kBlockThreads, 1, 1, 0, st, params,
                                   nullptr);
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_direct(const KernelArgs& a, const DirectArgs& d, uint32_t grid, hipStream_t st) {
  const dim3 g(grid), b(kBlockThreads);
  switch (a.kernel_id) {
    case CE_KERNEL_ESCAPE: hipLaunchKernelGGL(k_direct<EscapeTile>, g, b, 0, st, make_escape(a), d); break;
    case CE_KERNEL_BLUR5: hipLaunchKernelGGL(k_direct<Blur5Tile>, g, b, 0, st, make_blur(a), d); break;
    case CE_KERNEL_NBODY_ACC:
      if (a.strict)
        hipLaunchKernelGGL(k_direct<NbodyTile<true>>, g, b, 0, st, make_nbody<true>(a), d);
      else
        hipLaunchKernelGGL(k_direct<NbodyTile<false>>, g, b, 0, st, make_nbody<false>(a), d);
      break;
    case CE_KERNEL_NBODY_STEP:
      if (a.strict)
        hipLaunchKernelGGL(k_direct<NbodyStepTile<true>>, g, b, 0, st, make_nbody_step<true>(a), d);
      else
        hipLaunchKernelGGL(k_direct<NbodyStepTile<false>>, g, b, 0, st, make_nbody_step<false>(a), d);
      break;
    case CE_KERNEL_BINOMIAL: hipLaunchKernelGGL(k_direct<BinomialTile>, g, b, 0, st, make_binomial(a), d); break;
    case CE_KERNEL_RUNTIME: {
      if (!a.rt_fn_direct) return hipErrorInvalidValue;
      RtTile pay = make_rt(a);
      DirectArgs da = d;
      void* params[] = {&pay, &da};
      return hipModuleLaunchKernel((hipFunction_t)a.rt_fn_direct, grid, 1, 1, kBlockThreads, 1, 1, 0, st, params,
                                   nullptr);
    }
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
    case CE_KERNEL_NBODY_STEP:
      if (a.strict)
        hipLaunchKernelGGL(k_bare<NbodyStepTile<true>>, g, b, 0, st, make_nbody_step<true>(a), G);
      else
        hipLaunchKernelGGL(k_bare<NbodyStepTile<false>>, g, b, 0, st, make_nbody_step<false>(a), G);
      break;
    case CE_KERNEL_BINOMIAL: hipLaunchKernelGGL(k_bare<BinomialTile>, g, b, 0, st, make_binomial(a), G); break;
    case CE_KERNEL_RUNTIME: {
      if (!a.rt_fn_bare) return hipErrorInvalidValue;
      RtTile pay = make_rt(a);
      uint64_t g_arg = G;
      void* params[] = {&pay, &g_arg};
      return hipModuleLaunchKernel((hipFunction_t)a.rt_fn_bare, tiles, 1, 1, kBlockThreads, 1, 1, 0, st, params,
                                   nullptr);
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Streaming copy, the achievable-bandwidth reference for the HBM-bound
// payloads: one 16-byte non-temporal load and store per thread, one
// workgroup per 4 KiB (the fastest of the shapes measured on this GPU:
// 1, 2, 4 or 8 vectors per thread, temporal or not, one-shot or grid-stride).
__global__ __launch_bounds__(kBlockThreads) void k_stream_copy(f32x4* __restrict__ dst, const f32x4* __restrict__ src,
                                                               uint64_t n16) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlockThreads + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(void* dst, const void* src, uint64_t n16, hipStream_t st) {
  if (n16 == 0) return hipSuccess;
  const uint64_t blocks = (n16 + kBlockThreads - 1) / kBlockThreads;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream_copy, dim3((uint32_t)blocks), dim3(kBlockThreads), 0, st, (f32x4*)dst,
                     (const f32x4*)src, n16);
  return hipGetLastError();
}

hipError_t launch_calibrate(L1State* l1, uint32_t rounds, uint64_t spin_limit, hipStream_t st) {
  hipLaunchKernelGGL(k_calibrate, dim3(1), dim3(64), 0, st, l1, rounds, spin_limit);
  return hipGetLastError();
}

}  // namespace ce
