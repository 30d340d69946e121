// Tile of a payload supplied as source at run time. The host engine builds
// it (kernels.hip) and the runtime-compiled module runs it: both see this one
// definition, so its layout and its tile cut agree. A tile is a run of
// kRtTileItems consecutive work-items of one package; the workgroup's
// threads take them in turn and call the caller's work-item function.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/coexec.h"
#include "common.hpp"

namespace ce {

constexpr uint32_t kRtTileItems = 8 * kBlockThreads;

struct RtTile {
  static constexpr int kMinBlocksPerCu = 1;
  ce_rt_args args;  // device pointers and scalars
  uint64_t items;   // work-items of the index space
  uint64_t lws;     // work-items per granule
  CE_HD uint64_t granules() const { return (items + lws - 1) / lws; }
  CE_HD uint64_t item_at(uint64_t g) const { return g * lws < items ? g * lws : items; }
  CE_HD uint32_t ntiles(uint64_t g0, uint64_t g1) const {
    return (uint32_t)((item_at(g1) - item_at(g0) + kRtTileItems - 1) / kRtTileItems);
  }
#ifdef CE_RT_ENTRY
  __device__ void load_constants() {}
  __device__ void run(uint64_t g0, uint64_t g1, uint32_t t) const {
    const uint64_t i0 = item_at(g0) + (uint64_t)t * kRtTileItems;
    const uint64_t end = item_at(g1);
    const uint64_t i1 = i0 + kRtTileItems < end ? i0 + kRtTileItems : end;
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += kBlockThreads) CE_RT_ENTRY(i, &args);
  }
#endif
};

}  // namespace ce
