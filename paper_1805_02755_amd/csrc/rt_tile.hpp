// Tile of a payload supplied as source at run time. The host engine builds
// it (kernels.hip) and the runtime-compiled module runs it: both see this one
// definition, so its layout and its tile cut agree. A tile is a run of
// `tile` consecutive work-items of one package (a multiple of the workgroup
// size, chosen by the host); the workgroup's threads take them in turn and
// call the caller's work-item function.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/coexec.h"
#include "common.hpp"

namespace ce {

// Tile length for a space of `items` work-items: four items per thread, and
// eight from 16M items on, where a space still has 8192 tiles. On the
// 1024x1024 escape-time example, tiles of 512, 1024 and 2048 items gave
// 12.9e9, 13.1e9 and 8.9e9 co-executed items/s: shorter tiles spend more
// of their time in the dispenser, longer ones leave too few tiles to
// balance work-items of uneven cost.
CE_HD uint64_t rt_tile_items(uint64_t items) {
  return (uint64_t)kBlockThreads * (items >= (1ull << 24) ? 8u : 4u);
}

struct RtTile {
  static constexpr int kMinBlocksPerCu = 1;
  ce_rt_args args;  // device pointers and scalars
  uint64_t items;   // work-items of the index space
  uint64_t lws;     // work-items per granule
  uint64_t tile;    // work-items per tile (rt_tile_items)
  CE_HD uint64_t granules() const { return (items + lws - 1) / lws; }
  CE_HD uint64_t item_at(uint64_t g) const { return g * lws < items ? g * lws : items; }
  CE_HD uint32_t ntiles(uint64_t g0, uint64_t g1) const {
    return (uint32_t)((item_at(g1) - item_at(g0) + tile - 1) / tile);
  }
#ifdef CE_RT_ENTRY
  __device__ void load_constants() {}
  __device__ void run(uint64_t g0, uint64_t g1, uint32_t t) const {
    const uint64_t i0 = item_at(g0) + (uint64_t)t * tile;
    const uint64_t end = item_at(g1);
    const uint64_t i1 = i0 + tile < end ? i0 + tile : end;
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += kBlockThreads) CE_RT_ENTRY(i, &args);
  }
#endif
};

}  // namespace ce
