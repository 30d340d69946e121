// Batched form: many escape-time jobs of uneven sizes co-scheduled by one
// persistent kernel over the concatenation of their tiles.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "../../include/coexec.h"

namespace ce {

// One job of a batch, as the kernel reads it (64 bytes).
struct alignas(64) BatchJob {
  ce_escape_params p;   // 28 bytes
  uint32_t tiles_x;     // column blocks of this job
  uint64_t tile_base;   // first tile of this job in the concatenated space
  uint32_t* out;        // device output, h x w uint32
  uint64_t pad[2];
};

struct BatchArgs {
  const BatchJob* jobs;   // device table
  uint32_t n_jobs;
  uint32_t pkg_tiles;     // tiles claimed per workgroup request
  uint64_t total_tiles;
  uint64_t* counter;      // HBM: [0] next tile, [1] workgroups that left
};

// Tile shapes the autotuner chooses from (rows x columns, 256 pixels each).
constexpr int kBatchShapes = 5;
constexpr uint32_t kBatchShapeRows[kBatchShapes] = {1, 2, 4, 8, 16};
constexpr uint32_t kBatchMaxJobs = 4096;

uint32_t batch_shape_cols(int shape);
hipError_t batch_blocks_per_cu(int shape, size_t lds_bytes, int* blocks);
hipError_t launch_batch(int shape, const BatchArgs& a, uint32_t grid, hipStream_t st);

}  // namespace ce
