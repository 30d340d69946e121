// Internal interface between the host engine and the GPU kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "../../include/coexec.h"
#include "common.hpp"

namespace ce {

// Everything a payload kernel needs, by value.
struct KernelArgs {
  int32_t kernel_id;
  uint32_t strict;          // n-body: Lomont 1/sqrt (bitwise equal to the host)
  ce_escape_params esc;
  ce_blur5_params blur;
  ce_nbody_params nb;
  ce_nbody_step_params nbs;
  ce_binomial_params bin;
  const void* in0;          // device pointers
  const void* in1;
  void* out;
  void* out1;               // second output (n-body step: velocities)
};

// Granules of the index space and tiles of a package, as the GPU cuts them.
uint64_t gpu_granules(const KernelArgs& a);
uint32_t gpu_tiles(const KernelArgs& a, uint64_t g0, uint64_t g1);

// Resident workgroups per CU of the persistent kernel for this payload.
hipError_t persistent_blocks_per_cu(const KernelArgs& a, int* blocks);
hipError_t launch_persistent(const KernelArgs& a, const SchedArgs& s, uint32_t grid, hipStream_t st);
hipError_t launch_bare(const KernelArgs& a, hipStream_t st);
// Clock calibration: one thread answers `rounds` pings through the mailbox.
hipError_t launch_calibrate(L1State* l1, uint32_t rounds, uint64_t spin_limit, hipStream_t st);

}  // namespace ce
