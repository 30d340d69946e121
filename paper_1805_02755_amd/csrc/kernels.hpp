// Internal interface between the host engine and the GPU kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <string>

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
  // payload supplied at run time: device arguments, index space and the
  // loaded module's kernels (hipFunction_t)
  ce_rt_args rt;
  uint64_t rt_items;
  uint64_t rt_lws;
  uint32_t rt_item_bytes;
  void* rt_fn_persistent;
  void* rt_fn_bare;
  void* rt_fn_direct;
};

// Granules of the index space and tiles of a package, as the GPU cuts them.
uint64_t gpu_granules(const KernelArgs& a);
uint32_t gpu_tiles(const KernelArgs& a, uint64_t g0, uint64_t g1);

// Resident workgroups per CU of the persistent kernel for this payload.
hipError_t persistent_blocks_per_cu(const KernelArgs& a, int* blocks);
hipError_t launch_persistent(const KernelArgs& a, const SchedArgs& s, uint32_t grid, hipStream_t st);
hipError_t launch_direct(const KernelArgs& a, const DirectArgs& d, uint32_t grid, hipStream_t st);
hipError_t launch_bare(const KernelArgs& a, hipStream_t st);
// Runtime payloads (rt_module.cpp): compile the caller's work-item source
// for gfx950 (no GPU needed), and compile and load it on the current device.
// 0 on success; otherwise negative with the compiler's log.
int rt_compile(const char* source, const char* entry, std::string* code, std::string* lowered_persistent,
               std::string* lowered_bare, std::string* lowered_direct, std::string* log);
int rt_build(const char* source, const char* entry, void** module, void** fn_persistent, void** fn_bare,
             void** fn_direct, std::string* log);
void rt_release(void* module);
// Allocation-free runs (noalloc.hip): the address of this device's static
// scratch array (kNoallocScratchBytes), looked up once per device; and a
// zero fill of n 64-bit words on a stream.
hipError_t noalloc_scratch_address(int device, void** out);
hipError_t launch_zero_words(void* p, uint64_t n_words, hipStream_t st);
// Streaming copy of n16 16-byte vectors (the bandwidth reference).
hipError_t launch_stream_copy(void* dst, const void* src, uint64_t n16, hipStream_t st);
// Clock calibration: one thread answers `rounds` pings through the mailbox.
hipError_t launch_calibrate(L1State* l1, uint32_t rounds, uint64_t spin_limit, hipStream_t st);

}  // namespace ce
