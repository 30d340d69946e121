// Device scratch for the allocation-free run (ce_engine_run_noalloc): one
// statically sized array per GPU holds the level-2 queue state, the
// publication words and the package table that ce_engine_run keeps in
// memory the engine allocates. The array lives as long as the process.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace ce {

// Every run of the allocation-free entry point on a GPU uses this array, so
// two such runs that overlap on one GPU race on it.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxGpus = 64;
std::mutex g_mu;
void* g_addr[kMaxGpus] = {};
}  // namespace

hipError_t noalloc_scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxGpus) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[device]) {
    // the symbol has its own address on every device: look it up with that
    // device current, once
    int cur = 0;
    hipError_t he = hipGetDevice(&cur);
    if (he != hipSuccess) return he;
    if (cur != device && (he = hipSetDevice(device)) != hipSuccess) return he;
    void* p = nullptr;
    he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (he != hipSuccess) return he;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

// Zero fill of the queue state and the publication words before a run (a
// kernel rather than hipMemsetAsync, so the run may also be captured).
__global__ void k_zero_words(uint64_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t launch_zero_words(void* p, uint64_t n_words, hipStream_t st) {
  if (n_words == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(64, (n_words + 255) / 256);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, st, (uint64_t*)p, n_words);
  return hipGetLastError();
}

}  // namespace ce
