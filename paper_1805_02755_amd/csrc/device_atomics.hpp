// Clock and atomic helpers for the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ce {

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
}  // namespace ce
