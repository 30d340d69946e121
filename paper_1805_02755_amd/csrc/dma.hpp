// Host -> device copies on the GPU's system DMA (SDMA) engines, issued
// through the HSA runtime so that several engines work on one copy at once
// and no copy needs a compute unit (a persistent kernel holds all of them).
// The engine uses this for the host's share of a device-resident output.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace ce {

class SdmaCopier {
 public:
  SdmaCopier() = default;
  ~SdmaCopier();
  SdmaCopier(const SdmaCopier&) = delete;
  SdmaCopier& operator=(const SdmaCopier&) = delete;

  // Finds the HSA agents of HIP device `hip_device` (by PCI location) and its
  // host -> device copy engines. Returns false, with a reason in `why`, if
  // there is no such engine; the copier is then unusable.
  bool init(int hip_device, char* why, size_t why_len);
  bool ready() const { return n_engines_ > 0; }
  uint32_t engines() const { return n_engines_; }

  // Starts copying n bytes from pinned host memory to device memory, split
  // over the engines. Returns a handle >= 0, or -1 if the copy could not be
  // queued. Not thread-safe: the caller serialises start/poll/wait/release.
  int start(void* dst, const void* src, size_t n);
  // 1: the copy is complete (its bytes are in device memory), 0: pending.
  int poll(int h) const;
  // Waits for completion up to timeout_ns; true when complete.
  bool wait(int h, uint64_t timeout_ns) const;
  // Returns a completed handle for reuse.
  void release(int h);

 private:
  static constexpr uint32_t kMaxEngines = 4;
  static constexpr uint32_t kSlots = 256;
  uint64_t gpu_ = 0, cpu_ = 0;          // hsa_agent_t handles
  uint32_t engine_ids_[kMaxEngines] = {};
  uint32_t n_engines_ = 0;
  uint32_t next_engine_ = 0;
  uint64_t signals_[kSlots] = {};       // hsa_signal_t handles (0: not created)
  uint32_t free_[kSlots] = {};
  uint32_t n_free_ = 0;
  bool hsa_up_ = false;
};

}  // namespace ce
