// SDMA copier on the HSA runtime (see dma.hpp).
#include "dma.hpp"

#include <hip/hip_runtime_api.h>
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>
#include <stdio.h>

namespace ce {

namespace {

struct AgentSearch {
  uint32_t want_bdf;
  hsa_agent_t gpu{}, cpu{};
  bool have_gpu = false, have_cpu = false;
};

hsa_status_t visit_agent(hsa_agent_t a, void* data) {
  AgentSearch* s = static_cast<AgentSearch*>(data);
  hsa_device_type_t t;
  if (hsa_agent_get_info(a, HSA_AGENT_INFO_DEVICE, &t) != HSA_STATUS_SUCCESS) return HSA_STATUS_SUCCESS;
  if (t == HSA_DEVICE_TYPE_CPU && !s->have_cpu) {
    s->cpu = a;
    s->have_cpu = true;
  } else if (t == HSA_DEVICE_TYPE_GPU && !s->have_gpu) {
    uint32_t bdf = 0;
    if (hsa_agent_get_info(a, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_BDFID, &bdf) == HSA_STATUS_SUCCESS &&
        bdf == s->want_bdf) {
      s->gpu = a;
      s->have_gpu = true;
    }
  }
  return HSA_STATUS_SUCCESS;
}

}  // namespace

bool SdmaCopier::init(int hip_device, char* why, size_t why_len) {
  int bus = 0, dev = 0;
  if (hipDeviceGetAttribute(&bus, hipDeviceAttributePciBusId, hip_device) != hipSuccess ||
      hipDeviceGetAttribute(&dev, hipDeviceAttributePciDeviceId, hip_device) != hipSuccess) {
    snprintf(why, why_len, "no PCI location for device %d", hip_device);
    return false;
  }
  if (hsa_init() != HSA_STATUS_SUCCESS) {
    snprintf(why, why_len, "HSA runtime did not initialise");
    return false;
  }
  hsa_up_ = true;
  AgentSearch s;
  s.want_bdf = ((uint32_t)bus << 8) | ((uint32_t)dev << 3);
  if (hsa_iterate_agents(visit_agent, &s) != HSA_STATUS_SUCCESS || !s.have_gpu || !s.have_cpu) {
    snprintf(why, why_len, "no HSA agents for device %d", hip_device);
    return false;
  }
  uint32_t mask = 0;
  if (hsa_amd_memory_copy_engine_status(s.gpu, s.cpu, &mask) != HSA_STATUS_SUCCESS || mask == 0) {
    snprintf(why, why_len, "no host-to-device copy engine");
    return false;
  }
  gpu_ = s.gpu.handle;
  cpu_ = s.cpu.handle;
  for (uint32_t b = 0; b < 32 && n_engines_ < kMaxEngines; ++b)
    if (mask & (1u << b)) engine_ids_[n_engines_++] = 1u << b;
  for (uint32_t i = 0; i < kSlots; ++i) free_[i] = kSlots - 1 - i;
  n_free_ = kSlots;
  // The first copy on an engine sets up its queue and takes milliseconds:
  // pay that here, outside any run.
  void* hbuf = nullptr;
  void* dbuf = nullptr;
  bool pending = false;  // a test copy that did not finish keeps its buffers
  if (hipHostMalloc(&hbuf, 4096, hipHostMallocDefault) == hipSuccess && hipMalloc(&dbuf, 4096) == hipSuccess) {
    hsa_signal_t sg;
    if (hsa_signal_create(1, 0, nullptr, &sg) == HSA_STATUS_SUCCESS) {
      uint32_t usable = 0;
      for (uint32_t e = 0; e < n_engines_; ++e) {
        hsa_signal_store_screlease(sg, 1);
        if (hsa_amd_memory_async_copy_on_engine(dbuf, s.gpu, hbuf, s.cpu, 4096, 0, nullptr, sg,
                                                (hsa_amd_sdma_engine_id_t)engine_ids_[e], true) != HSA_STATUS_SUCCESS)
          continue;
        // bounded wait: the hint is in system-timestamp ticks, so re-check the value
        for (int i = 0; i < 20 && hsa_signal_load_scacquire(sg) > 0; ++i)
          hsa_signal_wait_scacquire(sg, HSA_SIGNAL_CONDITION_LT, 1, 100'000'000ull, HSA_WAIT_STATE_BLOCKED);
        if (hsa_signal_load_scacquire(sg) > 0) break;  // an engine that does not finish: leave the signal
        engine_ids_[usable++] = engine_ids_[e];
      }
      pending = hsa_signal_load_scacquire(sg) > 0;
      n_engines_ = usable;
      if (!pending) hsa_signal_destroy(sg);
    }
  }
  if (!pending) {
    if (dbuf) (void)hipFree(dbuf);
    if (hbuf) (void)hipHostFree(hbuf);
  }
  if (n_engines_ == 0) {
    snprintf(why, why_len, "no host-to-device copy engine completed a test copy");
    return false;
  }
  return true;
}

SdmaCopier::~SdmaCopier() {
  for (uint32_t i = 0; i < kSlots; ++i) {
    if (!signals_[i]) continue;
    hsa_signal_t sg{signals_[i]};
    // a copy still queued keeps its signal until it ends
    hsa_signal_wait_scacquire(sg, HSA_SIGNAL_CONDITION_LT, 1, 1'000'000'000ull, HSA_WAIT_STATE_BLOCKED);
    hsa_signal_destroy(sg);
  }
  if (hsa_up_) hsa_shut_down();
}

int SdmaCopier::start(void* dst, const void* src, size_t n) {
  if (!n_engines_ || !n_free_ || !n) return -1;
  const uint32_t h = free_[--n_free_];
  // pieces of at least 64 KiB, one per engine
  uint32_t pieces = (uint32_t)((n + (64u << 10) - 1) / (64u << 10));
  if (pieces > n_engines_) pieces = n_engines_;
  if (!signals_[h]) {
    hsa_signal_t sg;
    if (hsa_signal_create(1, 0, nullptr, &sg) != HSA_STATUS_SUCCESS) {
      free_[n_free_++] = h;
      return -1;
    }
    signals_[h] = sg.handle;
  }
  hsa_signal_t sg{signals_[h]};
  // every piece decrements the signal once it has landed
  hsa_signal_store_screlease(sg, pieces);
  const size_t step = ((n / pieces) + 255) & ~(size_t)255;
  size_t off = 0;
  for (uint32_t i = 0; i < pieces; ++i) {
    const size_t len = (i + 1 == pieces) ? n - off : step;
    const uint32_t e = engine_ids_[next_engine_++ % n_engines_];
    if (hsa_amd_memory_async_copy_on_engine(static_cast<char*>(dst) + off, hsa_agent_t{gpu_},
                                            static_cast<const char*>(src) + off, hsa_agent_t{cpu_}, len, 0, nullptr,
                                            sg, (hsa_amd_sdma_engine_id_t)e, true) != HSA_STATUS_SUCCESS) {
      // pieces already queued still decrement: account for the missing ones
      hsa_signal_subtract_screlease(sg, pieces - i);
      hsa_signal_wait_scacquire(sg, HSA_SIGNAL_CONDITION_LT, 1, 1'000'000'000ull, HSA_WAIT_STATE_BLOCKED);
      free_[n_free_++] = h;
      return -1;
    }
    off += len;
  }
  return (int)h;
}

int SdmaCopier::poll(int h) const {
  return hsa_signal_load_scacquire(hsa_signal_t{signals_[h]}) <= 0 ? 1 : 0;
}

bool SdmaCopier::wait(int h, uint64_t timeout_ns) const {
  const hsa_signal_t sg{signals_[h]};
  // the timeout of hsa_signal_wait is a hint in system-timestamp units; the
  // caller's deadline is enforced by re-checking the value
  uint64_t freq = 0;
  if (hsa_system_get_info(HSA_SYSTEM_INFO_TIMESTAMP_FREQUENCY, &freq) != HSA_STATUS_SUCCESS || !freq) freq = 1'000'000'000;
  const uint64_t hint = (uint64_t)((double)timeout_ns * (double)freq * 1e-9);
  hsa_signal_wait_scacquire(sg, HSA_SIGNAL_CONDITION_LT, 1, hint, HSA_WAIT_STATE_ACTIVE);
  return hsa_signal_load_scacquire(sg) <= 0;
}

void SdmaCopier::release(int h) {
  if (h >= 0 && (uint32_t)h < kSlots) free_[n_free_++] = (uint32_t)h;
}

}  // namespace ce
