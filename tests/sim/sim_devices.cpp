// Fake devices for CPU tests of the host engine (engine.cpp).
//
// The real engine is compiled against a stub HIP runtime in which:
//  - device memory is host memory;
//  - the "GPU" persistent kernel is one CPU thread that claims packages from
//    the same level-1 dispenser with the same rules as the device code
//    (Static bands, Dynamic fetch-add, HGuided compare-and-swap) and fills
//    the GPU package table, the summary and the completion run id;
//  - payloads do no arithmetic: every work-item's first output word is set
//    to the item's index (so the output merges can be checked), a per-run
//    coverage counter of the item is incremented, and the worker spins for
//    a configurable time per item, so device speeds are set by the test.
// Nothing here is part of the product library.
#include <hip/hip_runtime_api.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <thread>
#include <vector>

#include "../../paper_1805_02755_amd/csrc/host_payloads.hpp"
#include "../../paper_1805_02755_amd/csrc/kernels.hpp"

namespace {
std::thread g_gpu;
double g_gpu_ns_per_item = 1.0;
double g_host_ns_per_item = 10.0;
double g_gpu_claim_ns = 1000.0;
// faults: the fake GPU's first claim waits this long, then gives up as the
// kernel's bounded dispenser wait does (0: no stall); the runtime payload's
// host version fails on the tile holding this item (~0: never)
double g_gpu_stall_ms = 0.0;
uint64_t g_host_fail_item = ~0ull;
std::atomic<uint32_t>* g_cov = nullptr;
size_t g_cov_n = 0;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
void spin_until(int64_t until) {
  while (now_ns() < until) {
  }
}
void join_gpu() {
  if (g_gpu.joinable()) g_gpu.join();
}
}  // namespace

extern "C" void sim_reset(size_t n_items) {
  delete[] g_cov;
  g_cov = new std::atomic<uint32_t>[n_items];
  for (size_t i = 0; i < n_items; ++i) g_cov[i].store(0);
  g_cov_n = n_items;
}

extern "C" void sim_coverage(uint32_t* dst, size_t n) {
  for (size_t i = 0; i < n && i < g_cov_n; ++i) dst[i] = g_cov[i].load();
}

extern "C" void sim_set_faults(double gpu_stall_ms, uint64_t host_fail_item) {
  g_gpu_stall_ms = gpu_stall_ms;
  g_host_fail_item = host_fail_item;
}

extern "C" void sim_set_rates(double gpu_ns_per_item, double host_ns_per_item, double gpu_claim_ns) {
  g_gpu_ns_per_item = gpu_ns_per_item;
  g_host_ns_per_item = host_ns_per_item;
  g_gpu_claim_ns = gpu_claim_ns;
}

// ------------------------------------------------------------- HIP stubs
hipError_t hipGetDeviceCount(int* c) { *c = 1; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  strcpy(p->gcnArchName, "gfx950:sim");
  p->multiProcessorCount = 8;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 100000; return hipSuccess; }
// Streams are distinct tokens; the simulated GPU thread belongs to the stream
// its kernel was launched on, and only work on that stream waits for it.
static std::atomic<uintptr_t> g_next_stream{1};
static std::atomic<uintptr_t> g_gpu_stream{0};
static bool on_gpu_stream(hipStream_t s) { return (uintptr_t)s == 0 || (uintptr_t)s == g_gpu_stream.load(); }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (hipStream_t)g_next_stream.fetch_add(1); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (on_gpu_stream(s)) join_gpu();
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) { *p = calloc(1, n ? n : 1); return *p ? hipSuccess : 2; }
hipError_t hipFree(void* p) { free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { *p = calloc(1, n ? n : 1); return *p ? hipSuccess : 2; }
hipError_t hipHostFree(void* p) { free(p); return hipSuccess; }
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned) { *d = h; return hipSuccess; }
hipError_t hipMemset(void* p, int v, size_t n) { memset(p, v, n); return hipSuccess; }
hipError_t hipDeviceSynchronize() {
  join_gpu();
  return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { join_gpu(); memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t st) {
  if (on_gpu_stream(st)) join_gpu();  // stream order: after the kernel
  memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
// copies are synchronous here, so events are complete as soon as recorded
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = reinterpret_cast<hipEvent_t>(new char[1]);
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete[] reinterpret_cast<char*>(e);
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "sim"; }
hipError_t hipGetLastError() { return hipSuccess; }

// Memory a test marked as pinned (sim_pin) is "host memory" to the engine;
// everything else is pageable.
namespace {
std::mutex g_pin_mu;
std::vector<std::pair<uintptr_t, size_t>> g_pinned;
}  // namespace
extern "C" void sim_pin(void* p, size_t n) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pinned.emplace_back((uintptr_t)p, n);
}
extern "C" void sim_unpin_all() {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pinned.clear();
}
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  for (auto& r : g_pinned) {
    if ((uintptr_t)p >= r.first && (uintptr_t)p < r.first + r.second) {
      a->type = hipMemoryTypeHost;
      a->devicePointer = a->hostPointer = const_cast<void*>(p);
      return hipSuccess;
    }
  }
  return hipErrorInvalidValue;
}

namespace ce {

// ------------------------------------------------ coverage-marking payloads
namespace {
size_t item_words(const KernelArgs& a) {
  if (a.kernel_id == CE_KERNEL_RUNTIME) return a.rt_item_bytes / 4;
  const int kernel_id = a.kernel_id;
  return (kernel_id == CE_KERNEL_NBODY_ACC || kernel_id == CE_KERNEL_NBODY_STEP || kernel_id == CE_KERNEL_BINOMIAL)
             ? 4
             : 1;
}
uint32_t bodies_of(const KernelArgs& a) { return a.kernel_id == CE_KERNEL_NBODY_STEP ? a.nbs.n : a.nb.n; }
// the second output of the step payload gets the same item indices, uncounted
void mark_second(uint32_t* out1, uint64_t i0, uint64_t i1) {
  if (!out1) return;
  for (uint64_t i = i0; i < i1; ++i) out1[i * 4] = (uint32_t)i;
}
void mark(uint32_t* out, uint64_t i0, uint64_t i1, size_t words) {
  for (uint64_t i = i0; i < i1; ++i) {
    out[i * words] = (uint32_t)i;
    if (i < g_cov_n) g_cov[i].fetch_add(1, std::memory_order_relaxed);
  }
}
// Each call takes ns_per_item per item in total, marking included.
void h_escape(const ce_escape_params& p, uint64_t r0, uint64_t r1, uint32_t* out) {
  const int64_t until = now_ns() + (int64_t)(g_host_ns_per_item * (double)((r1 - r0) * p.w));
  mark(out, r0 * p.w, r1 * p.w, 1);
  spin_until(until);
}
void h_blur(const float*, uint32_t w, uint32_t, const float*, uint64_t r0, uint64_t r1, float* out) {
  const int64_t until = now_ns() + (int64_t)(g_host_ns_per_item * (double)((r1 - r0) * w));
  mark((uint32_t*)out, r0 * w, r1 * w, 1);
  spin_until(until);
}
void h_nbody(const float*, uint32_t, float, int, uint64_t i0, uint64_t i1, float* out4) {
  const int64_t until = now_ns() + (int64_t)(g_host_ns_per_item * (double)(i1 - i0));
  mark((uint32_t*)out4, i0, i1, 4);
  spin_until(until);
}
const HostPayloadFns kSim = {h_escape, h_blur, h_nbody, "sim"};

uint64_t rt_item(const KernelArgs& a, uint64_t g) { return std::min<uint64_t>(g * a.rt_lws, a.rt_items); }
uint64_t items_of(const KernelArgs& a, uint64_t g0, uint64_t g1) {
  if (a.kernel_id == CE_KERNEL_RUNTIME) return rt_item(a, g1) - rt_item(a, g0);
  if (a.kernel_id == CE_KERNEL_BINOMIAL) return g1 - g0;  // one output element per option group
  if (a.kernel_id == CE_KERNEL_ESCAPE) return (g1 - g0) * a.esc.w;
  if (a.kernel_id == CE_KERNEL_BLUR5) return (g1 - g0) * a.blur.w;
  const uint64_t lo = g0 * 256, hi = std::min<uint64_t>(g1 * 256, bodies_of(a));
  return hi > lo ? hi - lo : 0;
}
uint64_t first_item(const KernelArgs& a, uint64_t g) {
  if (a.kernel_id == CE_KERNEL_RUNTIME) return rt_item(a, g);
  if (a.kernel_id == CE_KERNEL_BINOMIAL) return g;
  if (a.kernel_id == CE_KERNEL_ESCAPE) return g * a.esc.w;
  if (a.kernel_id == CE_KERNEL_BLUR5) return g * a.blur.w;
  return std::min<uint64_t>(g * 256, bodies_of(a));
}
}  // namespace

const HostPayloadFns* host_payloads() { return &kSim; }

// Host version of a simulated runtime payload: scalars[0] is the index of
// the output buffer, scalars[1] its 32-bit words per work-item.
extern "C" int32_t sim_rt_host(uint64_t i0, uint64_t i1, const ce_rt_args* a) {
  // 2^63: every call fails
  if ((g_host_fail_item >= i0 && g_host_fail_item < i1) || g_host_fail_item == (1ull << 63)) return 42;
  const int64_t until = now_ns() + (int64_t)(g_host_ns_per_item * (double)(i1 - i0));
  mark((uint32_t*)a->buf[a->scalars[0]], i0, i1, a->scalars[1]);
  spin_until(until);
  return 0;
}

// The step's update after the (coverage-counting) force payload: the
// position output gets the same item indices.
// Binomial groups: one coverage mark per output element.
void binomial_groups(const float*, const float*, uint32_t, float, float, float, uint64_t g0, uint64_t g1,
                     float* out4) {
  const int64_t until = now_ns() + (int64_t)(g_host_ns_per_item * (double)(g1 - g0));
  mark((uint32_t*)out4, g0, g1, 4);
  spin_until(until);
}

void nbody_step_update(const float*, const float*, float, uint64_t i0, uint64_t i1, float* pos_out4, float* vel_out4) {
  uint32_t* po = (uint32_t*)pos_out4;
  const uint32_t* vo = (const uint32_t*)vel_out4;
  for (uint64_t i = i0; i < i1; ++i) po[i * 4] = vo[i * 4];
}

// ------------------------------------------------------ fake GPU kernels
uint64_t gpu_granules(const KernelArgs& a) {
  if (a.kernel_id == CE_KERNEL_RUNTIME) return (a.rt_items + a.rt_lws - 1) / a.rt_lws;
  if (a.kernel_id == CE_KERNEL_ESCAPE) return a.esc.h;
  if (a.kernel_id == CE_KERNEL_BLUR5) return a.blur.h;
  if (a.kernel_id == CE_KERNEL_BINOMIAL) return a.bin.n_groups;
  return (bodies_of(a) + 255) / 256;
}
uint32_t gpu_tiles(const KernelArgs& a, uint64_t g0, uint64_t g1) {
  if (a.kernel_id == CE_KERNEL_RUNTIME) return (uint32_t)ceil_div(items_of(a, g0, g1), 2048);
  if (a.kernel_id == CE_KERNEL_ESCAPE) return (uint32_t)(ceil_div(g1 - g0, kEscapeTileRows) * ceil_div(a.esc.w, kEscapeTileCols));
  if (a.kernel_id == CE_KERNEL_BLUR5) return (uint32_t)(ceil_div(g1 - g0, kBlurTileRows) * ceil_div(a.blur.w, kBlurTileCols));
  return (uint32_t)(g1 - g0);
}
hipError_t persistent_blocks_per_cu(const KernelArgs&, int* b) {
  *b = 2;
  return hipSuccess;
}

hipError_t launch_persistent(const KernelArgs& a, const SchedArgs& s, uint32_t, hipStream_t st) {
  join_gpu();
  g_gpu_stream.store((uintptr_t)st);
  g_gpu = std::thread([a, s] {
    // the next run's queue state, cleared as the real kernel clears it
    if (s.l2_next) {
      memset(s.l2_next, 0, sizeof(L2State));
      memset(s.pub_next, 0, (size_t)s.pub_next_words * sizeof(uint64_t));
    }
    uint64_t np = 0, gr = 0, stn = s.st_first, t_first = 0, t_last = 0;
    bool pre = s.pre_nt != 0;  // the package the host claimed for the GPU before the launch
    for (;;) {
      uint64_t g0 = 0, g1 = 0;
      spin_until(now_ns() + (int64_t)g_gpu_claim_ns);
      if (!pre && g_gpu_stall_ms > 0.0) {
        // a claim that never comes back: the bounded wait runs out and the
        // GPU's part ends after the package it already had, flagged
        spin_until(now_ns() + (int64_t)(g_gpu_stall_ms * 1e6));
        __atomic_store_n(&s.l1->gpu_flags, 1, __ATOMIC_RELEASE);
        break;
      }
      if (pre) {
        g0 = s.pre_g0;
        g1 = s.pre_g1;
        pre = false;
      } else if (s.kind == kStatic) {
        if (s.st_nbands == 0) {
          if (stn || s.st_begin >= s.st_end) break;
          g0 = s.st_begin;
          g1 = s.st_end;
        } else {
          const uint64_t b = s.st_begin + stn;
          if (b >= s.st_end) break;
          g0 = band_edge(b, s.G, s.st_nbands);
          g1 = band_edge(b + 1, s.G, s.st_nbands);
        }
        ++stn;
      } else if (s.kind == kDynamic) {
        const uint64_t x = __atomic_fetch_add(&s.l1->next, s.pkg, __ATOMIC_RELAXED);
        if (x >= s.G) break;
        g0 = x;
        g1 = std::min(x + s.pkg, s.G);
      } else {
        uint64_t cur = __atomic_load_n(&s.l1->next, __ATOMIC_ACQUIRE);
        bool ok = false;
        while (cur < s.G) {
          const uint64_t sz = hguided_size(s.G - cur, s.P_self, s.sumP, s.n_dev, s.k, s.min_self);
          if (__atomic_compare_exchange_n(&s.l1->next, &cur, cur + sz, false, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE)) {
            ok = true;
            g0 = cur;
            g1 = cur + sz;
            break;
          }
        }
        if (!ok) break;
      }
      if (np >= s.max_pkgs) {
        __atomic_store_n(&s.l1->gpu_flags, 1, __ATOMIC_RELEASE);
        break;
      }
      const uint64_t tc = (uint64_t)(now_ns() / 10);
      if (!np) {
        t_first = tc;
        __atomic_store_n(&s.l1->gpu_t_first, t_first, __ATOMIC_RELEASE);  // the start, as a workgroup stamps it
      }
      const uint64_t n = items_of(a, g0, g1);
      const int64_t until = now_ns() + (int64_t)(g_gpu_ns_per_item * (double)n);
      mark((uint32_t*)a.out, first_item(a, g0), first_item(a, g0) + n, item_words(a));
      mark_second((uint32_t*)a.out1, first_item(a, g0), first_item(a, g0) + n);
      spin_until(until);
      PkgSlot& ps = s.pkgs[np];
      ps.g0 = g0;
      ps.g1 = g1;
      ps.base = 0;
      ps.ntiles = 1;
      ps.tiles_done = 1;
      ps.t_claim = tc;
      ps.t_end = t_last = (uint64_t)(now_ns() / 10);
      ++np;
      gr += g1 - g0;
    }
    // gather: copy the host's finished tiles into the device output
    if (s.gather_wgs) {
      const uint64_t want = host_final_word(s.run_id, 0) >> 40;
      for (uint64_t j = 0;; ++j) {
        uint64_t w = 0;
        const int64_t t0 = now_ns();
        for (;;) {
          if (j < s.ring_cap) w = __atomic_load_n(&s.ring[j], __ATOMIC_ACQUIRE);
          if (w) break;
          const uint64_t f = __atomic_load_n(&s.l1->host_final, __ATOMIC_ACQUIRE);
          if ((f >> 40) == want && j >= (f & ((1ull << 40) - 1))) break;
          if (now_ns() - t0 > 10000000000LL) {
            __atomic_store_n(&s.l1->gpu_flags, 2, __ATOMIC_RELEASE);
            break;
          }
        }
        if (!w) break;
        memcpy(s.gdst + ring_off(w), s.gsrc + ring_off(w), ring_len(w));
        __atomic_fetch_add(&s.l1->gathered, ring_len(w), __ATOMIC_RELEASE);
        __atomic_store_n(&s.l1->gpu_t_gather, (uint64_t)(now_ns() / 10), __ATOMIC_RELEASE);
      }
    }
    __atomic_store_n(&s.l1->gpu_t_first, t_first, __ATOMIC_RELEASE);
    __atomic_store_n(&s.l1->gpu_t_last, t_last, __ATOMIC_RELEASE);
    __atomic_store_n(&s.l1->gpu_granules, gr, __ATOMIC_RELEASE);
    __atomic_store_n(&s.l1->gpu_packages, np, __ATOMIC_RELEASE);
    if (s.wg_end) {
      // light exit: one workgroup's end; the packages the kernel claimed
      // (beyond the one claimed before the launch) in its queue state
      __atomic_store_n(&s.wg_end[0], t_last, __ATOMIC_RELEASE);
      const uint64_t pre = s.pre_nt ? 1 : 0;
      s.l2->n_pkgs = (uint32_t)(np - std::min(np, pre));
      s.l2->granules = gr - (np && pre ? s.pre_g1 - s.pre_g0 : 0);
      s.l2->t_first = t_first;
    }
    __atomic_store_n(&s.l1->gpu_done, done_word(s.run_id, (uint64_t)(now_ns() / 10)), __ATOMIC_RELEASE);
  });
  return hipSuccess;
}

// the allocation-free run's static scratch: a static host array here
alignas(256) static unsigned char g_noalloc_scratch[kNoallocScratchBytes];
hipError_t noalloc_scratch_address(int, void** out) {
  *out = g_noalloc_scratch;
  return hipSuccess;
}
hipError_t launch_zero_words(void* p, uint64_t n_words, hipStream_t) {
  join_gpu();
  memset(p, 0, n_words * sizeof(uint64_t));
  return hipSuccess;
}

hipError_t launch_stream_copy(void* dst, const void* src, uint64_t n16, hipStream_t) {
  memcpy(dst, src, n16 * 16);
  return hipSuccess;
}

// The direct kernel: the one package claimed before the launch, then each
// workgroup's end tick (one workgroup here).
hipError_t launch_direct(const KernelArgs& a, const DirectArgs& d, uint32_t, hipStream_t st) {
  join_gpu();
  g_gpu_stream.store((uintptr_t)st);
  g_gpu = std::thread([a, d] {
    spin_until(now_ns() + (int64_t)g_gpu_claim_ns);
    const uint64_t tc = (uint64_t)(now_ns() / 10);
    __atomic_store_n(&d.l1->gpu_t_first, tc, __ATOMIC_RELEASE);
    const uint64_t n = items_of(a, d.g0, d.g1);
    const int64_t until = now_ns() + (int64_t)(g_gpu_ns_per_item * (double)n);
    mark((uint32_t*)a.out, first_item(a, d.g0), first_item(a, d.g0) + n, item_words(a));
    mark_second((uint32_t*)a.out1, first_item(a, d.g0), first_item(a, d.g0) + n);
    spin_until(until);
    d.pkgs[0].t_claim = tc;
    __atomic_store_n(&d.wg_end[0], (uint64_t)(now_ns() / 10), __ATOMIC_RELEASE);
  });
  return hipSuccess;
}

hipError_t launch_bare(const KernelArgs& a, hipStream_t) {
  const uint64_t G = gpu_granules(a);
  mark((uint32_t*)a.out, 0, items_of(a, 0, G), item_words(a));
  mark_second((uint32_t*)a.out1, 0, items_of(a, 0, G));
  return hipSuccess;
}

// Runtime payloads: the stand-in "compiler" accepts a source that names its
// entry; the simulated GPU marks coverage like the fixed payloads.
int rt_compile(const char* source, const char* entry, std::string* code, std::string* lp, std::string* lb,
               std::string* ld, std::string* log) {
  if (!source || !entry || !*entry || !strstr(source, entry)) {
    *log = "payload.hip: error: entry not found (simulated compiler)";
    return -1;
  }
  *code = "sim";
  *lp = *lb = *ld = entry;
  return 0;
}
int rt_build(const char* source, const char* entry, void** module, void** fn_persistent, void** fn_bare,
             void** fn_direct, std::string* log) {
  std::string c, a, b, d;
  const int rc = rt_compile(source, entry, &c, &a, &b, &d, log);
  if (rc != 0) return rc;
  *module = *fn_persistent = *fn_bare = *fn_direct = (void*)1;
  return 0;
}
void rt_release(void*) {}

hipError_t launch_calibrate(L1State* l1, uint32_t rounds, uint64_t, hipStream_t st) {
  join_gpu();
  g_gpu_stream.store((uintptr_t)st);
  g_gpu = std::thread([l1, rounds] {
    for (uint32_t i = 1; i <= rounds; ++i) {
      const int64_t t0 = now_ns();
      while (__atomic_load_n(&l1->ping, __ATOMIC_ACQUIRE) != i)
        if (now_ns() - t0 > 1000000000LL) return;
      __atomic_store_n(&l1->tick, (uint64_t)(now_ns() / 10), __ATOMIC_RELEASE);
      __atomic_store_n(&l1->pong, i, __ATOMIC_RELEASE);
    }
  });
  return hipSuccess;
}

}  // namespace ce
