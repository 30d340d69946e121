// Host engine of the co-execution library and the C ABI (include/coexec.h).
//
// Architecture (section 4.2, section 5): the engine owns a device set (the
// GPU and a host worker pool), an index space cut into granules, a scheduler
// (section 5.3) and a program (kernel, buffers, output pattern). A run arms
// the shared level-1 dispenser in host-coherent memory, launches the GPU's
// persistent kernel and wakes the host pool; both sides claim packages from
// the same dispenser until the space is exhausted. Outputs are then merged so
// that every bound output pointer holds the full result.
#include <hip/hip_runtime_api.h>
#include <immintrin.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <exception>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/coexec.h"
#include "common.hpp"
#include "dma.hpp"
#include "host_payloads.hpp"
#include "kernels.hpp"

namespace ce {
namespace {

inline int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

inline void cpu_relax() { _mm_pause(); }

constexpr uint32_t kHostNbodyTile = 16;  // bodies per host tile
constexpr int kMaxSlots = 2;
// Bounds on the waits inside the GPU kernel: every kernel ends, so the host
// can wait for it with a plain stream synchronisation.
constexpr uint64_t kDispenserWaitSeconds = 5;
constexpr uint64_t kGatherWaitSeconds = 60;
// Longest time between two re-anchorings of the GPU clock mapping: at the
// tens of parts per million the two clocks drift apart, a tenth of a
// microsecond at most.
constexpr uint64_t kDirectOneShotRounds = 4;  // direct kernel: one workgroup per tile from this many rounds
constexpr double kReanchorNs = 5e6;
// How long a re-anchoring run watches for the GPU's first workgroup.
constexpr int64_t kAnchorWatchNs = 2'000'000;

struct Binding {
  const void* host = nullptr;  // input: read by host workers
  const void* dev = nullptr;   // input: read by the GPU
  void* host_out = nullptr;
  void* dev_out = nullptr;
  size_t bytes = 0;
  bool bound = false;
  // The GPU's view of the host pointer when the caller's host memory is
  // pinned (hipHostMalloc, e.g. a pinned torch tensor): the kernel can then
  // read or write it over PCIe with no copy. Null for pageable memory.
  void* host_dev = nullptr;
};

// The device address of pinned host memory at p, or null if p is pageable.
void* pinned_device_view(const void* p) {
  if (!p) return nullptr;
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // pageable memory: not an error worth keeping
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost) return nullptr;
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, const_cast<void*>(p), 0) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return d;
}

// Engine-owned scratch memory that grows on demand.
struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  bool ensure(size_t bytes) {
    if (bytes <= n) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) return false;
    n = bytes;
    return true;
  }
};
struct PinnedBuf {
  void* p = nullptr;
  size_t n = 0;
  unsigned flags = hipHostMallocDefault;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  bool ensure(size_t bytes, bool zero = false) {
    if (bytes <= n) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    if (hipHostMalloc(&p, bytes, flags) != hipSuccess) return false;
    if (zero) memset(p, 0, bytes);
    n = bytes;
    return true;
  }
};

struct HostPkg {
  uint64_t g0 = 0, g1 = 0, base = 0;
  uint32_t ntiles = 0;
  std::atomic<uint32_t> tiles_done{0};
  int64_t t_claim = 0;
  std::atomic<int64_t> t_end{0};
};

// The host worker pool's own level-2 chain (same protocol as the GPU's).
struct HostQueue {
  alignas(64) std::atomic<uint64_t> ticket{0};
  alignas(64) std::atomic<uint64_t> total{0};
  alignas(64) std::atomic<uint32_t> done{0};
  uint32_t n_pkgs = 0;     // written by the claimer only
  uint64_t st_next = 0;    // static band cursor (claimer only)
  uint64_t granules = 0;   // claimer only
  std::unique_ptr<HostPkg[]> pkgs;
  size_t cap = 0;
  bool ensure(size_t n) {
    if (n <= cap) return true;
    pkgs.reset(new (std::nothrow) HostPkg[n]);
    cap = pkgs ? n : 0;
    return pkgs != nullptr;
  }
  void reset() {
    ticket.store(0, std::memory_order_relaxed);
    total.store(0, std::memory_order_relaxed);
    done.store(0, std::memory_order_relaxed);
    n_pkgs = 0;
    st_next = 0;
    granules = 0;
  }
};

}  // namespace
}  // namespace ce

using namespace ce;

struct ce_engine {
  // ---- device and HIP state
  int gpu = -1;
  int n_cu = 0;
  uint32_t wallclock_hz = 100000000;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // caller's, optional
  L1State* l1 = nullptr;       // host view
  L1State* l1_dev = nullptr;   // device view
  L2State* l2 = nullptr;
  DevBuf pkgs_dev;
  DevBuf pub_dev;  // publication words of the GPU's packages, zero between runs
  uint32_t pkgs_dev_cap = 0;
  // The allocation-free run keeps the queue state, publication words and
  // package table in this device's static scratch array instead.
  void* noalloc_base = nullptr;      // device address of the scratch (null: unavailable)
  hipError_t noalloc_err = hipSuccess;
  bool noalloc = false;              // the current run may not allocate
  PkgSlot* trace_pkgs = nullptr;     // package table of the last run
  uint32_t trace_pkgs_cap = 0;
  // GPU tick -> host ns: host_ns = anchor_ns + (tick - anchor_tick) * ns_per_tick.
  // The anchor is the latest GPU start the host saw as it happened (renewed
  // every few milliseconds); the rate is measured between the calibration
  // at creation and that anchor, since
  // the two clocks drift apart by a few parts per million (tens of
  // microseconds over a few seconds, as much as a whole blur run).
  uint64_t anchor0_tick = 0, anchor_tick = 0;
  double anchor0_ns = 0.0, anchor_ns = 0.0;
  double ns_per_tick = 10.0;
  double clock_latency_ns = 0.0; // one-way GPU -> host visibility latency (half the best round trip)
  bool clock_ok = false;
  double tick_to_host_ns(uint64_t tick) const {
    return anchor_ns + (tick >= anchor_tick ? (double)(tick - anchor_tick) : -(double)(anchor_tick - tick)) * ns_per_tick;
  }
  void re_anchor(uint64_t tick, double host_ns) {
    anchor_tick = tick;
    anchor_ns = host_ns;
    const double nominal = 1e9 / (double)wallclock_hz;
    if (tick > anchor0_tick + (uint64_t)wallclock_hz) {  // at least a second apart
      const double r = (host_ns - anchor0_ns) / (double)(tick - anchor0_tick);
      if (r > nominal * 0.999 && r < nominal * 1.001) ns_per_tick = r;
    }
  }
  const HostPayloadFns* hp = nullptr;

  // ---- configuration
  uint32_t dev_mask = CE_DEV_GPU;
  int host_threads = 0;  // resolved count
  uint32_t ndim = 0;
  uint64_t gws[2] = {0, 0};
  uint32_t lws0 = 256;
  ce_sched_desc sched{};
  bool sched_set = false;
  int kernel_id = 0;
  ce_escape_params esc{};
  ce_blur5_params blur{};
  ce_nbody_params nb{};
  ce_nbody_step_params nbs{};
  ce_binomial_params bin{};
  static constexpr int kOccSlots = 16;
  int occ_cache[kOccSlots] = {};  // persistent workgroups per CU by (kernel id, strict)
  Binding in[kMaxSlots];
  Binding out[kMaxSlots];
  uint32_t pat_outs = 1, pat_items = 1;

  // ---- scratch
  DevBuf in_dev[kMaxSlots];
  PinnedBuf in_host[kMaxSlots];
  DevBuf out_dev_scratch[kMaxSlots];
  PinnedBuf out_host_scratch[kMaxSlots];  // host output when only a device output is bound
  PinnedBuf ring_buf;           // host completion ring read by the GPU's gatherers
  int merge_mode = CE_MERGE_DMA;  // CE_MERGE_GPU_GATHER where the GPU has no copy engine
  bool gather = false;          // this run's host tiles are copied into HBM by the GPU
  bool push = false;            // this run's host packages are copied into HBM by DMA
  SdmaCopier sdma;              // the GPU's copy engines (none: CE_MERGE_DMA is unavailable)
  char sdma_why[128] = "";
  std::mutex push_mu;
  std::deque<std::pair<int, uint64_t>> push_pending;  // copies in flight (copier handle, bytes)
  uint64_t push_inflight = 0, push_total = 0;
  std::atomic<int> push_error{0};
  int64_t push_end_ns = 0;
  std::atomic<uint64_t> ring_count{0};
  std::atomic<uint64_t> ring_written{0};  // entries whose ring word is stored
  std::atomic<uint64_t> ring_bytes{0};    // bytes of those entries

  // ---- host pool
  std::vector<std::thread> pool;
  std::mutex mu;
  std::condition_variable cv;
  std::atomic<uint64_t> epoch{0};
  std::atomic<uint32_t> pool_done{0};
  std::atomic<bool> quit{false};
  std::atomic<int> sleeping{0};

  // ---- per-run state
  HostQueue hq;
  SchedArgs host_args{};
  KernelArgs kargs{};
  uint64_t run_id = 0;
  int64_t t0_ns = 0;
  const void* host_in0 = nullptr;
  const void* host_in1 = nullptr;
  // payload supplied as source at run time: its loaded module, its host
  // version, its slots and scalars, and the host workers' arguments
  void* rt_module = nullptr;
  void* rt_fn_persistent = nullptr;
  void* rt_fn_bare = nullptr;
  void* rt_fn_direct = nullptr;
  ce_rt_host_fn rt_host = nullptr;
  uint32_t rt_n_in = 0, rt_n_out = 0, rt_item_bytes = 0;
  uint64_t rt_in_bytes[2] = {0, 0};
  unsigned char rt_scalars[CE_RT_SCALAR_BYTES] = {};
  ce_rt_args rt_host_args{};
  void* host_out = nullptr;    // output slot 0 as the host workers write it
  void* host_out1 = nullptr;   // output slot 1 (n-body step velocities)
  std::atomic<int> host_error{0};

  // ---- results
  ce_run_stats stats{};
  bool stats_valid = false;
  // The statistics of a run are worked out when first asked for, not inside
  // the run: a run on the GPU alone would otherwise read every workgroup's
  // end tick back from host memory the GPU just wrote (2048 cache lines'
  // worth of misses for a 2048-workgroup grid) before returning.
  bool stats_pending = false;
  uint64_t pending_G = 0;
  int64_t pending_t_end = 0;
  void ensure_stats() {
    if (!stats_pending) return;
    stats_pending = false;
    fill_stats(pending_G, pending_t_end);
  }
  std::vector<ce_package_rec> trace;
  uint64_t gpu_pkgs_last = 0;
  uint32_t gpu_grid_last = 0;
  uint32_t grid_override = 0;  // persistent workgroups chosen by the caller (0: the engine chooses)
  bool pcie_stream = false;    // this run's kernel reads or writes pinned host memory directly
  uint64_t* wg_end = nullptr;      // host-coherent, kFastExitMaxWgs entries (light exit)
  uint64_t* wg_end_dev = nullptr;
  bool fast_exit = false;          // this run's kernel is the direct one
  bool light_exit = false;         // its workgroups leave without counting out
  // Two queue-state buffers (and two halves of the publication words) taken
  // in turn by successive GPU runs: a run's kernel clears the other one for
  // the next run, so no workgroup resets anything as it leaves.
  uint64_t gpu_seq = 0;            // GPU runs launched from the double buffers
  L2State* l2_last = nullptr;      // the queue state of the last run
  int64_t ph_launched = 0, ph_host_done = 0, ph_gpu_seen = 0, ph_synced = 0, ph_copies = 0;  // phase ends (ns)
  uint64_t fast_g0 = 0, fast_g1 = 0;  // its one package
  double dispenser_wait_s = (double)kDispenserWaitSeconds;  // bounds on the kernel's waits
  double gather_wait_s = (double)kGatherWaitSeconds;

  std::vector<std::string> errors;

  ce_status fail(ce_status code, const char* fmt, ...) __attribute__((format(printf, 3, 4))) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    errors.emplace_back(buf);
    return code;
  }
  ce_status hip_fail(hipError_t e, const char* what) {
    return fail(CE_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  }

  bool use_gpu() const { return dev_mask & CE_DEV_GPU; }
  bool use_host() const { return dev_mask & CE_DEV_HOST; }
  uint32_t n_devices() const { return (use_gpu() ? 1u : 0u) + (use_host() ? 1u : 0u); }
  int gpu_index() const { return use_gpu() ? 0 : -1; }
  int host_index() const { return use_host() ? (use_gpu() ? 1 : 0) : -1; }

  double tick_to_host_s(uint64_t tick) const {
    return (tick_to_host_ns(tick) - (double)t0_ns) * 1e-9;
  }

  // ------------------------------------------------------------ geometry
  uint64_t granules() const {
    switch (kernel_id) {
      case CE_KERNEL_ESCAPE: return esc.h;
      case CE_KERNEL_BLUR5: return blur.h;
      case CE_KERNEL_NBODY_ACC: return ceil_div(nb.n, kNbodyGranule);
      case CE_KERNEL_NBODY_STEP: return ceil_div(nbs.n, kNbodyGranule);
      case CE_KERNEL_BINOMIAL: return bin.n_groups;
      case CE_KERNEL_RUNTIME: return lws0 ? ceil_div(gws[0], lws0) : 0;
    }
    return 0;
  }
  // first work-item of granule g of a runtime payload
  uint64_t rt_item(uint64_t g) const { return std::min<uint64_t>(g * lws0, gws[0]); }
  uint32_t n_bodies() const { return kernel_id == CE_KERNEL_NBODY_STEP ? nbs.n : nb.n; }
  bool is_nbody() const { return kernel_id == CE_KERNEL_NBODY_ACC || kernel_id == CE_KERNEL_NBODY_STEP; }
  // Whether the GPU kernel reads each input byte about once (streaming), so a
  // pinned host input is better read over PCIe than copied first. N-body
  // reads every position once per body block; a runtime payload may read
  // its inputs any number of times.
  bool reads_input_once() const { return kernel_id == CE_KERNEL_BLUR5 || kernel_id == CE_KERNEL_BINOMIAL; }
  uint64_t items_in(uint64_t g0, uint64_t g1) const {
    switch (kernel_id) {
      case CE_KERNEL_ESCAPE: return (g1 - g0) * esc.w;
      case CE_KERNEL_BLUR5: return (g1 - g0) * blur.w;
      case CE_KERNEL_NBODY_ACC:
      case CE_KERNEL_NBODY_STEP: {
        const uint64_t a = g0 * kNbodyGranule, b = std::min<uint64_t>(g1 * kNbodyGranule, n_bodies());
        return b > a ? b - a : 0;
      }
      case CE_KERNEL_BINOMIAL: return (g1 - g0) * (bin.steps + 1);  // one work-group per granule
      case CE_KERNEL_RUNTIME: return rt_item(g1) - rt_item(g0);
    }
    return 0;
  }
  // output elements: one float4 per body, per option group, or one word per pixel
  size_t out_elem_bytes() const {
    if (kernel_id == CE_KERNEL_RUNTIME) return rt_item_bytes;
    return (is_nbody() || kernel_id == CE_KERNEL_BINOMIAL) ? 16 : 4;
  }
  // first output element of granule g (out pattern 1:(steps+1) for binomial)
  uint64_t item_offset(uint64_t g) const {
    if (kernel_id == CE_KERNEL_BINOMIAL) return g;
    if (kernel_id == CE_KERNEL_RUNTIME) return rt_item(g);
    return is_nbody() ? std::min<uint64_t>(g * kNbodyGranule, n_bodies()) : g * gws[0];
  }
  size_t in_bytes(int slot) const {
    switch (kernel_id) {
      case CE_KERNEL_BLUR5:
        return slot == 0 ? (size_t)blur.w * blur.h * 4 : (slot == 1 ? 25 * 4 : 0);
      case CE_KERNEL_NBODY_ACC: return slot == 0 ? (size_t)nb.n * 16 : 0;
      case CE_KERNEL_NBODY_STEP: return slot < 2 ? (size_t)nbs.n * 16 : 0;
      case CE_KERNEL_BINOMIAL: return slot == 0 ? (size_t)bin.n_groups * 16 : (slot == 1 ? (size_t)(bin.steps + 1) * 4 : 0);
      case CE_KERNEL_RUNTIME: return slot >= 0 && (uint32_t)slot < rt_n_in ? (size_t)rt_in_bytes[slot] : 0;
    }
    return 0;
  }
  int n_in_slots() const {
    switch (kernel_id) {
      case CE_KERNEL_BLUR5: return 2;
      case CE_KERNEL_NBODY_ACC: return 1;
      case CE_KERNEL_NBODY_STEP: return 2;
      case CE_KERNEL_BINOMIAL: return 2;
      case CE_KERNEL_RUNTIME: return (int)rt_n_in;
    }
    return 0;
  }
  int n_out_slots() const {
    if (kernel_id == CE_KERNEL_RUNTIME) return (int)rt_n_out;
    return kernel_id == CE_KERNEL_NBODY_STEP ? 2 : 1;
  }
  size_t out_bytes() const {
    switch (kernel_id) {
      case CE_KERNEL_ESCAPE: return (size_t)esc.w * esc.h * 4;
      case CE_KERNEL_BLUR5: return (size_t)blur.w * blur.h * 4;
      case CE_KERNEL_NBODY_ACC: return (size_t)nb.n * 16;
      case CE_KERNEL_NBODY_STEP: return (size_t)nbs.n * 16;
      case CE_KERNEL_BINOMIAL: return (size_t)bin.n_groups * 16;
      case CE_KERNEL_RUNTIME: return (size_t)gws[0] * rt_item_bytes;
    }
    return 0;
  }
  uint32_t host_tiles(uint64_t g0, uint64_t g1) const {
    if (is_nbody()) return (uint32_t)ceil_div(items_in(g0, g1), kHostNbodyTile);
    return (uint32_t)(g1 - g0);
  }

  // ------------------------------------------------------------ host pool
  // Threads start from the epoch current before the run that needs them is
  // published, so a thread created just before a run still takes part in it.
  void pool_start(int n) {
    const uint64_t start = epoch.load();
    for (int i = 0; i < n; ++i) pool.emplace_back([this, i, start] { pool_loop(i + 1, start); });
  }
  void pool_stop() {
    {
      std::lock_guard<std::mutex> lk(mu);
      quit.store(true);
    }
    cv.notify_all();
    for (auto& t : pool) t.join();
    pool.clear();
    quit.store(false);
  }
  void pool_loop(int tid, uint64_t seen) {
    for (;;) {
      // Spin briefly for low wake-up latency, then sleep. While spinning,
      // give the core up now and then: with a worker on every core, a thread
      // of the HIP runtime (or the caller's) that needs one would otherwise
      // preempt a worker for a whole time slice, possibly one holding a tile.
      const int64_t spin_until = now_ns() + 20'000'000;
      uint64_t e;
      uint32_t spins = 0;
      while ((e = epoch.load(std::memory_order_acquire)) == seen && !quit.load(std::memory_order_relaxed)) {
        if (now_ns() > spin_until) {
          std::unique_lock<std::mutex> lk(mu);
          sleeping.fetch_add(1);
          cv.wait(lk, [&] { return epoch.load() != seen || quit.load(); });
          sleeping.fetch_sub(1);
        }
        if ((++spins & 255u) == 0) std::this_thread::yield();
        cpu_relax();
      }
      if (quit.load()) return;
      seen = e;
      if (tid < host_threads) host_work();
      pool_done.fetch_add(1, std::memory_order_acq_rel);
    }
  }

  // Claims the GPU's first package on the host just before the launch, with
  // the same arithmetic the kernel's claimer uses, so that the workgroups find
  // work published when they start instead of racing for the claim lock.
  void gpu_preclaim(SchedArgs& gs, uint64_t round_wgs) {
    gs.pre_nt = 0;
    gs.st_first = 0;
    gs.pre_only = 0;
    uint64_t g0 = 0, g1 = 0;
    if (gs.kind == kStatic) {
      if (gs.st_begin >= gs.st_end) return;
      if (gs.st_nbands == 0) {
        g0 = gs.st_begin;
        g1 = (gs.st_end - g0 > kPubMaxSize) ? g0 + kPubMaxSize : gs.st_end;
        gs.pre_only = g1 == gs.st_end ? 1u : 0u;
      } else {
        g0 = band_edge(gs.st_begin, gs.G, gs.st_nbands);
        g1 = band_edge(gs.st_begin + 1, gs.G, gs.st_nbands);
        gs.pre_only = gs.st_begin + 1 == gs.st_end ? 1u : 0u;
      }
      gs.st_first = 1;
    } else if (gs.kind == kDynamic) {
      const uint64_t a = __atomic_fetch_add(&l1->next, gs.pkg, __ATOMIC_RELAXED);
      if (a >= gs.G) return;
      g0 = a;
      g1 = std::min(a + gs.pkg, gs.G);
    } else {
      // One HGuided package; and a second, consecutive one when the first
      // holds less than two rounds of tiles and two rounds' worth would
      // still remain after it. The kernel's first claim then falls due a round later:
      // a claim made as the first round ends queues behind every
      // workgroup's ticket atomic (when the first tiles are cheap they all
      // come at once), and the GPU would wait for it with nothing published.
      // No other device claims before the launch, so the two ranges are
      // contiguous: the GPU claims twice in a row, as one range.
      const uint64_t round = std::max<uint64_t>(1, round_wgs);
      uint64_t cur = __atomic_load_n(&l1->next, __ATOMIC_ACQUIRE);
      for (int n = 0; n < 2; ++n) {
        bool got = false;
        for (;;) {
          if (cur >= gs.G) break;
          uint64_t sz = hguided_size(gs.G - cur, gs.P_self, gs.sumP, gs.n_dev, gs.k, gs.min_self);
          if (g1 > g0 && sz > kPubMaxSize - (g1 - g0)) sz = kPubMaxSize - (g1 - g0);
          if (sz > kPubMaxSize) sz = kPubMaxSize;
          if (sz == 0) break;
          if (n == 1 && (cur != g1 || gpu_tiles(kargs, g0, g1) >= 2 * round ||
                         gpu_tiles(kargs, cur + sz, gs.G) < 2 * round))
            break;
          if (__atomic_compare_exchange_n(&l1->next, &cur, cur + sz, false, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE)) {
            if (n == 0) g0 = cur;
            g1 = cur + sz;
            cur += sz;
            got = true;
            break;
          }
        }
        if (!got) break;
      }
      if (g1 == g0) return;
    }
    gs.pre_g0 = g0;
    gs.pre_g1 = g1;
    gs.pre_nt = gpu_tiles(kargs, g0, g1);
  }

  // Claims the next package for the host device from the level-1 dispenser
  // (or the static plan). Only the host chain's claimer calls this.
  bool host_claim(uint64_t* g0, uint64_t* g1) {
    const SchedArgs& s = host_args;
    if (s.kind == kStatic) {
      if (s.st_nbands == 0) {
        if (hq.st_next != 0 || s.st_begin >= s.st_end) return false;
        *g0 = s.st_begin;
        *g1 = s.st_end;
      } else {
        const uint64_t b = s.st_begin + hq.st_next;
        if (b >= s.st_end) return false;
        *g0 = band_edge(b, s.G, s.st_nbands);
        *g1 = band_edge(b + 1, s.G, s.st_nbands);
      }
      hq.st_next++;
      return true;
    }
    if (s.kind == kDynamic) {
      const uint64_t a = __atomic_fetch_add(&l1->next, s.pkg, __ATOMIC_RELAXED);
      if (a >= s.G) return false;
      *g0 = a;
      *g1 = std::min(a + s.pkg, s.G);
      return true;
    }
    uint64_t cur = __atomic_load_n(&l1->next, __ATOMIC_ACQUIRE);
    for (;;) {
      if (cur >= s.G) return false;
      const uint64_t sz = hguided_size(s.G - cur, s.P_self, s.sumP, s.n_dev, s.k, s.min_self);
      if (__atomic_compare_exchange_n(&l1->next, &cur, cur + sz, false, __ATOMIC_ACQ_REL, __ATOMIC_ACQUIRE)) {
        *g0 = cur;
        *g1 = cur + sz;
        return true;
      }
    }
  }

  // Computes host tile ti of package p; 0, or the host function's failure code.
  int32_t host_tile(const HostPkg& p, uint32_t ti) {
    switch (kernel_id) {
      case CE_KERNEL_ESCAPE: hp->escape_rows(esc, p.g0 + ti, p.g0 + ti + 1, (uint32_t*)host_out); break;
      case CE_KERNEL_BLUR5:
        hp->blur5_rows((const float*)host_in0, blur.w, blur.h, (const float*)host_in1, p.g0 + ti, p.g0 + ti + 1,
                       (float*)host_out);
        break;
      case CE_KERNEL_NBODY_ACC: {
        const uint64_t i0 = p.g0 * kNbodyGranule + (uint64_t)ti * kHostNbodyTile;
        const uint64_t end = std::min<uint64_t>(p.g1 * kNbodyGranule, nb.n);
        const uint64_t i1 = std::min<uint64_t>(i0 + kHostNbodyTile, end);
        hp->nbody_bodies((const float*)host_in0, nb.n, nb.eps2, (int)nb.strict, i0, i1, (float*)host_out);
        break;
      }
      case CE_KERNEL_NBODY_STEP: {
        const uint64_t i0 = p.g0 * kNbodyGranule + (uint64_t)ti * kHostNbodyTile;
        const uint64_t end = std::min<uint64_t>(p.g1 * kNbodyGranule, nbs.n);
        const uint64_t i1 = std::min<uint64_t>(i0 + kHostNbodyTile, end);
        // the accelerations land in the velocity output first, then the step
        // turns them into the new velocities
        hp->nbody_bodies((const float*)host_in0, nbs.n, nbs.eps2, (int)nbs.strict, i0, i1, (float*)host_out1);
        nbody_step_update((const float*)host_in0, (const float*)host_in1, nbs.dt, i0, i1, (float*)host_out,
                          (float*)host_out1);
        break;
      }
      case CE_KERNEL_BINOMIAL:
        binomial_groups((const float*)host_in0, (const float*)host_in1, bin.steps, bin.strike, bin.pu, bin.pd,
                        p.g0 + ti, p.g0 + ti + 1, (float*)host_out);
        break;
      case CE_KERNEL_RUNTIME: return rt_host(rt_item(p.g0 + ti), rt_item(p.g0 + ti + 1), &rt_host_args);
    }
    return 0;
  }

  // The first host tile that failed in this run (host_fail_code 0: none).
  std::atomic<int32_t> host_fail_code{0};
  uint64_t host_fail_i0 = 0, host_fail_i1 = 0;
  void host_tile_failed(const HostPkg& p, uint32_t ti, int32_t code) {
    int32_t none = 0;
    if (host_fail_code.compare_exchange_strong(none, code)) {
      host_fail_i0 = kernel_id == CE_KERNEL_RUNTIME ? rt_item(p.g0 + ti) : p.g0 + ti;
      host_fail_i1 = kernel_id == CE_KERNEL_RUNTIME ? rt_item(p.g0 + ti + 1) : p.g0 + ti + 1;
    }
    // the host device claims nothing more; its claimed tiles still run
    hq.done.store(1, std::memory_order_release);
  }

  // Byte range of the output written by host tile ti of package p.
  void host_tile_bytes(const HostPkg& p, uint32_t ti, uint64_t* off, uint64_t* len) const {
    if (is_nbody()) {
      const uint64_t i0 = p.g0 * kNbodyGranule + (uint64_t)ti * kHostNbodyTile;
      const uint64_t end = std::min<uint64_t>(p.g1 * kNbodyGranule, n_bodies());
      const uint64_t i1 = std::min<uint64_t>(i0 + kHostNbodyTile, end);
      *off = i0 * 16;
      *len = (i1 - i0) * 16;
    } else if (kernel_id == CE_KERNEL_BINOMIAL) {
      *off = (p.g0 + ti) * 16;
      *len = 16;
    } else if (kernel_id == CE_KERNEL_RUNTIME) {
      *off = rt_item(p.g0 + ti) * rt_item_bytes;
      *len = (rt_item(p.g0 + ti + 1) - rt_item(p.g0 + ti)) * rt_item_bytes;
    } else {
      *off = (p.g0 + ti) * gws[0] * 4;
      *len = gws[0] * 4;
    }
  }
  // Makes a finished host tile visible to the GPU's gatherers (x86 stores
  // are seen in program order, so the data precede the ring entry).
  void publish_host_tile(const HostPkg& p, uint32_t ti) {
    uint64_t off, len;
    host_tile_bytes(p, ti, &off, &len);
    const uint64_t k = ring_count.fetch_add(1, std::memory_order_relaxed);
    uint64_t* ring = (uint64_t*)ring_buf.p;
    __atomic_store_n(&ring[k], ring_word(off, len), __ATOMIC_RELEASE);
    ring_bytes.fetch_add(len, std::memory_order_relaxed);
    ring_written.fetch_add(1, std::memory_order_release);
  }

  // Byte range of the output written by granules [g0, g1).
  void out_range(uint64_t g0, uint64_t g1, size_t* off, size_t* len) const {
    const size_t eb = out_elem_bytes();
    *off = (size_t)item_offset(g0) * eb;
    *len = (size_t)(item_offset(g1) - item_offset(g0)) * eb;
  }

  // DMA merge: a finished host package's output goes host -> HBM on the
  // GPU's copy engines while its kernel keeps every CU busy.
  void push_package(const HostPkg& p) {
    size_t off, len;
    out_range(p.g0, p.g1, &off, &len);
    if (!len) return;
    std::lock_guard<std::mutex> lk(push_mu);
    void* const src[2] = {host_out, host_out1};
    for (int s = 0; s < n_out_slots(); ++s) {
      const int h = sdma.start((char*)out[s].dev_out + off, (const char*)src[s] + off, len);
      if (h < 0) {
        push_error.store(1);
        return;
      }
      push_pending.emplace_back(h, (uint64_t)len);
      push_inflight += len;
      push_total += len;
    }
  }
  // Retires finished copies and blocks until the bytes in flight fit the
  // backlog (the host is worth only as much output as PCIe carries). Only
  // one thread drains at a time: the host claimer during a run, the caller
  // after it, so a handle waited on outside the lock stays valid.
  void push_drain(uint64_t backlog) {
    std::unique_lock<std::mutex> lk(push_mu);
    for (;;) {
      while (!push_pending.empty() && sdma.poll(push_pending.front().first)) {
        push_inflight -= push_pending.front().second;
        sdma.release(push_pending.front().first);
        push_pending.pop_front();
      }
      if (push_inflight <= backlog || push_pending.empty()) return;
      const int h = push_pending.front().first;
      lk.unlock();
      const bool ok = sdma.wait(h, 10'000'000'000ull);
      lk.lock();
      if (!ok) {  // a copy that does not finish in 10 s: fail the run, keep the handle
        push_error.store(1);
        return;
      }
    }
  }

  // With the GPU gathering the host's output, the host is worth only as much
  // output as PCIe can carry: its claimer waits while more than
  // kGatherBacklog bytes are published but not yet copied.
  static constexpr uint64_t kGatherBacklog = 512u << 10;
  void gather_throttle() {
    const int64_t limit = now_ns() + 1'000'000'000LL;  // never wait for a stalled GPU forever
    while (ring_bytes.load(std::memory_order_relaxed) >
               __atomic_load_n(&l1->gathered, __ATOMIC_ACQUIRE) + kGatherBacklog &&
           now_ns() < limit)
      cpu_relax();
  }

  // Host side of a run: every pool thread (and the caller) runs this loop.
  void host_work() {
    uint32_t p_cache = 0;
    for (;;) {
      const uint64_t t = hq.ticket.fetch_add(1, std::memory_order_acq_rel);
      bool have = false;
      for (;;) {
        const uint64_t tot = hq.total.load(std::memory_order_acquire);
        if (t < tot) {
          have = true;
          break;
        }
        if (hq.done.load(std::memory_order_acquire)) {
          // The count read above may predate the last package: the flag is
          // set only after the final count was stored, so read it again
          // before giving up a ticket.
          if (t < hq.total.load(std::memory_order_acquire)) {
            have = true;
            break;
          }
          break;
        }
        if (t == tot) {
          uint64_t g0 = 0, g1 = 0;
          if (gather) gather_throttle();
          if (push) push_drain(kGatherBacklog);
          const int64_t tc = now_ns();
          if (hq.n_pkgs >= hq.cap || !host_claim(&g0, &g1)) {
            if (hq.n_pkgs >= hq.cap) host_error.store(1);
            hq.done.store(1, std::memory_order_release);
            break;
          }
          HostPkg& p = hq.pkgs[hq.n_pkgs];
          p.g0 = g0;
          p.g1 = g1;
          p.base = tot;
          p.ntiles = host_tiles(g0, g1);
          p.tiles_done.store(0, std::memory_order_relaxed);
          p.t_claim = tc;
          p.t_end.store(0, std::memory_order_relaxed);
          hq.n_pkgs++;
          hq.granules += g1 - g0;
          hq.total.store(tot + p.ntiles, std::memory_order_release);
          have = true;
          break;
        }
        cpu_relax();
      }
      if (!have) return;
      uint32_t p = p_cache;
      while (t >= hq.pkgs[p].base + hq.pkgs[p].ntiles) ++p;
      p_cache = p;
      HostPkg& pk = hq.pkgs[p];
      const int32_t rc = host_tile(pk, (uint32_t)(t - pk.base));
      if (rc != 0) host_tile_failed(pk, (uint32_t)(t - pk.base), rc);
      if (gather) publish_host_tile(pk, (uint32_t)(t - pk.base));
      if (pk.tiles_done.fetch_add(1, std::memory_order_acq_rel) + 1 == pk.ntiles) {
        pk.t_end.store(now_ns(), std::memory_order_release);
        if (push) push_package(pk);
      }
    }
  }

  ce_status ensure_pool() {
    const int want = std::max(0, host_threads - 1);  // the caller is worker 0
    if ((int)pool.size() == want) return CE_OK;
    pool_stop();
    pool_start(want);
    return CE_OK;
  }

  // ------------------------------------------------------------ scheduler
  ce_status build_sched(uint64_t G, SchedArgs* gpu_s, SchedArgs* host_s, uint32_t grid, size_t* gpu_max,
                        size_t* host_max) {
    const uint32_t n = n_devices();
    const int gi = gpu_index(), hi = host_index();
    SchedArgs base{};
    base.kind = (uint32_t)sched.kind;
    base.n_dev = n;
    base.k = sched.k ? sched.k : 2;
    base.G = G;
    base.run_id = run_id;
    // Waits on the dispenser last microseconds (a claim over PCIe, a
    // package becoming visible); a workgroup that waits for a claimer that is
    // not running claims itself after milliseconds. Five seconds is thus only
    // reached when something is broken, and is well inside the host's own
    // deadline for the kernel.
    base.wait_ticks = std::max<uint64_t>(1, (uint64_t)((double)wallclock_hz * dispenser_wait_s));
    base.l1 = l1_dev;
    base.l2 = l2;
    *gpu_s = base;
    *host_s = base;
    host_s->l1 = l1;
    *gpu_max = 1;
    *host_max = 1;
    if (sched.kind == CE_SCHED_STATIC) {
      double props[CE_MAX_DEVICES] = {0, 0};
      for (uint32_t d = 0; d + 1 < n; ++d) props[d] = sched.props[d];
      uint32_t order[CE_MAX_DEVICES];
      if (n == 2) {
        order[0] = sched.order == CE_ORDER_GPU_FIRST ? (uint32_t)gi : (uint32_t)hi;
        order[1] = sched.order == CE_ORDER_GPU_FIRST ? (uint32_t)hi : (uint32_t)gi;
      } else {
        order[0] = 0;
      }
      uint64_t b[CE_MAX_DEVICES], e[CE_MAX_DEVICES];
      const uint32_t nb = sched.n_packages;
      if (ce_sched_static_plan(G, n, props, order, nb, b, e) != CE_OK)
        return fail(CE_E_INVALID, "static plan: invalid proportions or band count");
      auto fill = [&](SchedArgs* s, int d) {
        s->st_nbands = nb;
        if (nb == 0) {
          s->st_begin = b[d];
          s->st_end = e[d];
        } else {
          // first band index and one past the last band of this device
          uint64_t bb = 0, be = 0;
          for (uint64_t k = 0; k <= nb; ++k) {
            if (band_edge(k, G, nb) == b[d]) { bb = k; break; }
          }
          for (uint64_t k = bb; k <= nb; ++k) {
            if (band_edge(k, G, nb) == e[d]) { be = k; break; }
          }
          s->st_begin = bb;
          s->st_end = be;
        }
      };
      if (gi >= 0) fill(gpu_s, gi);
      if (hi >= 0) fill(host_s, hi);
      *gpu_max = *host_max = nb ? nb + 1 : 2;
      return CE_OK;
    }
    if (sched.kind == CE_SCHED_DYNAMIC) {
      uint64_t pkg = sched.package_granules;
      if (pkg == 0) {
        if (sched.n_packages == 0) return fail(CE_E_INVALID, "dynamic: package_granules or n_packages required");
        pkg = ceil_div(G, sched.n_packages);
      }
      if (pkg > kPubMaxSize) return fail(CE_E_INVALID, "dynamic: package larger than 2^24-1 granules");
      gpu_s->pkg = host_s->pkg = pkg;
      *gpu_max = *host_max = ceil_div(G, pkg) + 1;
      return CE_OK;
    }
    if (sched.kind == CE_SCHED_HGUIDED) {
      uint64_t P[CE_MAX_DEVICES];
      uint64_t sumP = 0;
      for (uint32_t d = 0; d < n; ++d) {
        P[d] = sched.power[d];
        if (P[d] == 0 || P[d] > (1ull << 20)) return fail(CE_E_INVALID, "hguided: power[%u] must be in [1, 2^20]", d);
        sumP += P[d];
      }
      if (G >= (1ull << 40)) return fail(CE_E_INVALID, "hguided: index space too large");
      auto fill = [&](SchedArgs* s, int d, uint64_t def_min) {
        s->P_self = P[d];
        s->sumP = sumP;
        s->min_self = sched.min_granules[d] ? sched.min_granules[d] : def_min;
      };
      if (gi >= 0) {
        // Default minimum: one tile for every resident workgroup. Each GPU
        // claim is a chain of PCIe atomics that the host's output copies slow
        // down, and each package boundary leaves partial tiles, so the GPU
        // takes few, large packages (the host then stops claiming early).
        const uint32_t tiles_per_g = std::max<uint32_t>(1, gpu_tiles(kargs, 0, 1));
        uint64_t rows_per_tile = 1;
        while (rows_per_tile < G && gpu_tiles(kargs, 0, rows_per_tile + 1) == tiles_per_g) ++rows_per_tile;
        uint64_t def = std::max<uint64_t>(1, ceil_div((uint64_t)grid, tiles_per_g) * rows_per_tile);
        // streaming over PCIe, a few workgroups already saturate the link: an
        // eighth of a round keeps the GPU's last package short
        if (pcie_stream) def = std::max<uint64_t>(rows_per_tile, ceil_div((uint64_t)grid / 8, tiles_per_g) * rows_per_tile);
        // ... but never more than the GPU's proportional share of the space
        // (where the host is the faster device the GPU must leave it work)
        def = std::min<uint64_t>(def, std::max<uint64_t>(1, G * P[gi] / sumP));
        fill(gpu_s, gi, std::min<uint64_t>(def, G));
        *gpu_max = G / std::max<uint64_t>(1, gpu_s->min_self) + 2;
      }
      if (hi >= 0) {
        // default minimum: one host tile for every worker thread
        const uint64_t tpg = std::max<uint32_t>(1, host_tiles(0, 1));
        fill(host_s, hi, std::min<uint64_t>(G, ceil_div((uint64_t)std::max(1, host_threads), tpg)));
        *host_max = G / std::max<uint64_t>(1, host_s->min_self) + 2;
      }
      return CE_OK;
    }
    return fail(CE_E_INVALID, "unknown scheduler kind %d", sched.kind);
  }

  // ------------------------------------------------------------ run
  ce_status run() {
    const ce_status st = run_impl();
    noalloc = false;
    return st;
  }

  // Persistent grid for T tiles on at most R resident workgroups over C
  // compute units: with g workgroups the busiest CU runs ceil(T / g) rounds
  // of ceil(g / C) workgroups, and the grid is the largest g that makes
  // that product least. 2048 blur tiles on 1280 resident workgroups: 1024
  // workgroups of two tiles each rather than a second round at 60 %; 8192
  // tiles: 1024 workgroups of eight (measured 3 % faster than 1171 of seven,
  // which leaves some CUs five workgroups and others four). The optimum is
  // a multiple of C or a whole-round split ceil(T / m), so only those are
  // tried.
  static uint32_t balanced_grid(uint64_t T, uint64_t R, uint64_t C) {
    const uint64_t top = std::max<uint64_t>(1, std::min(T, R));
    uint64_t best = 1, best_cost = ~0ull;
    auto consider = [&](uint64_t g) {
      if (g < 1 || g > top) return;
      const uint64_t cost = ceil_div(T, g) * ceil_div(g, C);
      if (cost < best_cost || (cost == best_cost && g > best)) {
        best_cost = cost;
        best = g;
      }
    };
    consider(top);
    for (uint64_t k = 1; k * C <= top; ++k) consider(k * C);
    const uint64_t m0 = ceil_div(T, top);
    for (uint64_t m = m0; m < m0 + 8; ++m) consider(ceil_div(T, m));
    return (uint32_t)best;
  }

  // Scratch layout of the allocation-free run: the queue state, then the
  // publication words, then the package table. Packages that fit:
  static uint64_t noalloc_max_pkgs() {
    return (kNoallocScratchBytes - sizeof(L2State)) / (sizeof(uint64_t) + sizeof(PkgSlot));
  }

  ce_status run_impl() {
    if (kernel_id == 0) return fail(CE_E_STATE, "run: no kernel bound");
    if (!sched_set) return fail(CE_E_STATE, "run: no scheduler set");
    if (ndim == 0) return fail(CE_E_STATE, "run: work_items not set");
    if (n_devices() == 0) return fail(CE_E_STATE, "run: empty device set");
    if (use_host() && !hp && kernel_id != CE_KERNEL_RUNTIME) return fail(CE_E_UNSUPPORTED, "run: host CPU lacks AVX2/FMA");
    if (noalloc) {
      if (!noalloc_base)
        return fail(CE_E_DEVICE, "run_noalloc: no device scratch (%s)", hipGetErrorString(noalloc_err));
      if (use_host() || !use_gpu()) return fail(CE_E_UNSUPPORTED, "run_noalloc: the device set must be the GPU alone");
      for (int s = 0; s < n_in_slots(); ++s)
        if (in[s].bound && !in[s].dev) return fail(CE_E_UNSUPPORTED, "run_noalloc: input slot %d has no device pointer", s);
      for (int s = 0; s < n_out_slots(); ++s)
        if (out[s].bound && !out[s].dev_out)
          return fail(CE_E_UNSUPPORTED, "run_noalloc: output slot %d has no device pointer", s);
      for (int s = 0; s < n_out_slots(); ++s)
        if (out[s].bound && out[s].host_out)
          return fail(CE_E_UNSUPPORTED, "run_noalloc: output slot %d also has a host pointer (it would need a copy)", s);
    }
    // index space must match the kernel
    if (is_nbody()) {
      if (ndim != 1 || gws[0] != n_bodies() || lws0 != kNbodyGranule)
        return fail(CE_E_INVALID, "run: n-body needs a 1-D space of n items with lws 256");
    } else if (kernel_id == CE_KERNEL_BINOMIAL) {
      if (ndim != 1 || lws0 != bin.steps + 1 || gws[0] != (uint64_t)(bin.steps + 1) * bin.n_groups)
        return fail(CE_E_INVALID, "run: binomial needs gws = (steps+1) * n_groups and lws = steps+1");
    } else if (kernel_id == CE_KERNEL_RUNTIME) {
      if (ndim != 1 || gws[0] == 0 || lws0 == 0) return fail(CE_E_INVALID, "run: a runtime payload needs a 1-D space");
      if (use_host() && !rt_host) return fail(CE_E_UNSUPPORTED, "run: the runtime payload has no host version");
      if (use_gpu() && !rt_fn_persistent) return fail(CE_E_STATE, "run: the runtime payload is not loaded");
    } else {
      const uint64_t w = kernel_id == CE_KERNEL_ESCAPE ? esc.w : blur.w;
      const uint64_t h = kernel_id == CE_KERNEL_ESCAPE ? esc.h : blur.h;
      if (ndim != 2 || gws[0] != w || gws[1] != h) return fail(CE_E_INVALID, "run: 2-D space must be w x h");
    }
    for (int s = 0; s < n_in_slots(); ++s)
      if (!in[s].bound) return fail(CE_E_STATE, "run: input slot %d not bound", s);
    for (int s = 0; s < n_out_slots(); ++s)
      if (!out[s].bound) return fail(CE_E_STATE, "run: output slot %d not bound", s);
    for (int s = 1; s < n_out_slots(); ++s)
      if ((out[s].host_out == nullptr) != (out[0].host_out == nullptr) ||
          (out[s].dev_out == nullptr) != (out[0].dev_out == nullptr))
        return fail(CE_E_UNSUPPORTED, "run: output slots must be bound alike (host, device or both)");

    const uint64_t G = granules();
    ++run_id;
    stats_valid = false;
    stats_pending = false;
    trace.clear();
    hipError_t he;

    // GPU-side pointers
    kargs = KernelArgs{};
    kargs.kernel_id = kernel_id;
    kargs.strict = kernel_id == CE_KERNEL_NBODY_STEP ? nbs.strict : nb.strict;
    kargs.esc = esc;
    kargs.blur = blur;
    kargs.nb = nb;
    kargs.nbs = nbs;
    kargs.bin = bin;
    const void* gin[kMaxSlots] = {nullptr, nullptr};
    if (use_gpu()) {
      for (int s = 0; s < n_in_slots(); ++s) {
        if (in[s].dev) {
          gin[s] = in[s].dev;
        } else if (in[s].host_dev && reads_input_once()) {
          gin[s] = in[s].host_dev;  // pinned: the kernel streams it over PCIe
        } else {
          if (!in_dev[s].ensure(in[s].bytes)) return fail(CE_E_NOMEM, "run: device staging for input %d", s);
          if ((he = hipMemcpyAsync(in_dev[s].p, in[s].host, in[s].bytes, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return hip_fail(he, "run: input upload");
          gin[s] = in_dev[s].p;
        }
      }
    }
    kargs.in0 = gin[0];
    kargs.in1 = gin[1];
    // the kernel reads or writes host memory over PCIe: its tiles are long
    pcie_stream = false;
    for (int s = 0; s < n_in_slots(); ++s) pcie_stream |= use_gpu() && gin[s] && gin[s] == in[s].host_dev;
    void* gpu_out[kMaxSlots] = {nullptr, nullptr};
    for (int s = 0; s < n_out_slots(); ++s) {
      gpu_out[s] = out[s].dev_out;
      // pinned host output alone: the kernel writes its rows straight into it
      if (use_gpu() && !gpu_out[s] && out[s].host_dev) gpu_out[s] = out[s].host_dev;
      if (use_gpu() && !gpu_out[s]) {
        if (!out_dev_scratch[s].ensure(out[s].bytes)) return fail(CE_E_NOMEM, "run: device output scratch");
        gpu_out[s] = out_dev_scratch[s].p;
      }
    }
    kargs.out = gpu_out[0];
    kargs.out1 = gpu_out[1];
    for (int s = 0; s < n_out_slots(); ++s) pcie_stream |= use_gpu() && gpu_out[s] && gpu_out[s] == out[s].host_dev;
    if (kernel_id == CE_KERNEL_RUNTIME) {
      // generic arguments: inputs, then outputs, then the scalar block
      for (uint32_t k = 0; k < rt_n_in; ++k) kargs.rt.buf[k] = const_cast<void*>(gin[k]);
      for (uint32_t k = 0; k < rt_n_out; ++k) kargs.rt.buf[rt_n_in + k] = gpu_out[k];
      memcpy(kargs.rt.scalars, rt_scalars, sizeof rt_scalars);
      kargs.rt_items = gws[0];
      kargs.rt_lws = lws0;
      kargs.rt_item_bytes = rt_item_bytes;
      kargs.rt_fn_persistent = rt_fn_persistent;
      kargs.rt_fn_bare = rt_fn_bare;
      kargs.rt_fn_direct = rt_fn_direct;
    }

    // host-side pointers
    host_in0 = host_in1 = nullptr;
    host_out = host_out1 = nullptr;
    if (use_host()) {
      const void* hin[kMaxSlots] = {nullptr, nullptr};
      for (int s = 0; s < n_in_slots(); ++s) {
        if (in[s].host) {
          hin[s] = in[s].host;
        } else {
          if (!in_host[s].ensure(in[s].bytes)) return fail(CE_E_NOMEM, "run: host staging for input %d", s);
          if ((he = hipMemcpyAsync(in_host[s].p, in[s].dev, in[s].bytes, hipMemcpyDeviceToHost, stream)) != hipSuccess)
            return hip_fail(he, "run: input download");
          hin[s] = in_host[s].p;
        }
      }
      host_in0 = hin[0];
      host_in1 = hin[1];
      void* hout[kMaxSlots] = {nullptr, nullptr};
      for (int s = 0; s < n_out_slots(); ++s) {
        hout[s] = out[s].host_out;
        if (!hout[s]) {
          // host-coherent so the GPU's gatherers can read it over PCIe
          out_host_scratch[s].flags = hipHostMallocCoherent | hipHostMallocMapped;
          if (!out_host_scratch[s].ensure(out[s].bytes)) return fail(CE_E_NOMEM, "run: host output scratch");
          hout[s] = out_host_scratch[s].p;
        }
      }
      host_out = hout[0];
      host_out1 = hout[1];
      if (kernel_id == CE_KERNEL_RUNTIME) {
        rt_host_args = ce_rt_args{};
        for (uint32_t k = 0; k < rt_n_in; ++k) rt_host_args.buf[k] = const_cast<void*>(hin[k]);
        for (uint32_t k = 0; k < rt_n_out; ++k) rt_host_args.buf[rt_n_in + k] = hout[k];
        memcpy(rt_host_args.scalars, rt_scalars, sizeof rt_scalars);
      }
      bool downloaded = false;
      for (int s = 0; s < n_in_slots(); ++s) downloaded |= (in[s].host == nullptr);
      if (downloaded) {
        if ((he = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(he, "run: input download");
      }
    }

    // the GPU copies the host's tiles into HBM when the output lives only there
    const bool merge_dev = use_gpu() && use_host() && out[0].dev_out && !out[0].host_out;
    if (merge_dev && merge_mode == CE_MERGE_GPU_GATHER && n_out_slots() > 1)
      return fail(CE_E_UNSUPPORTED, "run: the gather merge handles one output slot; use CE_MERGE_DMA");
    gather = merge_dev && merge_mode == CE_MERGE_GPU_GATHER;
    push = merge_dev && merge_mode == CE_MERGE_DMA;
    push_total = 0;
    push_error.store(0);
    // persistent grid: resident workgroups, plus gatherers (two per XCD)
    uint32_t grid = 0, gather_wgs = 0, resident_wgs = 0;
    if (use_gpu()) {
      // resident workgroups per CU: a property of the compiled kernel, asked once per payload
      const int occ_key = kernel_id * 2 + (kargs.strict ? 1 : 0);
      int bpc = occ_key < kOccSlots ? occ_cache[occ_key] : 0;
      if (bpc == 0) {
        if ((he = persistent_blocks_per_cu(kargs, &bpc)) != hipSuccess) return hip_fail(he, "run: occupancy");
        if (occ_key < kOccSlots) occ_cache[occ_key] = bpc;
      }
      const uint32_t resident = (uint32_t)std::max(1, bpc) * (uint32_t)n_cu;
      resident_wgs = resident;
      gather_wgs = gather ? std::min<uint32_t>(16, std::max<uint32_t>(1, resident / 4)) : 0;
      const uint64_t all_tiles = gpu_tiles(kargs, 0, G);
      if (grid_override) {
        grid = grid_override + gather_wgs;
      } else {
        const uint64_t r = std::max<uint64_t>(1, resident - gather_wgs);
        grid = balanced_grid(all_tiles, r, (uint64_t)std::max(1, n_cu)) + gather_wgs;
      }
      if (grid <= gather_wgs) grid = gather_wgs + 1;
    }

    SchedArgs gs{}, hs{};
    size_t gmax = 0, hmax = 0;
    ce_status st = build_sched(G, &gs, &hs, grid, &gmax, &hmax);
    if (st != CE_OK) return st;
    host_args = hs;
    if (use_gpu()) {
      if (noalloc) {
        const uint64_t cap = noalloc_max_pkgs();
        if (gmax > cap)
          return fail(CE_E_INVALID, "run_noalloc: the schedule needs up to %llu packages; the scratch holds %llu",
                      (unsigned long long)gmax, (unsigned long long)cap);
        char* base = (char*)noalloc_base;
        gs.l2 = (L2State*)base;
        gs.pub = (uint64_t*)(base + sizeof(L2State));
        gs.pkgs = (PkgSlot*)(base + sizeof(L2State) + gmax * sizeof(uint64_t));
        gs.max_pkgs = (uint32_t)gmax;
        // Another caller's run may have ended early and left the state dirty:
        // clear the queue state and the publication words (not the table,
        // which each run writes before reading) with a fill kernel.
        static_assert(sizeof(L2State) % sizeof(uint64_t) == 0, "queue state is whole words");
        if ((he = launch_zero_words(base, sizeof(L2State) / sizeof(uint64_t) + gmax, stream)) != hipSuccess)
          return hip_fail(he, "run_noalloc: clearing the scratch");
      } else if (gmax > pkgs_dev_cap) {
        if (!pkgs_dev.ensure(gmax * sizeof(PkgSlot)) || !pub_dev.ensure(2 * gmax * sizeof(uint64_t)))
          return fail(CE_E_NOMEM, "run: package table");
        // Cleared on the run's own stream, ahead of the kernel: a plain
        // hipMemset goes to the null stream, which a non-blocking stream does
        // not wait for, and could still be clearing the table while the
        // kernel writes its first records.
        static_assert(sizeof(PkgSlot) % sizeof(uint64_t) == 0, "package records are whole words");
        if ((he = launch_zero_words(pub_dev.p, 2 * gmax, stream)) != hipSuccess ||
            (he = launch_zero_words(pkgs_dev.p, gmax * (sizeof(PkgSlot) / sizeof(uint64_t)), stream)) != hipSuccess)
          return hip_fail(he, "run: package table");
        pkgs_dev_cap = (uint32_t)gmax;
      }
      if (!noalloc) {
        const uint32_t b = (uint32_t)(gpu_seq & 1);
        gs.pkgs = (PkgSlot*)pkgs_dev.p;
        gs.max_pkgs = pkgs_dev_cap;
        gs.l2 = l2 + b;
        gs.pub = (uint64_t*)pub_dev.p + (size_t)b * pkgs_dev_cap;
        gs.l2_next = l2 + (b ^ 1u);
        gs.pub_next = (uint64_t*)pub_dev.p + (size_t)(b ^ 1u) * pkgs_dev_cap;
        gs.pub_next_words = pkgs_dev_cap;
      }
      l2_last = gs.l2;
      trace_pkgs = gs.pkgs;
      trace_pkgs_cap = gs.max_pkgs;
      // Claim the next package while half a round of tiles is still to be
      // handed out: with the host in the set its output copies share PCIe
      // with the claim's atomics, which can then take tens of microseconds.
      // When the kernel streams host memory its tiles take milliseconds, a
      // claim's round trip is negligible beside them, and claiming early
      // would take work the host could still do: the GPU then claims only
      // when a workgroup runs out, as the paper's devices do.
      gs.lookahead = pcie_stream ? 0u : std::max<uint32_t>(1, (grid - gather_wgs) / 2);
      // A Dynamic claim takes as many packages as half a round of tiles holds:
      // the GPU's workgroups are that many requesters, and one PCIe atomic
      // per package would serialise them (about 1 us each).
      gs.batch = 1;
      gs.dyn_tiles = 0;
      if (gs.kind == kDynamic) {
        gs.dyn_tiles = std::max<uint32_t>(1, gpu_tiles(kargs, 0, std::min(gs.pkg, G)));
        gs.batch = std::max<uint32_t>(1, gs.lookahead / gs.dyn_tiles);
      }
      // Several tickets per atomic once there are several tiles per
      // workgroup: every ticket atomic goes to one counter, which serialises
      // them (escape-time 3072^2, nine tiles per workgroup, one ticket each:
      // twice the plain launch's time), while a large grab leaves the
      // workgroups uneven at the end. With k tiles per workgroup, taking
      // about sqrt(k) per atomic balances the two: sqrt(k) atomics per
      // workgroup and a last grab of sqrt(k) tiles (measured 2048^2 to
      // 8192^2: best at 2, 2-3, 4 and 8 for k = 4, 9, 16 and 64).
      const uint64_t per_wg = gpu_tiles(kargs, 0, G) / std::max<uint32_t>(1, grid - gather_wgs);
      gs.chunk = (uint32_t)std::min<uint64_t>(8, std::max<uint64_t>(1, (uint64_t)std::lround(std::sqrt((double)per_wg))));
      // Blur and n-body tiles all cost the same: a fixed round-robin needs no
      // atomics. Escape-time tiles vary, but a tile is one row segment and a
      // workgroup's rows lie far apart, which evens out its share; measured
      // on the 1024 x 1024 grid the round-robin beat an atomic ticket per
      // tile (52 us against 58 us), whose last round is one atomic per
      // workgroup on a single counter. With gatherers sharing some CUs the
      // fixed round-robin would leave the workgroups on those CUs behind, so
      // tiles are dealt dynamically then.
      // A binomial tile runs for tens of microseconds, so one atomic per tile
      // costs nothing, and dealing them one at a time keeps the GPU balanced
      // even when part of the grid becomes resident only as the rest leaves:
      // under the round-robin those late workgroups would still own a full
      // share of tickets and run them on an otherwise idle GPU.
      const bool long_tiles = kernel_id == CE_KERNEL_BINOMIAL;
      if (long_tiles) gs.chunk = 1;
      // Escape-time tiles of one column block over many rounds differ by
      // orders of magnitude (8192^2: workgroup w would run every 128th row of
      // one 512-pixel column, 64 tiles, the busiest columns all on the same
      // workgroups), and a payload supplied at run time has tiles of unknown
      // cost: beyond one round both are dealt by atomic tickets. Within one
      // round every workgroup runs one tile either way, and the round-robin
      // needs no atomic.
      const bool uneven = (kernel_id == CE_KERNEL_ESCAPE || kernel_id == CE_KERNEL_RUNTIME) &&
                          gpu_tiles(kargs, 0, G) > (uint64_t)(grid - gather_wgs);
      gs.stride = (gather || long_tiles || uneven) ? 0u : 1u;
      // the gatherers wait for the host's packages, whose length depends on the problem
      gs.gather_wait_ticks = std::max<uint64_t>(1, (uint64_t)((double)wallclock_hz * gather_wait_s));
      if (gather) {
        const uint64_t max_host_tiles =
            is_nbody() ? ceil_div(n_bodies(), kHostNbodyTile) : G;
        const size_t cap = (size_t)max_host_tiles + gather_wgs + 1;
        ring_buf.flags = hipHostMallocCoherent | hipHostMallocMapped;
        if (!ring_buf.ensure(cap * sizeof(uint64_t), true)) return fail(CE_E_NOMEM, "run: completion ring");
        void* rdev = nullptr;
        void* sdev = nullptr;
        if ((he = hipHostGetDevicePointer(&rdev, ring_buf.p, 0)) != hipSuccess ||
            (he = hipHostGetDevicePointer(&sdev, host_out, 0)) != hipSuccess)
          return hip_fail(he, "run: device view of the host output");
        gs.ring = (const uint64_t*)rdev;
        gs.gsrc = (const char*)sdev;
        gs.gdst = (char*)out[0].dev_out;
        gs.gather_wgs = gather_wgs;
        gs.ring_cap = (uint32_t)std::min<size_t>(cap, 0xFFFFFFFFu);
      }
    }
    ring_count.store(0, std::memory_order_relaxed);
    ring_written.store(0, std::memory_order_relaxed);
    ring_bytes.store(0, std::memory_order_relaxed);
    __atomic_store_n(&l1->gathered, 0, __ATOMIC_RELAXED);
    if (use_host()) {
      if (!hq.ensure(hmax)) return fail(CE_E_NOMEM, "run: host package table");
    }
    hq.reset();
    host_error.store(0);
    host_fail_code.store(0);

    // arm the level-1 dispenser
    __atomic_store_n(&l1->next, 0, __ATOMIC_RELAXED);
    __atomic_store_n(&l1->gpu_flags, 0, __ATOMIC_RELAXED);
    __atomic_thread_fence(__ATOMIC_SEQ_CST);

    t0_ns = now_ns();
    fast_exit = false;
    light_exit = false;
    // Once the clock mapping's anchor is old, the host watches for the
    // GPU's first workgroup to stamp its start and re-anchors on it (the
    // host's own work then starts a few microseconds late).
    bool anchor_watch = false;
    if (use_gpu()) {
      gpu_preclaim(gs, grid - gather_wgs);
      // Without gather workgroups every workgroup leaves on its own (the
      // next run's state is cleared by this run's kernel). When the GPU's
      // whole share was claimed before the launch and every workgroup walks
      // its own tickets, no dispenser is needed at all: the direct kernel
      // runs (the overhead of a single-device run is then that of a plain
      // launch).
      light_exit = !gather && grid <= kFastExitMaxWgs;
      // Tiles of very different cost over more than four rounds, all of
      // them this device's: one workgroup per tile, dealt by the hardware as
      // slots free up (each slot is refilled as soon as its workgroup ends,
      // where a persistent workgroup's waves wait at every tile's barrier
      // for the slowest of them), swizzled over the XCDs. Escape-time on the
      // GPU alone, against atomic tickets: 2048^2 (4 rounds) 0.105 against
      // 0.097 ms, 2560^2 0.099 against 0.140, 3072^2 0.125 against 0.177,
      // 3584^2 0.168 against 0.220, 4096^2 0.241 against 0.246.
      const bool uneven_one_shot = light_exit && gs.pre_only && !gs.stride && !grid_override &&
                                   (kernel_id == CE_KERNEL_ESCAPE || kernel_id == CE_KERNEL_RUNTIME) &&
                                   gs.pre_nt > kDirectOneShotRounds * (uint64_t)resident_wgs &&
                                   gs.pre_nt <= kFastExitMaxWgs;
      fast_exit = light_exit && gs.pre_only && (gs.stride || uneven_one_shot);
      // The fast path never touches its queue state, which therefore stays
      // clear for the next run: the buffers keep their roles, and nothing is
      // cleared either.
      if (fast_exit) {
        gs.l2_next = nullptr;
        gs.pub_next = nullptr;
        gs.pub_next_words = 0;
      }
      anchor_watch = clock_ok && gs.pre_nt && (double)t0_ns - anchor_ns > kReanchorNs;
      if (anchor_watch) __atomic_store_n(&l1->gpu_t_first, 0, __ATOMIC_RELAXED);  // before the doorbell
      gs.wg_end = light_exit ? wg_end_dev : nullptr;
      fast_g0 = gs.pre_g0;
      fast_g1 = gs.pre_g1;
      if (ev_start && (he = hipEventRecord(ev_start, stream)) != hipSuccess) return hip_fail(he, "run: event");
      if (fast_exit) {
        // the direct kernel: no dispenser, nothing of the queue state touched
        DirectArgs da{};
        da.g0 = gs.pre_g0;
        da.g1 = gs.pre_g1;
        da.ntiles = gs.pre_nt;
        da.l1 = gs.l1;
        da.pkgs = gs.pkgs;
        da.wg_end = wg_end_dev;
        // Tiles spanning several rounds of resident workgroups: one
        // workgroup per tile, dealt by the hardware as slots free up, as a
        // plain launch is. A fixed split over fewer workgroups keeps fewer
        // of them per CU than the hardware would (blur 16384^2: 1024
        // workgroups of eight tiles ran 2.8 % longer than 8192 of one).
        if (!grid_override && gs.pre_nt >= kDirectOneShotRounds * (uint64_t)resident_wgs &&
            gs.pre_nt <= kFastExitMaxWgs)
          grid = gs.pre_nt;
        if (uneven_one_shot) {
          grid = gs.pre_nt;
          da.swizzle = 1;
        }
        he = launch_direct(kargs, da, grid, stream);
      } else {
        he = launch_persistent(kargs, gs, grid, stream);
      }
      if (he != hipSuccess) return hip_fail(he, "run: kernel launch");
      if (!noalloc && !fast_exit) ++gpu_seq;  // the buffers' roles swap for the next run
      if (ev_stop && (he = hipEventRecord(ev_stop, stream)) != hipSuccess) return hip_fail(he, "run: event");
    }
    ph_launched = use_gpu() ? now_ns() : 0;
    ph_host_done = ph_gpu_seen = ph_synced = ph_copies = 0;
    if (anchor_watch) {
      // Only a start seen as it happens (the first read still finds zero)
      // is an anchor: the host time is then the tick's, give or take the
      // one-way latency measured at calibration.
      const int64_t give_up = now_ns() + kAnchorWatchNs;
      uint64_t tf = __atomic_load_n(&l1->gpu_t_first, __ATOMIC_ACQUIRE);
      if (tf == 0) {
        while ((tf = __atomic_load_n(&l1->gpu_t_first, __ATOMIC_ACQUIRE)) == 0 && now_ns() < give_up) cpu_relax();
        if (tf) re_anchor(tf, (double)now_ns() - clock_latency_ns);
      }
      ph_gpu_seen = now_ns();
    }
    gpu_grid_last = grid;
    if (use_host()) {
      ensure_pool();
      pool_done.store(0, std::memory_order_relaxed);
      epoch.fetch_add(1);  // seq_cst pairs with the sleepers' counter
      if (sleeping.load() > 0) {
        std::lock_guard<std::mutex> lk(mu);
        cv.notify_all();
      }
      host_work();
      if (gather) {
        // The host chain is closed, so its tile count is final: tell the
        // gatherers as soon as the last tile is in the ring, without waiting
        // for pool threads that have not noticed the end yet.
        const uint64_t n_tiles = hq.total.load(std::memory_order_acquire);
        while (ring_written.load(std::memory_order_acquire) < n_tiles) cpu_relax();
        __atomic_store_n(&l1->host_final, host_final_word(run_id, n_tiles), __ATOMIC_RELEASE);
      }
      const uint32_t want = (uint32_t)pool.size();
      while (pool_done.load(std::memory_order_acquire) < want) cpu_relax();
      ph_host_done = now_ns();
    }
    if (use_gpu() && fast_exit) {
      if ((he = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(he, "run: kernel");
      ph_synced = now_ns();
    } else if (use_gpu()) {
      if ((he = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(he, "run: kernel");
      ph_synced = now_ns();
      // with the regular exit the last workgroup out writes the done word
      // before the kernel ends
      if (!light_exit && !done_is(__atomic_load_n(&l1->gpu_done, __ATOMIC_ACQUIRE), run_id))
        return fail(CE_E_TIMEOUT, "run: GPU did not report completion");
      if (gather) memset(ring_buf.p, 0, ring_count.load() * sizeof(uint64_t));  // ready for the next run
      if (__atomic_load_n(&l1->gpu_flags, __ATOMIC_ACQUIRE))
        return fail(CE_E_TIMEOUT, "run: GPU dispenser wait exceeded its bound or package table overflow");
    }
    if (push) {
      // the last host packages' copies finish after the host's work
      push_drain(0);
      push_end_ns = now_ns();
      ph_copies = push_end_ns;
      if (push_error.load()) return fail(CE_E_DEVICE, "run: host output copy to the device failed");
    }
    if (host_error.load()) return fail(CE_E_DEVICE, "run: host package table overflow");
    if (const int32_t code = host_fail_code.load())
      return fail(CE_E_DEVICE, "run: the host version failed with code %d on work-items [%llu, %llu)", (int)code,
                  (unsigned long long)host_fail_i0, (unsigned long long)host_fail_i1);

    // merge outputs so each bound pointer holds the whole result
    st = merge_outputs(gpu_out);
    if (st != CE_OK) return st;
    pending_t_end = now_ns();
    pending_G = G;
    stats_pending = true;
    return CE_OK;
  }

  // Host packages sorted into maximal intervals.
  std::vector<std::pair<uint64_t, uint64_t>> host_intervals() const {
    std::vector<std::pair<uint64_t, uint64_t>> v;
    for (uint32_t i = 0; i < hq.n_pkgs; ++i) v.emplace_back(hq.pkgs[i].g0, hq.pkgs[i].g1);
    std::sort(v.begin(), v.end());
    std::vector<std::pair<uint64_t, uint64_t>> m;
    for (auto& iv : v) {
      if (!m.empty() && m.back().second == iv.first)
        m.back().second = iv.second;
      else
        m.push_back(iv);
    }
    return m;
  }

  ce_status merge_outputs(void* const* gpu_out) {
    hipError_t he;
    const size_t eb = out_elem_bytes();
    const uint64_t G = granules();
    auto bytes_of = [&](uint64_t g0, uint64_t g1, size_t* off, size_t* len) {
      *off = (size_t)item_offset(g0) * eb;
      *len = (size_t)(item_offset(g1) - item_offset(g0)) * eb;
    };
    const auto hiv = use_host() ? host_intervals() : std::vector<std::pair<uint64_t, uint64_t>>{};
    bool issued = false;
    // host-computed ranges into the device output (unless the GPU gathered them)
    void* const hsrc[kMaxSlots] = {host_out, host_out1};
    if (use_host() && out[0].dev_out && !gather && !push) {
      for (int s = 0; s < n_out_slots(); ++s) {
        for (auto& iv : hiv) {
          size_t off, len;
          bytes_of(iv.first, iv.second, &off, &len);
          if (!len) continue;
          if ((he = hipMemcpyAsync((char*)out[s].dev_out + off, (const char*)hsrc[s] + off, len,
                                   hipMemcpyHostToDevice, stream)) != hipSuccess)
            return hip_fail(he, "merge: host ranges to device");
          issued = true;
        }
      }
    }
    // GPU-computed ranges (the complement of the host's) into the host output,
    // unless the kernel wrote them there itself
    for (int slot = 0; slot < n_out_slots() && use_gpu() && out[slot].host_out; ++slot) {
      if (gpu_out[slot] == out[slot].host_dev) continue;
      uint64_t cur = 0;
      auto copy = [&](uint64_t a, uint64_t b) -> ce_status {
        size_t off, len;
        bytes_of(a, b, &off, &len);
        if (!len) return CE_OK;
        hipError_t e2 = hipMemcpyAsync((char*)out[slot].host_out + off, (const char*)gpu_out[slot] + off, len,
                                       hipMemcpyDeviceToHost, stream);
        if (e2 != hipSuccess) return hip_fail(e2, "merge: device ranges to host");
        issued = true;
        return CE_OK;
      };
      for (auto& iv : hiv) {
        if (iv.first > cur) {
          ce_status s = copy(cur, iv.first);
          if (s != CE_OK) return s;
        }
        cur = iv.second;
      }
      if (cur < G) {
        ce_status s = copy(cur, G);
        if (s != CE_OK) return s;
      }
    }
    // host output came from a scratch buffer while the caller gave a host pointer: impossible
    // (host workers write into out.host when given). Device output scratch with a dev pointer: impossible.
    if (issued) {
      if ((he = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(he, "merge: sync");
    }
    return CE_OK;
  }

  void fill_stats(uint64_t G, int64_t t_end) {
    ce_run_stats s{};
    s.t_run = (double)(t_end - t0_ns) * 1e-9;
    s.n_devices = n_devices();
    s.total_granules = G;
    s.gpu_workgroups = use_gpu() ? gpu_grid_last : 0;
    auto ph = [&](int64_t t) { return t ? (double)(t - t0_ns) * 1e-9 : 0.0; };
    s.t_launched = ph(ph_launched);
    s.t_host_done = ph(ph_host_done);
    s.t_gpu_seen = ph(ph_gpu_seen);
    s.t_synced = ph(ph_synced);
    s.t_copies_done = ph(ph_copies);
    s.host_threads = use_host() ? (uint32_t)host_threads : 0;
    const int gi = gpu_index(), hi = host_index();
    uint64_t host_items = 0;
    if (gi >= 0) {
      s.device_kind[gi] = CE_DEV_GPU;
      uint64_t np = __atomic_load_n(&l1->gpu_packages, __ATOMIC_ACQUIRE);
      uint64_t gr = __atomic_load_n(&l1->gpu_granules, __ATOMIC_ACQUIRE);
      const uint64_t tf = __atomic_load_n(&l1->gpu_t_first, __ATOMIC_ACQUIRE);
      uint64_t tl = __atomic_load_n(&l1->gpu_t_last, __ATOMIC_ACQUIRE);
      uint64_t tf_l = tf;
      if (light_exit) {
        // no last workgroup summarised the run: the GPU ended when its last
        // workgroup left, and the packages the kernel claimed are counted in
        // its queue state (read back only here, when statistics are asked for)
        const bool pre = fast_g1 > fast_g0;
        tl = 0;
        for (uint32_t i = 0; i < gpu_grid_last; ++i) tl = std::max(tl, __atomic_load_n(&wg_end[i], __ATOMIC_ACQUIRE));
        np = pre ? 1 : 0;
        gr = fast_g1 - fast_g0;
        if (!fast_exit) {
          L2State q;
          if (hipMemcpy(&q, l2_last, sizeof q, hipMemcpyDeviceToHost) == hipSuccess) {
            np += q.n_pkgs;
            gr += q.granules;
            if (!pre) tf_l = q.t_first;
          }
        }
      }
      s.packages[gi] = np;
      s.granules[gi] = gr;
      s.t_device[gi] = np ? std::max(0.0, tick_to_host_s(tl)) : 0.0;
      s.t_gpu_kernel = np ? (double)(tl - tf_l) / (double)wallclock_hz : 0.0;
      const uint64_t tg = __atomic_load_n(&l1->gpu_t_gather, __ATOMIC_ACQUIRE);
      s.t_gather = (gather && tg) ? std::max(0.0, tick_to_host_s(tg)) : 0.0;
      s.gathered_bytes = gather ? __atomic_load_n(&l1->gathered, __ATOMIC_ACQUIRE) : 0;
      if (push) {  // the copies were seen complete after the host's work, at push_end_ns at the latest
        s.t_gather = push_total ? (double)(push_end_ns - t0_ns) * 1e-9 : 0.0;
        s.gathered_bytes = push_total;
      }
      gpu_pkgs_last = np;
    }
    if (hi >= 0) {
      s.device_kind[hi] = CE_DEV_HOST;
      s.packages[hi] = hq.n_pkgs;
      s.granules[hi] = hq.granules;
      int64_t last = 0;
      for (uint32_t i = 0; i < hq.n_pkgs; ++i) {
        last = std::max(last, hq.pkgs[i].t_end.load());
        host_items += items_in(hq.pkgs[i].g0, hq.pkgs[i].g1);
      }
      s.t_device[hi] = hq.n_pkgs ? (double)(last - t0_ns) * 1e-9 : 0.0;
      s.items[hi] = host_items;
    }
    s.total_items = items_in(0, G);
    if (gi >= 0) s.items[gi] = s.total_items - host_items;
    double mn = 1e300, mx = 0.0;
    for (uint32_t d = 0; d < s.n_devices; ++d) {
      mn = std::min(mn, s.t_device[d]);
      mx = std::max(mx, s.t_device[d]);
    }
    s.balance = mx > 0.0 ? mn / mx : 0.0;
    stats = s;
    stats_valid = true;
  }

  size_t build_trace() {
    trace.clear();
    const int gi = gpu_index(), hi = host_index();
    if (gi >= 0 && gpu_pkgs_last && fast_exit) {
      // the one pre-claimed package: its record is the host's own
      uint64_t tl = 0;
      for (uint32_t i = 0; i < gpu_grid_last; ++i) tl = std::max(tl, __atomic_load_n(&wg_end[i], __ATOMIC_ACQUIRE));
      const uint64_t tf = __atomic_load_n(&l1->gpu_t_first, __ATOMIC_ACQUIRE);
      trace.push_back(ce_package_rec{(uint32_t)gi, 0, fast_g0, fast_g1, tick_to_host_s(tf), tick_to_host_s(tl)});
    } else if (gi >= 0 && gpu_pkgs_last) {
      std::vector<PkgSlot> v(std::min<uint64_t>(gpu_pkgs_last, trace_pkgs_cap));
      if (hipMemcpy(v.data(), trace_pkgs, v.size() * sizeof(PkgSlot), hipMemcpyDeviceToHost) == hipSuccess) {
        // with the light exit no last workgroup filled in the range of the
        // package claimed before the launch: the host knows it
        if (light_exit && fast_g1 > fast_g0 && !v.empty()) {
          v[0].g0 = fast_g0;
          v[0].g1 = fast_g1;
        }
        for (auto& p : v)
          trace.push_back(ce_package_rec{(uint32_t)gi, 0, p.g0, p.g1, tick_to_host_s(p.t_claim), tick_to_host_s(p.t_end)});
      }
    }
    if (hi >= 0) {
      for (uint32_t i = 0; i < hq.n_pkgs; ++i) {
        const HostPkg& p = hq.pkgs[i];
        trace.push_back(ce_package_rec{(uint32_t)hi, 0, p.g0, p.g1, (double)(p.t_claim - t0_ns) * 1e-9,
                                       (double)(p.t_end.load() - t0_ns) * 1e-9});
      }
    }
    return trace.size();
  }

  // ------------------------------------------------------------ init
  ce_status init() {
    hipError_t he;
    int count = 0;
    if ((he = hipGetDeviceCount(&count)) != hipSuccess || count <= 0)
      return fail(CE_E_DEVICE, "create: no HIP device (%s)", hipGetErrorString(he));
    if ((he = hipGetDevice(&gpu)) != hipSuccess) return hip_fail(he, "create: hipGetDevice");
    hipDeviceProp_t prop;
    if ((he = hipGetDeviceProperties(&prop, gpu)) != hipSuccess) return hip_fail(he, "create: properties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(CE_E_DEVICE, "create: GPU %s is not gfx950", prop.gcnArchName);
    n_cu = prop.multiProcessorCount;
    int clk = 0;
    if (hipDeviceGetAttribute(&clk, hipDeviceAttributeWallClockRate, gpu) == hipSuccess && clk > 0)
      wallclock_hz = (uint32_t)clk * 1000u;
    if (!sdma.init(gpu, sdma_why, sizeof(sdma_why))) merge_mode = CE_MERGE_GPU_GATHER;
    if ((he = hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(he, "create: stream");
    stream = own_stream;
    void* p = nullptr;
    if ((he = hipHostMalloc(&p, sizeof(L1State), hipHostMallocCoherent | hipHostMallocMapped)) != hipSuccess)
      return hip_fail(he, "create: coherent host memory");
    l1 = (L1State*)p;
    memset(l1, 0, sizeof(L1State));
    if ((he = hipHostGetDevicePointer((void**)&l1_dev, l1, 0)) != hipSuccess)
      return hip_fail(he, "create: device view of host memory");
    if ((he = hipHostMalloc(&p, kFastExitMaxWgs * sizeof(uint64_t), hipHostMallocCoherent | hipHostMallocMapped)) !=
        hipSuccess)
      return hip_fail(he, "create: coherent host memory");
    wg_end = (uint64_t*)p;
    memset(wg_end, 0, kFastExitMaxWgs * sizeof(uint64_t));
    if ((he = hipHostGetDevicePointer((void**)&wg_end_dev, wg_end, 0)) != hipSuccess)
      return hip_fail(he, "create: device view of host memory");
    if ((he = hipMalloc((void**)&l2, 2 * sizeof(L2State))) != hipSuccess) return hip_fail(he, "create: queue state");
    // the null stream's clear must be done before any run's kernel, which
    // goes to a stream that does not wait for the null stream
    if ((he = hipMemset(l2, 0, 2 * sizeof(L2State))) != hipSuccess || (he = hipDeviceSynchronize()) != hipSuccess)
      return hip_fail(he, "create: queue state");
    // the allocation-free run's scratch on this GPU (a failure only disables that run)
    noalloc_err = noalloc_scratch_address(gpu, &noalloc_base);
    hp = host_payloads();
    host_threads = (int)std::max(1u, std::thread::hardware_concurrency());
    calibrate_clock();
    return CE_OK;
  }

  // GPU tick -> host clock: the GPU answers pings through host-coherent
  // memory; the round trip with the smallest latency gives the offset.
  void calibrate_clock() {
    const uint32_t rounds = 64;
    __atomic_store_n(&l1->ping, 0, __ATOMIC_RELEASE);
    __atomic_store_n(&l1->pong, 0, __ATOMIC_RELEASE);
    if (launch_calibrate(l1_dev, rounds, 1ull << 24, stream) != hipSuccess) return;
    double best_rt = 1e300, best_ns = 0.0;
    uint64_t best_tick = 0;
    bool ok = true;
    for (uint32_t i = 1; i <= rounds && ok; ++i) {
      const int64_t ta = now_ns();
      __atomic_store_n(&l1->ping, (uint64_t)i, __ATOMIC_RELEASE);
      for (;;) {
        if (__atomic_load_n(&l1->pong, __ATOMIC_ACQUIRE) == i) break;
        if (now_ns() - ta > 2'000'000'000LL) {
          ok = false;
          break;
        }
        cpu_relax();
      }
      const int64_t tb = now_ns();
      if (!ok) break;
      const uint64_t tick = __atomic_load_n(&l1->tick, __ATOMIC_ACQUIRE);
      const double rt = (double)(tb - ta);
      if (rt < best_rt) {
        best_rt = rt;
        best_ns = 0.5 * (double)(ta + tb);
        best_tick = tick;
      }
    }
    // unblock the kernel if the host gave up early
    __atomic_store_n(&l1->ping, 0xFFFFFFFFull, __ATOMIC_RELEASE);
    (void)hipStreamSynchronize(stream);
    clock_ok = ok;
    if (ok) {
      ns_per_tick = 1e9 / (double)wallclock_hz;
      anchor0_tick = anchor_tick = best_tick;
      anchor0_ns = anchor_ns = best_ns;
      clock_latency_ns = 0.5 * best_rt;
    }
    else errors.emplace_back("create: GPU clock calibration failed; GPU times are unmapped");
  }

  ~ce_engine() {
    pool_stop();
    if (stream) (void)hipStreamSynchronize(stream);
    rt_release(rt_module);
    // SdmaCopier's destructor waits for copies still queued
    if (own_stream) (void)hipStreamDestroy(own_stream);
    if (l2) (void)hipFree(l2);
    if (l1) (void)hipHostFree(l1);
    if (wg_end) (void)hipHostFree(wg_end);
  }
};

// =================================================================== C ABI
extern "C" {

ce_status ce_engine_create(ce_engine** out) {
  if (!out) return CE_E_INVALID;
  *out = nullptr;
  try {
    ce_engine* e = new ce_engine();
    ce_status st = e->init();
    if (st != CE_OK) {
      delete e;
      return st;
    }
    *out = e;
    return CE_OK;
  } catch (...) {
    return CE_E_NOMEM;
  }
}

void ce_engine_destroy(ce_engine* e) { delete e; }

ce_status ce_engine_use(ce_engine* e, uint32_t dev_mask, int gpu_ordinal, int host_threads) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (dev_mask == 0 || (dev_mask & ~(CE_DEV_GPU | CE_DEV_HOST)))
    return e->fail(CE_E_INVALID, "use: device mask 0x%x", dev_mask);
  if ((dev_mask & CE_DEV_GPU) && gpu_ordinal != e->gpu)
    return e->fail(CE_E_INVALID, "use: GPU ordinal %d is not the engine's GPU %d", gpu_ordinal, e->gpu);
  if ((dev_mask & CE_DEV_HOST) && !e->hp) return e->fail(CE_E_UNSUPPORTED, "use: host CPU lacks AVX2/FMA");
  e->dev_mask = dev_mask;
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  e->host_threads = host_threads <= 0 ? hw : std::min(host_threads, 1024);
  return CE_OK;
}

ce_status ce_engine_work_items(ce_engine* e, uint32_t ndim, const uint64_t* gws, const uint32_t* lws) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (ndim < 1 || ndim > 2 || !gws) return e->fail(CE_E_INVALID, "work_items: ndim must be 1 or 2");
  for (uint32_t d = 0; d < ndim; ++d)
    if (gws[d] == 0 || gws[d] > 0xFFFFFFFFull) return e->fail(CE_E_INVALID, "work_items: gws[%u] out of range", d);
  e->ndim = ndim;
  e->gws[0] = gws[0];
  e->gws[1] = ndim > 1 ? gws[1] : 1;
  e->lws0 = (lws && lws[0]) ? lws[0] : 256;
  return CE_OK;
}

ce_status ce_engine_scheduler(ce_engine* e, const ce_sched_desc* s) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (!s) return e->fail(CE_E_INVALID, "scheduler: NULL descriptor");
  if (s->kind < CE_SCHED_STATIC || s->kind > CE_SCHED_HGUIDED)
    return e->fail(CE_E_INVALID, "scheduler: unknown kind %d", s->kind);
  if (s->order != CE_ORDER_HOST_FIRST && s->order != CE_ORDER_GPU_FIRST)
    return e->fail(CE_E_INVALID, "scheduler: unknown order %d", s->order);
  if (s->n_packages > (1u << 20)) return e->fail(CE_E_INVALID, "scheduler: too many packages");
  e->sched = *s;
  e->sched_set = true;
  return CE_OK;
}

ce_status ce_engine_stream(ce_engine* e, void* hip_stream) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  e->stream = hip_stream ? (hipStream_t)hip_stream : e->own_stream;
  return CE_OK;
}

ce_status ce_engine_output_merge(ce_engine* e, int mode) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (mode != CE_MERGE_DMA && mode != CE_MERGE_GPU_GATHER) return e->fail(CE_E_INVALID, "output_merge: mode %d", mode);
  if (mode == CE_MERGE_DMA && !e->sdma.ready())
    return e->fail(CE_E_UNSUPPORTED, "output_merge: no DMA engine (%s)", e->sdma_why);
  e->merge_mode = mode;
  return CE_OK;
}

ce_status ce_engine_wait_bounds(ce_engine* e, double dispenser_s, double gather_s) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (!(dispenser_s >= 0.0 && dispenser_s <= 3600.0) || !(gather_s >= 0.0 && gather_s <= 3600.0))
    return e->fail(CE_E_INVALID, "wait_bounds: each bound must lie in [0, 3600] s");
  e->dispenser_wait_s = dispenser_s > 0.0 ? dispenser_s : (double)kDispenserWaitSeconds;
  e->gather_wait_s = gather_s > 0.0 ? gather_s : (double)kGatherWaitSeconds;
  return CE_OK;
}

ce_status ce_engine_gpu_workgroups(ce_engine* e, uint32_t workgroups) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (workgroups > (1u << 20)) return e->fail(CE_E_INVALID, "gpu_workgroups: %u is above 2^20", workgroups);
  e->grid_override = workgroups;
  return CE_OK;
}

ce_status ce_engine_kernel_events(ce_engine* e, void* start_event, void* stop_event) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if ((start_event == nullptr) != (stop_event == nullptr))
    return e->fail(CE_E_INVALID, "kernel_events: give both events or neither");
  e->ev_start = (hipEvent_t)start_event;
  e->ev_stop = (hipEvent_t)stop_event;
  return CE_OK;
}

ce_status ce_program_kernel(ce_engine* e, int kernel_id, const void* params, size_t params_size) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (!params) return e->fail(CE_E_INVALID, "kernel: NULL params");
  switch (kernel_id) {
    case CE_KERNEL_ESCAPE: {
      if (params_size != sizeof(ce_escape_params)) return e->fail(CE_E_INVALID, "kernel: escape params size");
      ce_escape_params p;
      memcpy(&p, params, sizeof p);
      if (p.w == 0 || p.h == 0) return e->fail(CE_E_INVALID, "kernel: empty escape grid");
      e->esc = p;
      break;
    }
    case CE_KERNEL_BLUR5: {
      if (params_size != sizeof(ce_blur5_params)) return e->fail(CE_E_INVALID, "kernel: blur params size");
      ce_blur5_params p;
      memcpy(&p, params, sizeof p);
      if (p.w == 0 || p.h == 0) return e->fail(CE_E_INVALID, "kernel: empty image");
      e->blur = p;
      break;
    }
    case CE_KERNEL_NBODY_ACC: {
      if (params_size != sizeof(ce_nbody_params)) return e->fail(CE_E_INVALID, "kernel: n-body params size");
      ce_nbody_params p;
      memcpy(&p, params, sizeof p);
      if (p.n == 0) return e->fail(CE_E_INVALID, "kernel: no bodies");
      if (!(p.eps2 >= 1.17549435e-38f) || !std::isfinite(p.eps2))
        return e->fail(CE_E_INVALID, "kernel: eps2 must be a positive normal float");
      e->nb = p;
      break;
    }
    case CE_KERNEL_BINOMIAL: {
      if (params_size != sizeof(ce_binomial_params)) return e->fail(CE_E_INVALID, "kernel: binomial params size");
      ce_binomial_params p;
      memcpy(&p, params, sizeof p);
      if (p.n_groups == 0) return e->fail(CE_E_INVALID, "kernel: no option groups");
      if (p.steps == 0 || p.steps + 1 > kBlockThreads)
        return e->fail(CE_E_INVALID, "kernel: binomial steps must be in [1, %u]", kBlockThreads - 1);
      if (!std::isfinite(p.strike) || !std::isfinite(p.pu) || !std::isfinite(p.pd))
        return e->fail(CE_E_INVALID, "kernel: binomial strike and probabilities must be finite");
      e->bin = p;
      break;
    }
    case CE_KERNEL_NBODY_STEP: {
      if (params_size != sizeof(ce_nbody_step_params)) return e->fail(CE_E_INVALID, "kernel: n-body step params size");
      ce_nbody_step_params p;
      memcpy(&p, params, sizeof p);
      if (p.n == 0) return e->fail(CE_E_INVALID, "kernel: no bodies");
      if (!(p.eps2 >= 1.17549435e-38f) || !std::isfinite(p.eps2))
        return e->fail(CE_E_INVALID, "kernel: eps2 must be a positive normal float");
      if (!std::isfinite(p.dt)) return e->fail(CE_E_INVALID, "kernel: dt must be finite");
      e->nbs = p;
      break;
    }
    default: return e->fail(CE_E_INVALID, "kernel: unknown kernel id %d", kernel_id);
  }
  e->kernel_id = kernel_id;
  for (auto& b : e->in) b = Binding{};
  for (auto& b : e->out) b = Binding{};
  return CE_OK;
}

ce_status ce_program_in(ce_engine* e, uint32_t slot, const void* host_ptr, const void* dev_ptr, size_t bytes) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (e->kernel_id == 0) return e->fail(CE_E_STATE, "in: bind a kernel first");
  if ((int)slot >= e->n_in_slots()) return e->fail(CE_E_INVALID, "in: kernel has no input slot %u", slot);
  if (!host_ptr && !dev_ptr) return e->fail(CE_E_INVALID, "in: slot %u needs a host or device pointer", slot);
  if (bytes != e->in_bytes((int)slot))
    return e->fail(CE_E_INVALID, "in: slot %u expects %zu bytes, got %zu", slot, e->in_bytes((int)slot), bytes);
  e->in[slot] = Binding{host_ptr, dev_ptr, nullptr, nullptr, bytes, true, dev_ptr ? nullptr : pinned_device_view(host_ptr)};
  return CE_OK;
}

ce_status ce_program_out(ce_engine* e, uint32_t slot, void* host_ptr, void* dev_ptr, size_t bytes) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (e->kernel_id == 0) return e->fail(CE_E_STATE, "out: bind a kernel first");
  if ((int)slot >= e->n_out_slots()) return e->fail(CE_E_INVALID, "out: kernel has no output slot %u", slot);
  if (!host_ptr && !dev_ptr) return e->fail(CE_E_INVALID, "out: needs a host or device pointer");
  if (bytes != e->out_bytes()) return e->fail(CE_E_INVALID, "out: expects %zu bytes, got %zu", e->out_bytes(), bytes);
  e->out[slot] = Binding{nullptr, nullptr, host_ptr, dev_ptr, bytes, true, dev_ptr ? nullptr : pinned_device_view(host_ptr)};
  return CE_OK;
}

ce_status ce_program_out_pattern(ce_engine* e, uint32_t outs, uint32_t items) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (outs == 0 || items == 0) return e->fail(CE_E_INVALID, "out_pattern: zero term");
  // the pattern is fixed by the payload: 1:(steps+1) for binomial, 1:1 otherwise
  const uint32_t want = e->kernel_id == CE_KERNEL_BINOMIAL ? e->bin.steps + 1 : 1;
  if (outs != 1 || items != want)
    return e->fail(CE_E_UNSUPPORTED, "out_pattern: this payload writes 1 output per %u work-items", want);
  e->pat_outs = outs;
  e->pat_items = items;
  return CE_OK;
}

namespace {
void copy_log(const std::string& text, char* log, size_t log_len) {
  if (!log || log_len == 0) return;
  const size_t n = std::min(text.size(), log_len - 1);
  memcpy(log, text.data(), n);
  log[n] = '\0';
}
}  // namespace

ce_status ce_rt_compile_check(const char* source, const char* entry, char* log, size_t log_len) {
  std::string code, lp, lb, ld, text;
  const int rc = rt_compile(source, entry, &code, &lp, &lb, &ld, &text);
  copy_log(text, log, log_len);
  return rc == 0 ? CE_OK : (rc == -1 ? CE_E_INVALID : CE_E_DEVICE);
}

ce_status ce_rt_code_object(const char* source, const char* entry, void* buf, size_t cap, size_t* size, char* log,
                            size_t log_len) {
  if (!size) return CE_E_INVALID;
  *size = 0;
  std::string code, lp, lb, ld, text;
  const int rc = rt_compile(source, entry, &code, &lp, &lb, &ld, &text);
  copy_log(text, log, log_len);
  if (rc != 0) return rc == -1 ? CE_E_INVALID : CE_E_DEVICE;
  *size = code.size();
  if (buf && cap >= code.size()) memcpy(buf, code.data(), code.size());
  return CE_OK;
}

ce_status ce_program_source(ce_engine* e, const ce_rt_desc* d, char* log, size_t log_len) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  copy_log("", log, log_len);
  if (!d || !d->source || !d->entry) return e->fail(CE_E_INVALID, "source: NULL descriptor, source or entry");
  if (d->n_in > 2 || d->n_out < 1 || d->n_out > 2)
    return e->fail(CE_E_INVALID, "source: 0..2 inputs and 1..2 outputs (got %u, %u)", d->n_in, d->n_out);
  if (d->out_item_bytes == 0 || d->out_item_bytes > 256)
    return e->fail(CE_E_INVALID, "source: out_item_bytes must be in [1, 256]");
  if (d->scalar_bytes > CE_RT_SCALAR_BYTES || (d->scalar_bytes && !d->scalars))
    return e->fail(CE_E_INVALID, "source: at most %d scalar bytes", CE_RT_SCALAR_BYTES);
  for (uint32_t k = 0; k < d->n_in; ++k)
    if (d->in_bytes[k] == 0) return e->fail(CE_E_INVALID, "source: input %u has no bytes", k);
  // the previous payload is unbound whatever happens next
  e->kernel_id = 0;
  for (auto& b : e->in) b = Binding{};
  for (auto& b : e->out) b = Binding{};
  rt_release(e->rt_module);
  e->rt_module = e->rt_fn_persistent = e->rt_fn_bare = e->rt_fn_direct = nullptr;
  std::string text;
  const int rc =
      rt_build(d->source, d->entry, &e->rt_module, &e->rt_fn_persistent, &e->rt_fn_bare, &e->rt_fn_direct, &text);
  copy_log(text, log, log_len);
  if (rc != 0) {
    if (rc == -1) return e->fail(CE_E_INVALID, "source: the payload did not compile (see the log)");
    return e->fail(CE_E_DEVICE, "source: hipRTC or module load failed: %s", text.c_str());
  }
  e->rt_host = d->host;
  e->rt_n_in = d->n_in;
  e->rt_n_out = d->n_out;
  e->rt_item_bytes = d->out_item_bytes;
  e->rt_in_bytes[0] = d->n_in > 0 ? d->in_bytes[0] : 0;
  e->rt_in_bytes[1] = d->n_in > 1 ? d->in_bytes[1] : 0;
  memset(e->rt_scalars, 0, sizeof e->rt_scalars);
  if (d->scalar_bytes) memcpy(e->rt_scalars, d->scalars, d->scalar_bytes);
  // a new module: its occupancy is asked afresh
  for (int k = 0; k < 2; ++k)
    if (CE_KERNEL_RUNTIME * 2 + k < ce_engine::kOccSlots) e->occ_cache[CE_KERNEL_RUNTIME * 2 + k] = 0;
  e->kernel_id = CE_KERNEL_RUNTIME;
  return CE_OK;
}

ce_status ce_engine_bare_run_source(ce_engine* e, uint64_t gws, uint32_t lws, const void* const* ins,
                                    void* const* outs, void* hip_stream, int sync) {
  if (!e) return CE_E_INVALID;
  e->ensure_stats();  // the last run's statistics, before its settings change
  if (e->kernel_id != CE_KERNEL_RUNTIME || !e->rt_fn_bare) return e->fail(CE_E_STATE, "bare: no runtime payload bound");
  if (gws == 0 || lws == 0 || !outs) return e->fail(CE_E_INVALID, "bare: empty space or no outputs");
  KernelArgs a{};
  a.kernel_id = CE_KERNEL_RUNTIME;
  for (uint32_t k = 0; k < e->rt_n_in; ++k) {
    if (!ins || !ins[k]) return e->fail(CE_E_INVALID, "bare: input %u missing", k);
    a.rt.buf[k] = const_cast<void*>(ins[k]);
  }
  for (uint32_t k = 0; k < e->rt_n_out; ++k) {
    if (!outs[k]) return e->fail(CE_E_INVALID, "bare: output %u missing", k);
    a.rt.buf[e->rt_n_in + k] = outs[k];
  }
  memcpy(a.rt.scalars, e->rt_scalars, sizeof e->rt_scalars);
  a.rt_items = gws;
  a.rt_lws = lws;
  a.rt_item_bytes = e->rt_item_bytes;
  a.rt_fn_persistent = e->rt_fn_persistent;
  a.rt_fn_bare = e->rt_fn_bare;
  a.rt_fn_direct = e->rt_fn_direct;
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t he;
  if ((he = launch_bare(a, st)) != hipSuccess) return e->hip_fail(he, "bare: launch");
  if (sync && (he = hipStreamSynchronize(st)) != hipSuccess) return e->hip_fail(he, "bare: sync");
  return CE_OK;
}

ce_status ce_engine_run_noalloc(ce_engine* e) {
  if (!e) return CE_E_INVALID;
  try {
    e->noalloc = true;
    return e->run();
  } catch (const std::exception& ex) {
    e->noalloc = false;
    return e->fail(CE_E_NOMEM, "run_noalloc: %s", ex.what());
  } catch (...) {
    e->noalloc = false;
    return e->fail(CE_E_NOMEM, "run_noalloc: unknown exception");
  }
}

ce_status ce_engine_run(ce_engine* e) {
  if (!e) return CE_E_INVALID;
  try {
    return e->run();
  } catch (const std::exception& ex) {
    return e->fail(CE_E_NOMEM, "run: %s", ex.what());
  } catch (...) {
    return e->fail(CE_E_NOMEM, "run: unknown exception");
  }
}

ce_status ce_engine_stats(const ce_engine* ce, ce_run_stats* out) {
  if (!ce || !out) return CE_E_INVALID;
  ce_engine* e = const_cast<ce_engine*>(ce);
  e->ensure_stats();
  if (!e->stats_valid) return CE_E_STATE;
  *out = e->stats;
  return CE_OK;
}

size_t ce_engine_trace(const ce_engine* ce, ce_package_rec* buf, size_t cap) {
  if (!ce) return 0;
  ce_engine* e = const_cast<ce_engine*>(ce);
  e->ensure_stats();
  if (!e->stats_valid) return 0;
  size_t n = 0;
  try {
    n = e->build_trace();
  } catch (...) {
    return 0;
  }
  if (buf)
    for (size_t i = 0; i < std::min(n, cap); ++i) buf[i] = e->trace[i];
  return n;
}

int ce_engine_has_errors(const ce_engine* e) { return e && !e->errors.empty(); }
int ce_engine_error_count(const ce_engine* e) { return e ? (int)e->errors.size() : 0; }
const char* ce_engine_error(const ce_engine* e, int i) {
  if (!e || i < 0 || i >= (int)e->errors.size()) return nullptr;
  return e->errors[(size_t)i].c_str();
}
void ce_engine_clear_errors(ce_engine* e) {
  if (e) e->errors.clear();
}

ce_status ce_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream, int sync) {
  if (!dst || !src || (bytes % 16) != 0 || ((uintptr_t)dst % 16) != 0 || ((uintptr_t)src % 16) != 0)
    return CE_E_INVALID;
  hipStream_t st = (hipStream_t)hip_stream;
  if (launch_stream_copy(dst, src, bytes / 16, st) != hipSuccess) return CE_E_DEVICE;
  if (sync && hipStreamSynchronize(st) != hipSuccess) return CE_E_DEVICE;
  return CE_OK;
}

ce_status ce_bare_run(int kernel_id, const void* params, size_t params_size, const void* const* ins, void* out,
                      void* hip_stream, int sync) {
  void* const outs[1] = {out};
  return ce_bare_run_outs(kernel_id, params, params_size, ins, outs, 1, hip_stream, sync);
}

ce_status ce_bare_run_outs(int kernel_id, const void* params, size_t params_size, const void* const* ins,
                           void* const* outs, uint32_t n_outs, void* hip_stream, int sync) {
  if (!params || !outs || !outs[0]) return CE_E_INVALID;
  if (n_outs != (kernel_id == CE_KERNEL_NBODY_STEP ? 2u : 1u)) return CE_E_INVALID;
  void* const out = outs[0];
  KernelArgs a{};
  a.kernel_id = kernel_id;
  switch (kernel_id) {
    case CE_KERNEL_ESCAPE:
      if (params_size != sizeof(ce_escape_params)) return CE_E_INVALID;
      memcpy(&a.esc, params, sizeof a.esc);
      if (a.esc.w == 0 || a.esc.h == 0) return CE_E_INVALID;
      break;
    case CE_KERNEL_BLUR5:
      if (params_size != sizeof(ce_blur5_params) || !ins || !ins[0] || !ins[1]) return CE_E_INVALID;
      memcpy(&a.blur, params, sizeof a.blur);
      if (a.blur.w == 0 || a.blur.h == 0) return CE_E_INVALID;
      a.in0 = ins[0];
      a.in1 = ins[1];
      break;
    case CE_KERNEL_NBODY_ACC:
      if (params_size != sizeof(ce_nbody_params) || !ins || !ins[0]) return CE_E_INVALID;
      memcpy(&a.nb, params, sizeof a.nb);
      if (a.nb.n == 0 || !(a.nb.eps2 >= 1.17549435e-38f)) return CE_E_INVALID;
      a.strict = a.nb.strict;
      a.in0 = ins[0];
      break;
    case CE_KERNEL_BINOMIAL:
      if (params_size != sizeof(ce_binomial_params) || !ins || !ins[0] || !ins[1]) return CE_E_INVALID;
      memcpy(&a.bin, params, sizeof a.bin);
      if (a.bin.n_groups == 0 || a.bin.steps == 0 || a.bin.steps + 1 > kBlockThreads) return CE_E_INVALID;
      a.in0 = ins[0];
      a.in1 = ins[1];
      break;
    case CE_KERNEL_NBODY_STEP:
      if (params_size != sizeof(ce_nbody_step_params) || !ins || !ins[0] || !ins[1] || !outs[1]) return CE_E_INVALID;
      memcpy(&a.nbs, params, sizeof a.nbs);
      if (a.nbs.n == 0 || !(a.nbs.eps2 >= 1.17549435e-38f) || !std::isfinite(a.nbs.dt)) return CE_E_INVALID;
      a.strict = a.nbs.strict;
      a.in0 = ins[0];
      a.in1 = ins[1];
      a.out1 = outs[1];
      break;
    default: return CE_E_INVALID;
  }
  a.out = out;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return CE_E_DEVICE;
  hipStream_t st = (hipStream_t)hip_stream;
  if (launch_bare(a, st) != hipSuccess) return CE_E_DEVICE;
  if (sync && hipStreamSynchronize(st) != hipSuccess) return CE_E_DEVICE;
  return CE_OK;
}

ce_status ce_sched_static_plan(uint64_t G, uint32_t n, const double* props, const uint32_t* order, uint32_t n_bands,
                               uint64_t* begin, uint64_t* end) {
  if (n == 0 || n > CE_MAX_DEVICES || !order || !begin || !end || (n > 1 && !props)) return CE_E_INVALID;
  double share[CE_MAX_DEVICES];
  double rest = 1.0;
  for (uint32_t d = 0; d + 1 < n; ++d) {
    if (!(props[d] >= 0.0) || props[d] > 1.0) return CE_E_INVALID;
    share[d] = props[d];
    rest -= props[d];
  }
  if (rest < -1e-12) return CE_E_INVALID;
  share[n - 1] = rest < 0.0 ? 0.0 : rest;
  bool seen[CE_MAX_DEVICES] = {false, false};
  for (uint32_t k = 0; k < n; ++k) {
    if (order[k] >= n || seen[order[k]]) return CE_E_INVALID;
    seen[order[k]] = true;
  }
  if (n_bands == 0) {
    double cum = 0.0;
    uint64_t prev = 0;
    for (uint32_t k = 0; k < n; ++k) {
      const uint32_t d = order[k];
      cum += share[d];
      uint64_t b = (k + 1 == n) ? G : (uint64_t)std::floor(cum * (double)G);
      b = std::min(b, G);
      b = std::max(b, prev);
      begin[d] = prev;
      end[d] = b;
      prev = b;
    }
    return CE_OK;
  }
  if (n_bands < n || (uint64_t)n_bands > G) return CE_E_INVALID;
  uint64_t nb[CE_MAX_DEVICES];
  uint64_t used = 0;
  for (uint32_t d = 0; d + 1 < n; ++d) {
    const double r = std::floor(share[d] * (double)n_bands + 0.5);
    const uint64_t want = r < 1.0 ? 1 : (uint64_t)r;
    const uint64_t cap = n_bands - used - (n - 1 - d);
    nb[d] = std::min(want, cap);
    used += nb[d];
  }
  nb[n - 1] = n_bands - used;
  uint64_t band = 0;
  for (uint32_t k = 0; k < n; ++k) {
    const uint32_t d = order[k];
    begin[d] = band_edge(band, G, n_bands);
    band += nb[d];
    end[d] = band_edge(band, G, n_bands);
  }
  return CE_OK;
}

uint64_t ce_sched_hguided_size(uint64_t G_r, const uint64_t* power, uint32_t n, uint32_t k, uint32_t i,
                               uint64_t min_i) {
  if (!power || n == 0 || i >= n) return 0;
  uint64_t sumP = 0;
  for (uint32_t j = 0; j < n; ++j) sumP += power[j];
  return hguided_size(G_r, power[i], sumP, n, k, min_i);
}

ce_status ce_gauss5_weights(double sigma, float* w25) {
  if (!w25 || !(sigma > 0.0)) return CE_E_INVALID;
  double e[25], sum = 0.0;
  for (int dy = -2; dy <= 2; ++dy)
    for (int dx = -2; dx <= 2; ++dx) {
      const double v = std::exp(-(double)(dx * dx + dy * dy) / (2.0 * sigma * sigma));
      e[(dy + 2) * 5 + dx + 2] = v;
      sum += v;
    }
  for (int k = 0; k < 25; ++k) w25[k] = (float)(e[k] / sum);
  return CE_OK;
}

ce_status ce_binomial_table(uint32_t steps, double sigma, double rate, double T, float* factors, float* pu,
                            float* pd) {
  if (!factors || !pu || !pd || steps == 0 || !(sigma > 0.0) || !(T > 0.0) || !std::isfinite(rate))
    return CE_E_INVALID;
  const double dt = T / (double)steps;
  const double lu = sigma * std::sqrt(dt);
  const double u = std::exp(lu);
  const double d = 1.0 / u;
  const double p = (std::exp(rate * dt) - d) / (u - d);
  const double disc = std::exp(-rate * dt);
  *pu = (float)(disc * p);
  *pd = (float)(disc * (1.0 - p));
  for (uint32_t j = 0; j <= steps; ++j) factors[j] = (float)std::exp(lu * ((double)(2 * (int64_t)j) - (double)steps));
  return CE_OK;
}

const char* ce_version(void) { return "coexec-mi355x 0.1 (gfx950)"; }

}  // extern "C"
