// Serving form: continuous batching of co-execution jobs on the GPU.
//
// A session is one persistent serving kernel (serve_kernels.hip) that runs
// every job admitted while it lives. Clients submit jobs from any thread; a
// server thread admits them in arrival order as soon as an in-flight slot and
// enough of the HBM budget are free (the job's output, and its inputs when
// they come from host memory, are placed in one device arena), publishes them
// in the job ring, and watches the completion words the kernel writes. Jobs
// admitted while others run share the device tile by tile. Buffers stay in
// HBM until the client releases them (or, without keep_outputs, as soon as the
// job finishes). Latency is measured from submission to the moment the
// server thread sees the job's completion word.
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
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/coexec.h"
#include "common.hpp"
#include "serve.hpp"

using namespace ce;

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over one device allocation (offsets, 256-byte aligned).
struct Arena {
  char* base = nullptr;
  uint64_t size = 0, used = 0, peak = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  void reset() {
    free_.clear();
    if (size) free_[0] = size;
    used = 0;
  }
  bool alloc(uint64_t n, uint64_t* off) {
    n = (n + 255) & ~255ull;
    if (n == 0) n = 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, o = it->first + n;
        free_.erase(it);
        if (rest) free_[o] = rest;
        used += n;
        peak = std::max(peak, used);
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = (n + 255) & ~255ull;
    if (n == 0) n = 256;
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// Pinned staging for copies between pageable client memory and HBM while
// the serving kernel runs: the client's buffer is copied through two pinned
// halves by the CPU, and the DMA side only ever sees pinned memory.
struct Staging {
  static constexpr size_t kHalf = 16u << 20;
  char* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t init() {
    hipError_t he;
    for (int i = 0; i < 2; ++i) {
      if ((he = hipHostMalloc((void**)&buf[i], kHalf, hipHostMallocDefault)) != hipSuccess) return he;
      if ((he = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming)) != hipSuccess) return he;
    }
    return hipSuccess;
  }
  void destroy() {
    for (int i = 0; i < 2; ++i) {
      if (ev[i]) (void)hipEventDestroy(ev[i]);
      if (buf[i]) (void)hipHostFree(buf[i]);
    }
  }
  hipError_t to_device(void* dst, const void* src, size_t n, hipStream_t st) {
    hipError_t he = hipSuccess;
    bool used[2] = {false, false};
    for (size_t off = 0, k = 0; off < n; off += kHalf, ++k) {
      const int b = (int)(k & 1);
      const size_t len = std::min(kHalf, n - off);
      if (used[b] && (he = hipEventSynchronize(ev[b])) != hipSuccess) return he;  // this half was sent
      memcpy(buf[b], (const char*)src + off, len);
      if ((he = hipMemcpyAsync((char*)dst + off, buf[b], len, hipMemcpyHostToDevice, st)) != hipSuccess) return he;
      if ((he = hipEventRecord(ev[b], st)) != hipSuccess) return he;
      used[b] = true;
    }
    return hipStreamSynchronize(st);
  }
  hipError_t to_host(void* dst, const void* src, size_t n, hipStream_t st) {
    hipError_t he = hipSuccess;
    for (size_t off = 0; off < n; off += kHalf) {
      const size_t len = std::min(kHalf, n - off);
      if ((he = hipMemcpyAsync(buf[0], (const char*)src + off, len, hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (he = hipStreamSynchronize(st)) != hipSuccess)
        return he;
      memcpy((char*)dst + off, buf[0], len);
    }
    return hipSuccess;
  }
};

struct JobRec {
  ce_job job{};
  ServeDesc desc{};
  int32_t state = CE_JOB_QUEUED;
  int64_t t_submit = 0, t_admit = 0, t_done = 0;
  uint64_t tick_first = 0, tick_done = 0;  // GPU ticks: first tile start, last tile end
  std::string why;                        // why the job failed
  uint64_t mem_off = 0, mem_bytes = 0, out_bytes = 0;
  bool has_mem = false;
  uint64_t items = 0;
};

size_t in_bytes_of(const ce_job& j, int slot) {
  if (j.kernel_id == CE_KERNEL_BLUR5) return slot == 0 ? (size_t)j.blur.w * j.blur.h * 4 : (slot == 1 ? 100 : 0);
  if (j.kernel_id == CE_KERNEL_NBODY_ACC) return slot == 0 ? (size_t)j.nb.n * 16 : 0;
  return 0;
}
size_t out_bytes_of(const ce_job& j) {
  switch (j.kernel_id) {
    case CE_KERNEL_ESCAPE: return (size_t)j.esc.w * j.esc.h * 4;
    case CE_KERNEL_BLUR5: return (size_t)j.blur.w * j.blur.h * 4;
    case CE_KERNEL_NBODY_ACC: return (size_t)j.nb.n * 16;
  }
  return 0;
}
uint64_t items_of(const ce_job& j) {
  switch (j.kernel_id) {
    case CE_KERNEL_ESCAPE: return (uint64_t)j.esc.w * j.esc.h;
    case CE_KERNEL_BLUR5: return (uint64_t)j.blur.w * j.blur.h;
    case CE_KERNEL_NBODY_ACC: return j.nb.n;
  }
  return 0;
}

}  // namespace

struct ce_server {
  ce_server_config cfg{};
  hipStream_t stream = nullptr, copy_stream = nullptr;
  bool own_stream = false;
  int n_cu = 0;
  uint32_t wallclock_hz = 100000000;

  // device memory
  Arena arena;
  ServeDesc* table = nullptr;
  uint32_t* tiles_done = nullptr;
  uint64_t* pub = nullptr;
  ServeState* state = nullptr;
  // host-coherent memory
  ServeDesc* ring = nullptr;
  ServeCtl* ctl = nullptr;
  uint64_t* done_words = nullptr;
  uint64_t* first_words = nullptr;
  ServeDesc* ring_dev = nullptr;
  ServeCtl* ctl_dev = nullptr;
  uint64_t* done_dev = nullptr;
  uint64_t* first_dev = nullptr;

  std::mutex mu;
  std::mutex copy_mu;                // serialises use of copy_stream and staging
  Staging staging;
  std::condition_variable cv;
  std::deque<JobRec> jobs;           // by ticket; a deque so references stay valid as jobs are added
  std::deque<uint64_t> pending;      // tickets waiting for admission
  std::vector<uint64_t> inflight;    // tickets admitted, not finished
  std::vector<uint64_t> seq_ticket;  // session sequence -> ticket
  uint64_t session = 0;
  bool session_on = false;
  uint64_t head = 0;                 // jobs published in this session
  uint64_t session_tiles = 0;        // tiles published in this session
  uint32_t grid_ = 0;
  std::thread worker;
  std::atomic<bool> quit{false};
  int64_t t_first_submit = 0, t_last_done = 0;
  uint64_t max_inflight_seen = 0;
  mutable std::mutex err_mu;
  std::string error;

  ce_status fail(ce_status code, const char* fmt, ...) __attribute__((format(printf, 3, 4))) {
    char buf[400];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::lock_guard<std::mutex> lk(err_mu);
    error = buf;
    return code;
  }

  ce_status init(const ce_server_config* c, void* s) {
    cfg = *c;
    if (cfg.max_inflight == 0) cfg.max_inflight = 64;
    if (cfg.max_jobs == 0) cfg.max_jobs = 65536;
    if (cfg.max_jobs > kServeMaxJobs) return fail(CE_E_INVALID, "config: max_jobs above %u", kServeMaxJobs);
    if (cfg.session_timeout_s <= 0.0) cfg.session_timeout_s = 300.0;
    if (cfg.hbm_budget == 0) return fail(CE_E_INVALID, "config: zero HBM budget");
    hipError_t he;
    int count = 0, dev = 0, clk = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(CE_E_DEVICE, "no HIP device");
    if ((he = hipGetDevice(&dev)) != hipSuccess ||
        (he = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
      return fail(CE_E_DEVICE, "device: %s", hipGetErrorString(he));
    if (hipDeviceGetAttribute(&clk, hipDeviceAttributeWallClockRate, dev) == hipSuccess && clk > 0)
      wallclock_hz = (uint32_t)clk * 1000u;
    if (s) {
      stream = (hipStream_t)s;
    } else {
      if ((he = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking)) != hipSuccess)
        return fail(CE_E_DEVICE, "stream: %s", hipGetErrorString(he));
      own_stream = true;
    }
    if ((he = hipStreamCreateWithFlags(&copy_stream, hipStreamNonBlocking)) != hipSuccess)
      return fail(CE_E_DEVICE, "stream: %s", hipGetErrorString(he));
    if ((he = staging.init()) != hipSuccess) return fail(CE_E_NOMEM, "pinned staging: %s", hipGetErrorString(he));
    if ((he = hipMalloc((void**)&arena.base, cfg.hbm_budget)) != hipSuccess)
      return fail(CE_E_NOMEM, "HBM budget of %llu bytes: %s", (unsigned long long)cfg.hbm_budget,
                  hipGetErrorString(he));
    arena.size = cfg.hbm_budget;
    arena.reset();
    const size_t cap = cfg.max_jobs;
    if ((he = hipMalloc((void**)&table, cap * sizeof(ServeDesc))) != hipSuccess ||
        (he = hipMalloc((void**)&tiles_done, cap * sizeof(uint32_t))) != hipSuccess ||
        (he = hipMalloc((void**)&pub, cap * sizeof(uint64_t))) != hipSuccess ||
        (he = hipMalloc((void**)&state, sizeof(ServeState))) != hipSuccess)
      return fail(CE_E_NOMEM, "serving tables: %s", hipGetErrorString(he));
    const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
    if ((he = hipHostMalloc((void**)&ring, cap * sizeof(ServeDesc), fl)) != hipSuccess ||
        (he = hipHostMalloc((void**)&ctl, sizeof(ServeCtl), fl)) != hipSuccess ||
        (he = hipHostMalloc((void**)&done_words, cap * sizeof(uint64_t), fl)) != hipSuccess ||
        (he = hipHostMalloc((void**)&first_words, cap * sizeof(uint64_t), fl)) != hipSuccess)
      return fail(CE_E_NOMEM, "host-coherent rings: %s", hipGetErrorString(he));
    memset(ring, 0, cap * sizeof(ServeDesc));
    memset(ctl, 0, sizeof(ServeCtl));
    memset(done_words, 0, cap * sizeof(uint64_t));
    memset(first_words, 0, cap * sizeof(uint64_t));
    if ((he = hipHostGetDevicePointer((void**)&ring_dev, ring, 0)) != hipSuccess ||
        (he = hipHostGetDevicePointer((void**)&ctl_dev, ctl, 0)) != hipSuccess ||
        (he = hipHostGetDevicePointer((void**)&done_dev, done_words, 0)) != hipSuccess ||
        (he = hipHostGetDevicePointer((void**)&first_dev, first_words, 0)) != hipSuccess)
      return fail(CE_E_DEVICE, "device views: %s", hipGetErrorString(he));
    worker = std::thread([this] { loop(); });
    return CE_OK;
  }

  ~ce_server() {
    (void)drain(30.0);
    quit.store(true);
    cv.notify_all();
    if (worker.joinable()) worker.join();
    if (stream) (void)hipStreamSynchronize(stream);
    staging.destroy();
    if (copy_stream) (void)hipStreamDestroy(copy_stream);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    if (arena.base) (void)hipFree(arena.base);
    if (table) (void)hipFree(table);
    if (tiles_done) (void)hipFree(tiles_done);
    if (pub) (void)hipFree(pub);
    if (state) (void)hipFree(state);
    if (ring) (void)hipHostFree(ring);
    if (ctl) (void)hipHostFree(ctl);
    if (done_words) (void)hipHostFree(done_words);
    if (first_words) (void)hipHostFree(first_words);
  }

  // Starts a serving session: clears the kernel's state and launches it.
  // Called with mu held.
  ce_status start_session() {
    hipError_t he;
    ++session;
    head = 0;
    session_tiles = 0;
    seq_ticket.clear();
    const size_t cap = cfg.max_jobs;
    __atomic_store_n(&ctl->head, 0, __ATOMIC_RELEASE);
    __atomic_store_n(&ctl->stop, 0, __ATOMIC_RELEASE);
    __atomic_store_n(&ctl->flags, 0, __ATOMIC_RELEASE);
    __atomic_store_n(&ctl->consumed, 0, __ATOMIC_RELEASE);
    memset(done_words, 0, cap * sizeof(uint64_t));
    memset(first_words, 0, cap * sizeof(uint64_t));
    if ((he = hipMemsetAsync(state, 0, sizeof(ServeState), stream)) != hipSuccess ||
        (he = hipMemsetAsync(pub, 0, cap * sizeof(uint64_t), stream)) != hipSuccess ||
        (he = hipMemsetAsync(tiles_done, 0, cap * sizeof(uint32_t), stream)) != hipSuccess)
      return fail(CE_E_DEVICE, "session reset: %s", hipGetErrorString(he));
    int bpc = 0;
    if ((he = serve_blocks_per_cu(&bpc)) != hipSuccess) return fail(CE_E_DEVICE, "occupancy");
    ServeArgs a{};
    a.ring = ring_dev;
    a.table = table;
    a.tiles_done = tiles_done;
    a.pub = pub;
    a.q = state;
    a.ctl = ctl_dev;
    a.done_words = done_dev;
    a.first_words = first_dev;
    a.cap = (uint32_t)cap;
    a.session = session;
    a.idle_ticks = (uint64_t)(cfg.session_timeout_s * (double)wallclock_hz);
    const uint32_t per_cu = cfg.workgroups_per_cu ? std::min<uint32_t>(cfg.workgroups_per_cu, (uint32_t)std::max(1, bpc))
                                                  : (uint32_t)std::max(1, bpc - 1);
    const uint32_t grid = per_cu * (uint32_t)n_cu;
    grid_ = grid;
    if ((he = launch_serve(a, grid, stream)) != hipSuccess)
      return fail(CE_E_DEVICE, "serving kernel launch: %s", hipGetErrorString(he));
    session_on = true;
    return CE_OK;
  }

  // Admission: the oldest pending job goes in when a slot and memory are free.
  bool admit_one(std::unique_lock<std::mutex>& lk) {
    if (pending.empty() || !session_on) return false;
    if (inflight.size() >= cfg.max_inflight || head >= cfg.max_jobs) return false;
    const uint64_t tk = pending.front();
    JobRec& r = jobs[tk];
    {
      ServeDesc probe{};
      probe.kind = (uint32_t)r.job.kernel_id;
      probe.esc = r.job.esc;
      probe.blur = r.job.blur;
      probe.nb = r.job.nb;
      if (session_tiles + serve_tiles(probe) > kServeTotalMask) return false;  // waits for the next session
    }
    const size_t ob = out_bytes_of(r.job);
    size_t need = (ob + 255) & ~(size_t)255;
    const bool copy0 = !r.job.in0_dev && in_bytes_of(r.job, 0);
    const bool copy1 = !r.job.in1_dev && in_bytes_of(r.job, 1);
    const size_t i0 = copy0 ? ((in_bytes_of(r.job, 0) + 255) & ~(size_t)255) : 0;
    const size_t i1 = copy1 ? ((in_bytes_of(r.job, 1) + 255) & ~(size_t)255) : 0;
    need += i0 + i1;
    uint64_t off = 0;
    if (!arena.alloc(need, &off)) return false;
    pending.pop_front();
    r.mem_off = off;
    r.mem_bytes = need;
    r.has_mem = true;
    r.out_bytes = ob;
    char* mem = arena.base + off;
    ServeDesc d{};
    d.kind = (uint32_t)r.job.kernel_id;
    d.esc = r.job.esc;
    d.blur = r.job.blur;
    d.nb = r.job.nb;
    d.strict = r.job.nb.strict;
    d.out = mem;
    d.in0 = copy0 ? (const void*)(mem + ((ob + 255) & ~(size_t)255)) : r.job.in0_dev;
    d.in1 = copy1 ? (const void*)(mem + ((ob + 255) & ~(size_t)255) + i0) : r.job.in1_dev;
    d.granules = serve_granules(d);
    d.ntiles = serve_tiles(d);
    d.seq = head;
    lk.unlock();
    std::unique_lock<std::mutex> ck(copy_mu);
    hipError_t ce_ = hipSuccess;
    if (copy0) ce_ = staging.to_device((void*)d.in0, r.job.in0_host, in_bytes_of(r.job, 0), copy_stream);
    if (ce_ == hipSuccess && copy1)
      ce_ = staging.to_device((void*)d.in1, r.job.in1_host, in_bytes_of(r.job, 1), copy_stream);
    const bool ok = ce_ == hipSuccess;
    ck.unlock();
    lk.lock();
    if (ok && !session_on) {  // the session ended while the inputs were copied: retry in the next one
      arena.release(r.mem_off, r.mem_bytes);
      r.has_mem = false;
      pending.push_front(tk);
      return false;
    }
    if (!ok) {
      r.state = CE_JOB_FAILED;
      r.why = std::string("copying its inputs into HBM failed: ") + hipGetErrorString(ce_);
      arena.release(r.mem_off, r.mem_bytes);
      r.has_mem = false;
      cv.notify_all();
      return true;
    }
    r.desc = d;
    r.t_admit = now_ns();
    r.state = CE_JOB_ADMITTED;
    publish(tk);
    inflight.push_back(tk);
    max_inflight_seen = std::max<uint64_t>(max_inflight_seen, inflight.size());
    return true;
  }

  bool collect(std::unique_lock<std::mutex>&) {
    bool any = false;
    for (size_t i = 0; i < inflight.size();) {
      const uint64_t tk = inflight[i];
      JobRec& r = jobs[tk];
      const uint64_t dw = __atomic_load_n(&done_words[r.desc.seq], __ATOMIC_ACQUIRE);
      if (dw != 0) {
        r.t_done = now_ns();
        r.tick_done = dw & ~1ull;
        r.tick_first = __atomic_load_n(&first_words[r.desc.seq], __ATOMIC_ACQUIRE);
        t_last_done = r.t_done;
        r.state = CE_JOB_DONE;
        if (!cfg.keep_outputs && r.has_mem) {
          arena.release(r.mem_off, r.mem_bytes);
          r.has_mem = false;
        }
        inflight[i] = inflight.back();
        inflight.pop_back();
        any = true;
      } else {
        ++i;
      }
    }
    if (any) cv.notify_all();
    return any;
  }

  // Publishes an admitted job in the current session (mu held).
  void publish(uint64_t tk) {
    JobRec& r = jobs[tk];
    r.desc.seq = head;
    session_tiles += r.desc.ntiles;
    ring[head] = r.desc;  // the descriptor is complete before head moves
    seq_ticket.push_back(tk);
    ++head;
    __atomic_store_n(&ctl->head, head, __ATOMIC_RELEASE);
  }

  // The session can take no more jobs (its kernel left when idle, or the
  // ring or the tile space is full): end it, and start the next one for the
  // jobs waiting, publishing first any admitted job the kernel never took.
  // Called with mu held, by the server thread only.
  void roll_over(std::unique_lock<std::mutex>& lk, bool ended) {
    if (!ended) __atomic_store_n(&ctl->stop, 1, __ATOMIC_SEQ_CST);
    const uint64_t sess = session;
    lk.unlock();
    const int64_t limit = now_ns() + 10'000'000'000LL;
    while (__atomic_load_n(&ctl->exited, __ATOMIC_ACQUIRE) != sess && now_ns() < limit) _mm_pause();
    const hipError_t he = hipStreamSynchronize(stream);
    lk.lock();
    if (he != hipSuccess || __atomic_load_n(&ctl->exited, __ATOMIC_ACQUIRE) != sess) {
      fail(CE_E_DEVICE, "serving kernel did not end: %s", hipGetErrorString(he));
      return;
    }
    collect(lk);
    const uint64_t consumed = __atomic_load_n(&ctl->consumed, __ATOMIC_ACQUIRE);
    std::vector<uint64_t> again;
    for (size_t i = 0; i < inflight.size();) {
      JobRec& r = jobs[inflight[i]];
      if (r.desc.seq >= consumed) {
        again.push_back(inflight[i]);
      } else {
        // taken by the kernel but never finished (it gave up on an invisible job)
        r.state = CE_JOB_FAILED;
        r.why = "the serving kernel took it but ended before finishing it";
        if (r.has_mem) {
          arena.release(r.mem_off, r.mem_bytes);
          r.has_mem = false;
        }
        fail(CE_E_DEVICE, "serving kernel dropped job %llu", (unsigned long long)inflight[i]);
      }
      inflight[i] = inflight.back();
      inflight.pop_back();
    }
    std::sort(again.begin(), again.end(), [&](uint64_t a, uint64_t b) { return jobs[a].desc.seq < jobs[b].desc.seq; });
    session_on = false;
    if (again.empty() && pending.empty()) return;
    if (start_session() != CE_OK) {
      for (uint64_t tk : again) {
        jobs[tk].state = CE_JOB_FAILED;
        jobs[tk].why = "no new session could be started for it";
        if (jobs[tk].has_mem) {
          arena.release(jobs[tk].mem_off, jobs[tk].mem_bytes);
          jobs[tk].has_mem = false;
        }
      }
      cv.notify_all();
      return;
    }
    for (uint64_t tk : again) {
      publish(tk);
      inflight.push_back(tk);
    }
    cv.notify_all();
  }

  // Whether the oldest pending job would fit this session's tile space.
  bool next_fits_tiles() const {
    if (pending.empty()) return true;
    const JobRec& r = jobs[pending.front()];
    ServeDesc probe{};
    probe.kind = (uint32_t)r.job.kernel_id;
    probe.esc = r.job.esc;
    probe.blur = r.job.blur;
    probe.nb = r.job.nb;
    return session_tiles + serve_tiles(probe) <= kServeTotalMask;
  }

  void loop() {
    std::unique_lock<std::mutex> lk(mu);
    while (!quit.load()) {
      bool progress = collect(lk);
      if (session_on) {
        const bool ended = __atomic_load_n(&ctl->exited, __ATOMIC_ACQUIRE) == session;
        const bool full = !pending.empty() && (head >= cfg.max_jobs || !next_fits_tiles());
        if (ended || (full && inflight.empty())) {
          roll_over(lk, ended);
          progress = true;
        }
      }
      while (admit_one(lk)) progress = true;
      if (!progress) {
        if (inflight.empty() && pending.empty()) {
          cv.wait_for(lk, std::chrono::milliseconds(2));
        } else {
          lk.unlock();
          for (int k = 0; k < 64; ++k) _mm_pause();
          lk.lock();
        }
      }
    }
  }

  ce_status submit(const ce_job* j, uint64_t* ticket) {
    const size_t ob = out_bytes_of(*j);
    if (ob == 0) return fail(CE_E_INVALID, "submit: unknown kernel or empty job");
    if (j->kernel_id == CE_KERNEL_BLUR5 && (!(j->in0_dev || j->in0_host) || !(j->in1_dev || j->in1_host)))
      return fail(CE_E_INVALID, "submit: blur needs an image and weights");
    if (j->kernel_id == CE_KERNEL_NBODY_ACC && !(j->in0_dev || j->in0_host))
      return fail(CE_E_INVALID, "submit: n-body needs bodies");
    if (j->kernel_id == CE_KERNEL_NBODY_ACC && !(j->nb.eps2 >= 1.17549435e-38f))
      return fail(CE_E_INVALID, "submit: eps2 must be a positive normal float");
    size_t need = (ob + 255) & ~(size_t)255;
    for (int s = 0; s < 2; ++s) {
      const void* d = s ? j->in1_dev : j->in0_dev;
      if (!d) need += (in_bytes_of(*j, s) + 255) & ~(size_t)255;
    }
    if (need > cfg.hbm_budget) return fail(CE_E_BUDGET, "submit: job needs %zu bytes, budget %llu", need,
                                          (unsigned long long)cfg.hbm_budget);
    std::lock_guard<std::mutex> lk(mu);
    if (!session_on) {
      ce_status st = start_session();
      if (st != CE_OK) return st;
    }
    JobRec r;
    r.job = *j;
    r.t_submit = now_ns();
    r.items = items_of(*j);
    if (!t_first_submit) t_first_submit = r.t_submit;
    jobs.push_back(r);
    const uint64_t tk = jobs.size() - 1;
    pending.push_back(tk);
    if (ticket) *ticket = tk;
    cv.notify_all();
    return CE_OK;
  }

  ce_status wait(uint64_t tk, double timeout_s) {
    std::unique_lock<std::mutex> lk(mu);
    if (tk >= jobs.size()) return fail(CE_E_INVALID, "wait: unknown ticket");
    const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (jobs[tk].state != CE_JOB_DONE && jobs[tk].state != CE_JOB_FAILED) {
      if (cv.wait_until(lk, until) == std::cv_status::timeout && std::chrono::steady_clock::now() >= until)
        return fail(CE_E_TIMEOUT, "wait: job %llu not done", (unsigned long long)tk);
    }
    return jobs[tk].state == CE_JOB_DONE
               ? CE_OK
               : fail(CE_E_DEVICE, "job %llu failed: %s", (unsigned long long)tk, jobs[tk].why.c_str());
  }

  // Waits for every submitted job, then ends the session (the kernel leaves).
  ce_status drain(double timeout_s) {
    std::unique_lock<std::mutex> lk(mu);
    if (!session_on) return CE_OK;
    const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (!pending.empty() || !inflight.empty()) {
      if (cv.wait_until(lk, until) == std::cv_status::timeout && std::chrono::steady_clock::now() >= until)
        break;
    }
    const bool all_done = pending.empty() && inflight.empty();
    __atomic_store_n(&ctl->stop, 1, __ATOMIC_SEQ_CST);
    session_on = false;
    lk.unlock();
    const int64_t limit = now_ns() + (int64_t)((cfg.session_timeout_s + 5.0) * 1e9);
    while (__atomic_load_n(&ctl->exited, __ATOMIC_ACQUIRE) != session && now_ns() < limit) _mm_pause();
    const hipError_t he = hipStreamSynchronize(stream);
    if (he != hipSuccess) return fail(CE_E_DEVICE, "serving kernel: %s", hipGetErrorString(he));
    if (__atomic_load_n(&ctl->flags, __ATOMIC_ACQUIRE)) return fail(CE_E_TIMEOUT, "serving kernel reached its deadline");
    if (!all_done) return fail(CE_E_TIMEOUT, "drain: jobs still pending after %.1f s", timeout_s);
    return CE_OK;
  }
};

extern "C" {

ce_status ce_server_create(const ce_server_config* cfg, void* hip_stream, ce_server** out) {
  if (!out || !cfg) return CE_E_INVALID;
  *out = nullptr;
  try {
    ce_server* s = new ce_server();
    ce_status st = s->init(cfg, hip_stream);
    if (st != CE_OK) {
      delete s;
      return st;
    }
    *out = s;
    return CE_OK;
  } catch (...) {
    return CE_E_NOMEM;
  }
}

void ce_server_destroy(ce_server* s) { delete s; }

ce_status ce_server_submit(ce_server* s, const ce_job* job, uint64_t* ticket) {
  if (!s || !job) return CE_E_INVALID;
  try {
    return s->submit(job, ticket);
  } catch (...) {
    return CE_E_NOMEM;
  }
}

ce_status ce_server_job_ticks(ce_server* s, uint64_t ticket, uint64_t* first_tile_tick, uint64_t* done_tick) {
  if (!s || !first_tile_tick || !done_tick) return CE_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket >= s->jobs.size()) return s->fail(CE_E_INVALID, "job_ticks: unknown ticket");
  const JobRec& r = s->jobs[ticket];
  if (r.state != CE_JOB_DONE) return s->fail(CE_E_STATE, "job_ticks: job not done");
  *first_tile_tick = r.tick_first;
  *done_tick = r.tick_done;
  return CE_OK;
}

ce_status ce_server_poll(ce_server* s, uint64_t ticket, int32_t* state) {
  if (!s || !state) return CE_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket >= s->jobs.size()) return CE_E_INVALID;
  *state = s->jobs[ticket].state;
  return CE_OK;
}

ce_status ce_server_wait(ce_server* s, uint64_t ticket, double timeout_s) {
  if (!s) return CE_E_INVALID;
  return s->wait(ticket, timeout_s);
}

ce_status ce_server_output(ce_server* s, uint64_t ticket, void** dev_ptr, size_t* bytes) {
  if (!s || !dev_ptr || !bytes) return CE_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket >= s->jobs.size()) return s->fail(CE_E_INVALID, "output: unknown ticket");
  const JobRec& r = s->jobs[ticket];
  if (r.state != CE_JOB_DONE) return s->fail(CE_E_STATE, "output: job not done");
  if (!r.has_mem) return s->fail(CE_E_STATE, "output: released (keep_outputs is off)");
  *dev_ptr = r.desc.out;
  *bytes = r.out_bytes;
  return CE_OK;
}

ce_status ce_server_copy_output(ce_server* s, uint64_t ticket, void* host_dst, size_t bytes) {
  if (!s || !host_dst) return CE_E_INVALID;
  void* src = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticket >= s->jobs.size()) return s->fail(CE_E_INVALID, "copy_output: unknown ticket");
    const JobRec& r = s->jobs[ticket];
    if (r.state != CE_JOB_DONE) return s->fail(CE_E_STATE, "copy_output: job not done");
    if (!r.has_mem) return s->fail(CE_E_STATE, "copy_output: released (keep_outputs is off)");
    if (bytes != r.out_bytes) return s->fail(CE_E_INVALID, "copy_output: %zu bytes, output has %llu", bytes,
                                             (unsigned long long)r.out_bytes);
    src = r.desc.out;
  }
  std::lock_guard<std::mutex> ck(s->copy_mu);
  const hipError_t he = s->staging.to_host(host_dst, src, bytes, s->copy_stream);
  if (he != hipSuccess) return s->fail(CE_E_DEVICE, "copy_output: %s", hipGetErrorString(he));
  return CE_OK;
}

ce_status ce_server_release(ce_server* s, uint64_t ticket) {
  if (!s) return CE_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticket >= s->jobs.size()) return s->fail(CE_E_INVALID, "release: unknown ticket");
  JobRec& r = s->jobs[ticket];
  if (r.state != CE_JOB_DONE && r.state != CE_JOB_FAILED) return s->fail(CE_E_STATE, "release: job not done");
  if (r.has_mem) {
    s->arena.release(r.mem_off, r.mem_bytes);
    r.has_mem = false;
    s->cv.notify_all();
  }
  return CE_OK;
}

ce_status ce_server_drain(ce_server* s, double timeout_s) {
  if (!s) return CE_E_INVALID;
  return s->drain(timeout_s);
}

ce_status ce_server_stats(const ce_server* cs, ce_server_report* r) {
  if (!cs || !r) return CE_E_INVALID;
  ce_server* s = const_cast<ce_server*>(cs);
  std::lock_guard<std::mutex> lk(s->mu);
  memset(r, 0, sizeof *r);
  std::vector<double> lat;
  for (const JobRec& j : s->jobs) {
    ++r->submitted;
    if (j.state == CE_JOB_DONE) {
      ++r->completed;
      r->items += j.items;
      lat.push_back((double)(j.t_done - j.t_submit) * 1e-9);
    }
  }
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
      const double x = p * (double)(lat.size() - 1);
      const size_t i = (size_t)x;
      const double f = x - (double)i;
      return i + 1 < lat.size() ? lat[i] * (1.0 - f) + lat[i + 1] * f : lat[i];
    };
    r->p50_s = pct(0.50);
    r->p99_s = pct(0.99);
    double sum = 0.0;
    for (double v : lat) sum += v;
    r->mean_s = sum / (double)lat.size();
    r->max_s = lat.back();
  }
  if (s->t_first_submit && s->t_last_done > s->t_first_submit) {
    r->wall_s = (double)(s->t_last_done - s->t_first_submit) * 1e-9;
    r->items_per_s = (double)r->items / r->wall_s;
    r->jobs_per_s = (double)r->completed / r->wall_s;
  }
  r->peak_hbm = s->arena.peak;
  r->max_inflight_seen = s->max_inflight_seen;
  return CE_OK;
}

const char* ce_server_error(const ce_server* s) {
  if (!s) return nullptr;
  static thread_local std::string copy;  // stable for the calling thread until its next call
  std::lock_guard<std::mutex> lk(s->err_mu);
  copy = s->error;
  return copy.c_str();
}

}  // extern "C"
