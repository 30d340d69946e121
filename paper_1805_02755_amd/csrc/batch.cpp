// Batched form of the engine: a batch of escape-time jobs of uneven sizes
// runs as ONE persistent kernel launch, captured once in a hipGraph and
// replayed, instead of one launch per job (or per package). The tile shape
// and the number of tiles per workgroup request are chosen by an autotuner
// that times every candidate on the batch itself.
#include <hip/hip_runtime_api.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "../../include/coexec.h"
#include "batch.hpp"
#include "common.hpp"
#include "kernels.hpp"

using namespace ce;

namespace {
constexpr uint32_t kTunePackages[] = {1, 2, 4, 8, 16, 32};
}

struct ce_batch {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<ce_escape_params> params;
  std::vector<uint32_t*> outs;
  int shape = 4;           // 16 x 16 tiles
  uint32_t pkg_tiles = 4;
  bool dirty = true;       // job table or configuration changed since the graph was built
  BatchJob* jobs_dev = nullptr;
  size_t jobs_cap = 0;
  uint64_t* counter = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  uint32_t grid = 0;
  uint64_t total_tiles = 0;
  uint64_t items = 0;
  double last_run_s = 0.0, last_kernel_ms = 0.0;
  uint64_t launches = 0;
  std::string error;

  ce_status fail(ce_status code, const char* fmt, ...) __attribute__((format(printf, 3, 4))) {
    char buf[400];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    error = buf;
    return code;
  }

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }

  ce_status init(void* s) {
    hipError_t he;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(CE_E_DEVICE, "no HIP device");
    if (s) {
      stream = (hipStream_t)s;
    } else {
      if ((he = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking)) != hipSuccess)
        return fail(CE_E_DEVICE, "stream: %s", hipGetErrorString(he));
      own_stream = true;
    }
    // cleared before anything runs on the (non-blocking) stream, which does
    // not wait for the null stream's memset
    if ((he = hipMalloc((void**)&counter, 2 * sizeof(uint64_t))) != hipSuccess ||
        (he = hipMemset(counter, 0, 2 * sizeof(uint64_t))) != hipSuccess || (he = hipDeviceSynchronize()) != hipSuccess)
      return fail(CE_E_DEVICE, "counter: %s", hipGetErrorString(he));
    if ((he = hipEventCreate(&ev0)) != hipSuccess || (he = hipEventCreate(&ev1)) != hipSuccess)
      return fail(CE_E_DEVICE, "events: %s", hipGetErrorString(he));
    return CE_OK;
  }

  ~ce_batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    drop_graph();
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (jobs_dev) (void)hipFree(jobs_dev);
    if (counter) (void)hipFree(counter);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  // Builds the job table for the current tile shape, uploads it and captures
  // the launch in a graph.
  ce_status build() {
    hipError_t he;
    if (params.empty()) return fail(CE_E_STATE, "batch has no jobs");
    const uint32_t TR = kBatchShapeRows[shape], TC = batch_shape_cols(shape);
    std::vector<BatchJob> table(params.size());
    uint64_t base = 0;
    items = 0;
    for (size_t j = 0; j < params.size(); ++j) {
      BatchJob& J = table[j];
      memset(&J, 0, sizeof J);
      J.p = params[j];
      J.tiles_x = (uint32_t)ceil_div(J.p.w, TC);
      J.tile_base = base;
      J.out = outs[j];
      base += ceil_div(J.p.h, TR) * J.tiles_x;
      items += (uint64_t)J.p.w * J.p.h;
    }
    total_tiles = base;
    if (table.size() > jobs_cap) {
      if (jobs_dev) (void)hipFree(jobs_dev);
      jobs_dev = nullptr;
      jobs_cap = 0;
      if ((he = hipMalloc((void**)&jobs_dev, table.size() * sizeof(BatchJob))) != hipSuccess)
        return fail(CE_E_NOMEM, "job table: %s", hipGetErrorString(he));
      jobs_cap = table.size();
    }
    if ((he = hipStreamSynchronize(stream)) != hipSuccess ||
        (he = hipMemcpy(jobs_dev, table.data(), table.size() * sizeof(BatchJob), hipMemcpyHostToDevice)) !=
            hipSuccess)
      return fail(CE_E_DEVICE, "job table upload: %s", hipGetErrorString(he));
    const size_t lds = table.size() * sizeof(uint64_t);
    int bpc = 0, dev = 0, cus = 0;
    if ((he = batch_blocks_per_cu(shape, lds, &bpc)) != hipSuccess || (he = hipGetDevice(&dev)) != hipSuccess ||
        (he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
      return fail(CE_E_DEVICE, "occupancy: %s", hipGetErrorString(he));
    const uint64_t packages = ceil_div(total_tiles, pkg_tiles);
    grid = (uint32_t)std::min<uint64_t>((uint64_t)std::max(1, bpc) * (uint64_t)cus, packages);
    BatchArgs a{jobs_dev, (uint32_t)table.size(), pkg_tiles, total_tiles, counter};
    drop_graph();
    if ((he = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return fail(CE_E_DEVICE, "capture: %s", hipGetErrorString(he));
    const hipError_t le = launch_batch(shape, a, grid, stream);
    he = hipStreamEndCapture(stream, &graph);
    if (le != hipSuccess || he != hipSuccess)
      return fail(CE_E_DEVICE, "capture: %s", hipGetErrorString(le != hipSuccess ? le : he));
    if ((he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess)
      return fail(CE_E_DEVICE, "instantiate: %s", hipGetErrorString(he));
    dirty = false;
    return CE_OK;
  }

  ce_status run(bool timed) {
    if (dirty) {
      ce_status st = build();
      if (st != CE_OK) return st;
    }
    hipError_t he;
    const auto t0 = std::chrono::steady_clock::now();
    if (timed && (he = hipEventRecord(ev0, stream)) != hipSuccess) return fail(CE_E_DEVICE, "event");
    if ((he = hipGraphLaunch(exec, stream)) != hipSuccess)
      return fail(CE_E_DEVICE, "graph launch: %s", hipGetErrorString(he));
    if (timed && (he = hipEventRecord(ev1, stream)) != hipSuccess) return fail(CE_E_DEVICE, "event");
    if ((he = hipStreamSynchronize(stream)) != hipSuccess) return fail(CE_E_DEVICE, "run: %s", hipGetErrorString(he));
    last_run_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (timed) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) last_kernel_ms = ms;
    }
    ++launches;
    return CE_OK;
  }
};

extern "C" {

ce_status ce_batch_create(ce_batch** out, void* hip_stream) {
  if (!out) return CE_E_INVALID;
  *out = nullptr;
  try {
    ce_batch* b = new ce_batch();
    ce_status st = b->init(hip_stream);
    if (st != CE_OK) {
      delete b;
      return st;
    }
    *out = b;
    return CE_OK;
  } catch (...) {
    return CE_E_NOMEM;
  }
}

void ce_batch_destroy(ce_batch* b) { delete b; }

ce_status ce_batch_add_escape(ce_batch* b, const ce_escape_params* p, void* dev_out, uint32_t* index) {
  if (!b) return CE_E_INVALID;
  if (!p || !dev_out) return b->fail(CE_E_INVALID, "add: NULL params or output");
  if (p->w == 0 || p->h == 0) return b->fail(CE_E_INVALID, "add: empty job");
  if (b->params.size() >= kBatchMaxJobs) return b->fail(CE_E_INVALID, "add: more than %u jobs", kBatchMaxJobs);
  try {
    b->params.push_back(*p);
    b->outs.push_back((uint32_t*)dev_out);
  } catch (...) {
    return CE_E_NOMEM;
  }
  if (index) *index = (uint32_t)(b->params.size() - 1);
  b->dirty = true;
  return CE_OK;
}

ce_status ce_batch_clear(ce_batch* b) {
  if (!b) return CE_E_INVALID;
  b->params.clear();
  b->outs.clear();
  b->dirty = true;
  return CE_OK;
}

ce_status ce_batch_set_config(ce_batch* b, const ce_batch_config* c) {
  if (!b || !c) return CE_E_INVALID;
  int shape = -1;
  for (int i = 0; i < kBatchShapes; ++i)
    if (kBatchShapeRows[i] == c->tile_rows) shape = i;
  if (shape < 0) return b->fail(CE_E_INVALID, "config: tile_rows must be 1, 2, 4, 8 or 16");
  if (c->package_tiles == 0 || c->package_tiles > (1u << 20))
    return b->fail(CE_E_INVALID, "config: package_tiles out of range");
  b->shape = shape;
  b->pkg_tiles = c->package_tiles;
  b->dirty = true;
  return CE_OK;
}

ce_status ce_batch_get_config(const ce_batch* b, ce_batch_config* c) {
  if (!b || !c) return CE_E_INVALID;
  c->tile_rows = kBatchShapeRows[b->shape];
  c->tile_cols = batch_shape_cols(b->shape);
  c->package_tiles = b->pkg_tiles;
  return CE_OK;
}

ce_status ce_batch_tune(ce_batch* b, uint32_t reps, ce_batch_config* chosen) {
  if (!b) return CE_E_INVALID;
  if (reps == 0) reps = 3;
  try {
    double best = 1e300;
    int best_shape = b->shape;
    uint32_t best_pkg = b->pkg_tiles;
    for (int sh = 0; sh < kBatchShapes; ++sh) {
      for (uint32_t pk : kTunePackages) {
        b->shape = sh;
        b->pkg_tiles = pk;
        b->dirty = true;
        ce_status st = b->run(true);  // build + warm-up
        if (st != CE_OK) return st;
        double tot = 0.0;
        for (uint32_t r = 0; r < reps; ++r) {
          st = b->run(true);
          if (st != CE_OK) return st;
          tot += b->last_kernel_ms;
        }
        if (tot < best) {
          best = tot;
          best_shape = sh;
          best_pkg = pk;
        }
      }
    }
    b->shape = best_shape;
    b->pkg_tiles = best_pkg;
    b->dirty = true;
    if (chosen) ce_batch_get_config(b, chosen);
    return CE_OK;
  } catch (...) {
    return CE_E_NOMEM;
  }
}

ce_status ce_batch_run(ce_batch* b) {
  if (!b) return CE_E_INVALID;
  try {
    return b->run(true);
  } catch (...) {
    return CE_E_NOMEM;
  }
}

ce_status ce_batch_run_separate(ce_batch* b) {
  if (!b) return CE_E_INVALID;
  if (b->params.empty()) return b->fail(CE_E_STATE, "batch has no jobs");
  const auto t0 = std::chrono::steady_clock::now();
  hipError_t he;
  if ((he = hipEventRecord(b->ev0, b->stream)) != hipSuccess) return b->fail(CE_E_DEVICE, "event");
  for (size_t j = 0; j < b->params.size(); ++j) {
    KernelArgs a{};
    a.kernel_id = CE_KERNEL_ESCAPE;
    a.esc = b->params[j];
    a.out = b->outs[j];
    if ((he = launch_bare(a, b->stream)) != hipSuccess)
      return b->fail(CE_E_DEVICE, "launch: %s", hipGetErrorString(he));
  }
  if ((he = hipEventRecord(b->ev1, b->stream)) != hipSuccess) return b->fail(CE_E_DEVICE, "event");
  if ((he = hipStreamSynchronize(b->stream)) != hipSuccess)
    return b->fail(CE_E_DEVICE, "run: %s", hipGetErrorString(he));
  b->last_run_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, b->ev0, b->ev1) == hipSuccess) b->last_kernel_ms = ms;
  return CE_OK;
}

ce_status ce_batch_stats(const ce_batch* b, ce_batch_report* s) {
  if (!b || !s) return CE_E_INVALID;
  memset(s, 0, sizeof *s);
  s->jobs = (uint32_t)b->params.size();
  s->items = b->items;
  s->total_tiles = b->total_tiles;
  s->workgroups = b->grid;
  s->tile_rows = kBatchShapeRows[b->shape];
  s->tile_cols = batch_shape_cols(b->shape);
  s->package_tiles = b->pkg_tiles;
  s->t_run = b->last_run_s;
  s->t_gpu_ms = b->last_kernel_ms;
  s->launches = b->launches;
  return CE_OK;
}

const char* ce_batch_error(const ce_batch* b) { return b ? b->error.c_str() : nullptr; }

}  // extern "C"
