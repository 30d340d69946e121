// Serving form: a persistent GPU kernel runs jobs that the host admits while
// earlier jobs are still running (continuous batching). Layouts shared by the
// host server (serve.cpp) and the serving kernel (serve_kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "../../include/coexec.h"

namespace ce {

// One admitted job, as written by the host into the job ring (host-coherent
// memory) and copied by the kernel into its table in HBM. 128 bytes.
struct alignas(128) ServeDesc {
  uint32_t kind;       // CE_KERNEL_*
  uint32_t strict;     // n-body rsqrt mode
  uint32_t ntiles;     // tiles of the job (GPU tiling of the payload)
  uint32_t pad0;
  uint64_t granules;   // granules of the job's index space
  uint64_t seq;        // admission sequence number
  ce_escape_params esc;  // 28 B
  ce_blur5_params blur;  // 8 B
  ce_nbody_params nb;    // 12 B
  uint32_t pad1;
  const void* in0;
  const void* in1;
  void* out;
  uint64_t pad2;
};

// Serving kernel state in HBM (zero at the start of a session).
struct alignas(64) ServeState {
  uint64_t ticket;      // next tile ticket
  uint64_t ct;          // done << 63 | jobs copied from the host ring << 40 | tiles of those jobs
  uint32_t pad_done;
  uint32_t exit_count;
  uint32_t flags;       // bit 0: a published job stayed invisible past the idle bound
  uint32_t pad0;
  uint64_t t_active;    // s_memrealtime when the last job was appended (0: none yet)
  uint64_t pad[3];
};
constexpr uint32_t kServeTotalBits = 40;  // tiles per session < 2^40
constexpr uint64_t kServeTotalMask = (1ull << kServeTotalBits) - 1;
constexpr uint64_t kServeDone = 1ull << 63;  // no more jobs: workgroups leave
constexpr uint32_t kServeMaxJobs = (1u << 23) - 1;  // jobs per session (the count's field)

// Host control block (host-coherent memory), read and written by both sides.
struct alignas(64) ServeCtl {
  uint64_t head;        // jobs published in the ring (host writes)
  uint64_t stop;        // 1: no more jobs will be published (host writes)
  uint64_t exited;      // session id, written by the last workgroup out
  uint64_t flags;       // error bits from the kernel
  uint64_t consumed;    // jobs the kernel took from the ring (written before exited)
  uint64_t pad[3];
};

struct ServeArgs {
  const ServeDesc* ring;  // device view of the host ring
  ServeDesc* table;       // HBM copy of admitted jobs
  uint32_t* tiles_done;   // HBM, one counter per job
  uint64_t* pub;          // HBM, tiles of job k (0 = not published yet)
  ServeState* q;          // HBM
  ServeCtl* ctl;          // device view of the host control block
  uint64_t* done_words;   // device view of host completion words, one per job
  uint64_t* first_words;  // device view of host words: tick of each job's first tile
  uint32_t cap;           // jobs per session
  uint32_t pad;
  uint64_t session;
  uint64_t idle_ticks;    // the kernel leaves after this many ticks with no new job
};

uint32_t serve_tiles(const ServeDesc& d);  // GPU tiles of a job
uint64_t serve_granules(const ServeDesc& d);
hipError_t serve_blocks_per_cu(int* blocks);
hipError_t launch_serve(const ServeArgs& a, uint32_t grid, hipStream_t st);

}  // namespace ce
