// Layouts and integer helpers shared by the host engine (g++) and the GPU
// kernels (hipcc). Nothing here does payload arithmetic.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIPCC_RTC__)
#define CE_HD __host__ __device__ inline
#else
#define CE_HD inline
#endif

namespace ce {

enum SchedKind : uint32_t { kStatic = 0, kDynamic = 1, kHGuided = 2 };

// Tiles: how a package of granules is cut for the GPU's workgroups.
// 2-D payloads: a tile is kTileRows rows by one column block.
constexpr uint32_t kEscapeTileRows = 1;
constexpr uint32_t kEscapeTileCols = 512;
constexpr uint32_t kBlurTileRows = 32;
constexpr uint32_t kBlurTileCols = 1024;  // 256 threads x 4 columns
constexpr uint32_t kNbodyGranule = 256;   // bodies per granule (1-D lws)
constexpr uint32_t kBlockThreads = 256;

// Dispenser state shared by the GPU and the host, in host-coherent pinned
// memory. The GPU uses system-scope atomics on it.
struct alignas(64) L1State {
  uint64_t next;        // next granule not yet handed to any device
  uint64_t pad0[7];
  // written with system-scope stores and read by the host once the kernel
  // has ended: the start tick by the first workgroup (the host also watches
  // it as it changes, to re-anchor its clock mapping), the flags by any
  // workgroup, the rest by the last workgroup of a run with the counted exit
  uint64_t gpu_done;    // done_word(run id, tick at which the last workgroup left)
  uint64_t gpu_t_first; // s_memrealtime of the first package claim
  uint64_t gpu_t_last;  // s_memrealtime of the last package end
  uint64_t gpu_granules;
  uint64_t gpu_packages;
  uint64_t gpu_flags;   // bit 0: a wait on the dispenser timed out
  uint64_t pad1[2];
  // clock calibration mailbox
  uint64_t ping;
  uint64_t pong;
  uint64_t tick;
  uint64_t pad2[5];
  // host completion ring (device-resident output): once the host device has
  // finished it publishes the number of ring entries of the run
  uint64_t host_final;  // host_final_word(run id, entries), written once per run
  uint64_t pad3[7];
  uint64_t gathered;    // bytes of host output the GPU's gatherers have copied this run
  uint64_t gpu_t_gather;// s_memrealtime at the end of the last gather copy (0: none)
  uint64_t pad4[6];
};

// The GPU's completion as one word, so the host sees the run id and the
// moment it was written together: run id low 24 bits over the low 40 bits
// of the s_memrealtime tick (at 100 MHz they wrap every three hours; the
// host restores the high bits from its own estimate of the tick).
constexpr uint64_t kTick40 = (1ull << 40) - 1;
CE_HD uint64_t done_word(uint64_t run_id, uint64_t tick) { return ((run_id & 0xFFFFFFull) << 40) | (tick & kTick40); }
CE_HD bool done_is(uint64_t w, uint64_t run_id) { return (w >> 40) == (run_id & 0xFFFFFFull); }

// The host's final ring size and the run it belongs to, in one word so the
// GPU reads both with one atomic load: run id low 24 bits over a 40-bit count.
CE_HD uint64_t host_final_word(uint64_t run_id, uint64_t count) { return ((run_id & 0xFFFFFFull) << 40) | count; }

// A host tile whose output the GPU must copy into HBM: byte length in the top
// 24 bits, byte offset in the low 40 bits; 0 means "not published yet".
CE_HD uint64_t ring_word(uint64_t off, uint64_t len) { return (len << 40) | off; }
CE_HD uint64_t ring_off(uint64_t w) { return w & ((1ull << 40) - 1); }
CE_HD uint64_t ring_len(uint64_t w) { return w >> 40; }

constexpr uint32_t kExitLines = 8;

// Size of the static device scratch of the allocation-free run: queue state,
// publication words and package table (72 bytes per package, so about
// 14,000 packages).
constexpr uint64_t kNoallocScratchBytes = 1ull << 20;

// Per-run GPU queue state in HBM (device-scope atomics only), two of them
// taken in turn: each run's kernel clears the other one for the next run
// (with the counted exit the last workgroup also resets its own). Contended
// atomics on one cache line serialise at the memory side, so the ticket
// counter, the read-mostly publication state, the claim lock and the
// bookkeeping each get a line of their own.
struct alignas(128) L2State {
  uint64_t ticket;      // next tile ticket
  uint64_t pad_ticket[15];
  uint64_t total;       // tiles of all published packages | kTotalDone once no more will come
  uint64_t pad_total[15];
  uint32_t lock;        // held by the workgroup claiming the next package
  uint32_t pad_lock[31];
  uint32_t n_pkgs;      // packages published
  uint32_t exit_count;  // exit lines whose workgroups have all left
  uint32_t st_next;     // static: next band of this device
  uint32_t exit_compute;// computing (non-gather) workgroups that left
  uint64_t granules;    // granules published
  uint64_t t_first;     // first claim tick
  uint64_t t_last;      // tick at which the last computing workgroup left
  uint64_t gather_next; // next host completion-ring entry to copy
  uint64_t pad_pre[2];
  uint64_t t_gather;    // latest end tick of a gather copy
  uint64_t pad_misc[7];
  // Workgroups that left, counted on kExitLines lines of their own by
  // blockIdx mod kExitLines (the XCD a workgroup is dealt to): a thousand
  // workgroups leaving together would otherwise queue on one line.
  uint32_t exit_x[kExitLines][32];
};

constexpr uint64_t kTotalDone = 1ull << 63;
constexpr uint64_t kTotalMask = kTotalDone - 1;

// A published GPU package as one 64-bit word: granule count in the top 24
// bits, first granule in the low 40 bits; 0 means "not published yet".
constexpr uint64_t kPubG0Bits = 40;
constexpr uint64_t kPubMaxSize = (1ull << 24) - 1;
CE_HD uint64_t pub_word(uint64_t g0, uint64_t size) { return (size << kPubG0Bits) | g0; }
CE_HD uint64_t pub_g0(uint64_t w) { return w & ((1ull << kPubG0Bits) - 1); }
CE_HD uint64_t pub_size(uint64_t w) { return w >> kPubG0Bits; }

// One GPU package as published to the workgroups; also its trace record.
struct alignas(64) PkgSlot {
  uint64_t g0, g1;      // granules [g0, g1)
  uint64_t base;        // first tile ticket of the package
  uint32_t ntiles;
  uint32_t tiles_done;
  uint64_t t_claim;     // s_memrealtime at claim
  uint64_t t_end;       // s_memrealtime when its last tile finished
  uint64_t pad[2];
};

// Scheduler arguments of one device for one run (kernel argument by value).
struct SchedArgs {
  uint32_t kind;
  uint32_t n_dev;       // devices in the set (HGuided n)
  uint32_t k;           // HGuided k
  uint32_t batch;       // Dynamic: packages taken by one claim (>= 1)
  uint64_t G;           // granules in the index space
  uint64_t pkg;         // Dynamic package size (granules)
  uint64_t P_self;      // HGuided power of this device
  uint64_t sumP;        // HGuided sum of powers
  uint64_t min_self;    // HGuided minimum package of this device
  uint64_t st_begin, st_end;  // Static: this device's granule range
  uint64_t st_nbands;   // Static: band grid (0 = one package)
  uint64_t run_id;
  uint64_t wait_ticks;  // longest wait on the dispenser, in s_memrealtime ticks
  L1State* l1;          // device address of the host-coherent dispenser
  L2State* l2;          // HBM
  PkgSlot* pkgs;        // trace records of the GPU's packages
  uint64_t* pub;        // publication words, zero between runs
  uint32_t max_pkgs;
  uint32_t lookahead;   // claim the next package this many tiles early
  uint32_t chunk;       // tile tickets taken per atomic
  uint32_t stride;      // 1: workgroup w runs tickets w, w + n, w + 2n ... (uniform-cost tiles)
  // The GPU's first package, claimed by the host just before the launch
  // (pre_nt == 0: none), so the workgroups start without a claim race.
  uint64_t pre_g0, pre_g1;
  uint32_t pre_nt;      // its tiles
  uint32_t st_first;    // static: bands taken by that claim
  // Dynamic: tiles of every GPU package but the one that ends the index
  // space, so ticket t lies in package t / dyn_tiles (0: walk the packages)
  uint32_t dyn_tiles;
  // 1: the pre-claimed package is all this device will run (a static plan
  // with one package for it), so no workgroup needs to look for another
  uint32_t pre_only;
  // gather of host-computed output into HBM (gather_wgs == 0: off)
  const uint64_t* ring; // device view of the host completion ring
  const char* gsrc;     // device view of the host output buffer
  char* gdst;           // device output buffer
  uint32_t gather_wgs;  // workgroups 0 .. gather_wgs-1 only gather
  uint32_t ring_cap;    // entries in the ring
  uint64_t gather_wait_ticks;  // longest wait for the host's next finished tile
  // Light exit (no gather workgroups): no workgroup counts itself out or
  // resets anything; each stores the tick at which it left into
  // wg_end[blockIdx.x] (host-coherent) and the host takes the GPU's end from
  // them after the kernel. This run's queue state is left as it is: the next
  // run uses the other buffer. Null: the regular exit (count out; the last
  // workgroup publishes the summary and resets the state).
  uint64_t* wg_end;
  // The other of the two queue-state buffers and its publication words, the
  // next run's: cleared by this run's workgroups as they start, while
  // nothing uses them (null: single-buffered, as in the allocation-free run,
  // which clears its state before each run).
  L2State* l2_next;
  uint64_t* pub_next;
  uint32_t pub_next_words;
  uint32_t pad_next;
};

constexpr uint32_t kFastExitMaxWgs = 65536;  // entries of the host's wg_end array

// Arguments of the direct kernel, for a run whose whole GPU share is the
// package the host claimed before the launch, dealt round-robin: no
// dispenser at all, so nothing of it is passed.
struct DirectArgs {
  uint64_t g0, g1;      // the package
  uint32_t ntiles;      // its tiles
  uint32_t swizzle;     // 1: one workgroup per tile, dealt over the XCDs in turn (see k_direct)
  L1State* l1;          // device address of the dispenser: the first workgroup stamps the GPU's start
  PkgSlot* pkgs;        // ... and the package's claim time into its trace record
  uint64_t* wg_end;     // each workgroup's end tick (host-coherent)
};

// HGuided package size (section 5.3 equation), integer only. Callers keep
// G_r < 2^40 and P <= 2^20 so the products fit in 64 bits.
CE_HD uint64_t hguided_size(uint64_t G_r, uint64_t P_i, uint64_t sumP, uint32_t n, uint32_t k,
                            uint64_t min_i) {
  const uint64_t den = (uint64_t)k * (uint64_t)n * sumP;
  uint64_t s = den ? (G_r * P_i) / den : G_r;
  if (s < min_i) s = min_i;
  if (s > G_r) s = G_r;
  return s;
}

// Static: the b-th band of a grid of nb bands over G granules.
CE_HD uint64_t band_edge(uint64_t b, uint64_t G, uint64_t nb) { return nb ? (b * G) / nb : 0; }

CE_HD uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

}  // namespace ce
