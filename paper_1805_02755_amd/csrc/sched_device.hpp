// Device side of the dispenser: the level-2 ticket chain, package claims
// and publication, the persistent kernel template that runs any payload
// tile type through them, and the plain one-launch form of a payload. The
// fixed payloads instantiate these templates in kernels.hip; a payload
// supplied as source at run time is compiled together with this header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "device_atomics.hpp"

namespace ce {

__device__ __forceinline__ uint64_t max_u64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// ---------------------------------------------------------------- dispenser
// Bounded waits: true once more than `limit` ticks have passed since the
// first call with *t0 == 0 (which starts the clock). Every wait in the
// dispenser ends this way, well before the host gives up on the kernel.
__device__ __forceinline__ bool waited_out(uint64_t* t0, uint64_t limit) {
  const uint64_t now = now_tick();
  if (*t0 == 0) {
    *t0 = now;
    return false;
  }
  return now - *t0 > limit;
}

// Claims the next level-1 package for the GPU. Only the holder of the claim
// lock runs this.
__device__ bool claim_package(const SchedArgs& s, uint64_t* g0, uint64_t* g1, bool* timed_out) {
  L2State* q = s.l2;
  if (s.kind == kStatic) {
    const uint32_t bk = dev_load(&q->st_next);
    const uint32_t b = bk + s.st_first;
    if (s.st_nbands == 0) {
      // one package per device, cut only if it exceeds the descriptor's size field
      const uint64_t a = s.st_begin + (uint64_t)b * kPubMaxSize;
      if (a >= s.st_end) return false;
      *g0 = a;
      *g1 = (s.st_end - a > kPubMaxSize) ? a + kPubMaxSize : s.st_end;
    } else {
      const uint64_t b0 = s.st_begin + b;  // st_begin/st_end hold band indices here
      if (b0 >= s.st_end) return false;
      *g0 = band_edge(b0, s.G, s.st_nbands);
      *g1 = band_edge(b0 + 1, s.G, s.st_nbands);
    }
    dev_store(&q->st_next, bk + 1);
    return true;
  }
  if (s.kind == kDynamic) {
    // `batch` consecutive packages with one atomic (split up by the caller)
    const uint64_t span = s.pkg * s.batch;
    const uint64_t a = sys_fetch_add(&s.l1->next, span);
    if (a >= s.G) return false;
    *g0 = a;
    *g1 = (a + span < s.G) ? a + span : s.G;
    return true;
  }
  // HGuided: the size follows the pending granules at the moment of the claim.
  uint64_t cur = sys_load(&s.l1->next);
  for (uint64_t t0 = 0;;) {
    if (cur >= s.G) return false;
    uint64_t sz = hguided_size(s.G - cur, s.P_self, s.sumP, s.n_dev, s.k, s.min_self);
    if (sz > kPubMaxSize) sz = kPubMaxSize;
    if (sys_cas(&s.l1->next, &cur, cur + sz)) {
      *g0 = cur;
      *g1 = cur + sz;
      return true;
    }
    if (waited_out(&t0, s.wait_ticks)) {
      *timed_out = true;
      return false;
    }
  }
}

// Publishes one package at the end of the GPU's tile sequence (lock held).
template <class T>
__device__ void publish(const T& pay, const SchedArgs& s, uint64_t tot, uint64_t g0, uint64_t g1, uint64_t tc) {
  L2State* q = s.l2;
  const uint32_t nk = dev_load(&q->n_pkgs);   // packages published by the kernel
  const uint32_t n = nk + (s.pre_nt ? 1u : 0u);  // slot 0 holds the pre-claimed one
  const uint32_t nt = pay.ntiles(g0, g1);
  PkgSlot* ps = &s.pkgs[n];  // trace record, read by the host after the run;
  ps->g0 = g0;               // its tile counter was cleared at the end of the last run
  ps->g1 = g1;
  ps->base = tot;
  ps->ntiles = nt;
  ps->t_claim = tc;
  // t_end is written by the workgroup that runs the package's last ticket.
  if (n == 0) dev_store(&q->t_first, tc);
  dev_store(&q->n_pkgs, nk + 1);
  dev_store(&q->granules, dev_load(&q->granules) + (g1 - g0));
  dev_store(&s.pub[n], pub_word(g0, g1 - g0));  // readers spin until it is visible
  dev_store(&q->total, tot + nt);
}

// Publishes the packages of one Dynamic claim ([g0, g1) holds `batch`
// packages of `pkg` granules, the last one possibly short). The publication
// words and the published count go out first, so workgroups start on the
// packages at once; the trace records, which only the host reads after the
// run, follow.
template <class T>
__device__ void publish_dynamic(const T& pay, const SchedArgs& s, uint64_t tot, uint64_t g0, uint64_t g1,
                                uint64_t tc) {
  // The arguments live in LDS and the stores below are flat ones, which may
  // alias LDS and count against its counter: with the fields re-read from
  // LDS after every store, each package would wait for all stores before it.
  L2State* const q = s.l2;
  PkgSlot* const pkgs = s.pkgs;
  uint64_t* const pub = s.pub;
  const uint64_t pkg = s.pkg;
  const uint32_t max_pkgs = s.max_pkgs;
  const uint32_t pre = s.pre_nt ? 1u : 0u;
  const uint32_t nk0 = dev_load(&q->n_pkgs);
  // packages that fit the table (the host sizes it so that all do)
  uint64_t end = g1;
  const uint64_t room = max_pkgs > nk0 + pre ? (uint64_t)(max_pkgs - nk0 - pre) : 0;
  if (ceil_div(g1 - g0, pkg) > room) end = g0 + room * pkg;
  const uint64_t tot0 = tot;  // first ticket of the claim
  uint32_t nk = nk0;
  for (uint64_t x = g0; x < end; x += pkg) {
    const uint64_t y = (x + pkg < end) ? x + pkg : end;
    dev_store(&pub[nk + pre], pub_word(x, y - x));
    tot += pay.ntiles(x, y);
    ++nk;
    // the published count is the line every waiting workgroup polls: move
    // it in steps of 32 packages rather than once per package
    if (((nk - nk0) & 31u) == 0) dev_store(&q->total, tot);
  }
  dev_store(&q->total, tot);
  uint64_t base = tot0;
  if (nk0 + pre == 0) dev_store(&q->t_first, tc);
  nk = nk0;
  for (uint64_t x = g0; x < end; x += pkg) {
    const uint64_t y = (x + pkg < end) ? x + pkg : end;
    const uint32_t nt = pay.ntiles(x, y);
    PkgSlot* ps = &pkgs[nk + pre];
    ps->g0 = x;
    ps->g1 = y;
    ps->base = base;
    ps->ntiles = nt;
    ps->t_claim = tc;
    base += nt;
    ++nk;
  }
  dev_store(&q->n_pkgs, nk);
  dev_store(&q->granules, dev_load(&q->granules) + (end - g0));
  if (end < g1) sys_store(&s.l1->gpu_flags, 1);
}

// What one workgroup knows of the ticket chain, held by the lane that talks
// to the dispenser: tickets taken but not yet run, the published total it
// last read (it only grows, so it is a safe lower bound), the package of its
// current ticket and that ticket. Completion needs no per-tile atomics: the
// workgroup that runs a package's last ticket stamps the package's end, and
// the GPU's end is the moment the last workgroup leaves (a report from every
// workgroup at the end of a run would queue ~1000 atomics on one line).
struct Cursor {  // zero-initialised at the start of a run
  uint64_t t_next, t_end;
  uint64_t tot_seen;
  uint64_t base, g0, g1;
  uint64_t cur_t;  // ticket of the tile being run
  uint32_t p, nt;  // nt == 0: no package yet
};

// After a tile: if it held its package's last ticket, stamp the package end.
__device__ __forceinline__ void tile_finished(const SchedArgs& s, const Cursor& c) {
  if (c.nt == 0 || c.cur_t + 1 != c.base + c.nt) return;
  dev_store(&s.pkgs[c.p].t_end, now_tick());
}

// Ticket chain with lookahead. Every workgroup's first ticket is its own
// index among the n computing workgroups. After that, with uniform-cost
// tiles (s.stride) workgroup w simply runs tickets w + n, w + 2n, ... with no
// atomic at all; otherwise it takes s.chunk tickets per atomic from a
// counter that starts past the first round. When a ticket is within `lookahead` tiles of the end of the
// published tiles it tries to take the claim lock and append the next
// level-1 package, so the PCIe round trip of the claim overlaps the last
// round of tiles. The GPU thus acts as one device towards the scheduler while
// its workgroups share each package. Returns false when this workgroup
// should leave.
template <class T>
__device__ bool next_tile(const T& pay, const SchedArgs& s, Cursor& c, uint32_t* ti_out) {
  L2State* q = s.l2;
  if (c.t_next == c.t_end) {
    const uint64_t n = gridDim.x - s.gather_wgs;
    if (s.stride) {
      c.t_next = c.t_end - 1 + n;
      c.t_end = c.t_next + 1;
    } else {
      c.t_next = n + dev_add(&q->ticket, (uint64_t)s.chunk);
      c.t_end = c.t_next + s.chunk;
    }
  }
  const uint64_t t = c.t_next++;
  if (s.pre_only && t >= s.pre_nt) return false;
  uint64_t spins = 0, t0 = 0;
  while (!s.pre_only && t + s.lookahead >= c.tot_seen) {
    // The published tile count and the "no more packages" flag share one
    // word, so a workgroup never pairs a stale count with a fresh flag (which
    // would make it leave with a ticket that did get published).
    const uint64_t w = dev_load(&q->total);
    const uint64_t tot = max_u64(w & kTotalMask, s.pre_nt);
    c.tot_seen = tot;
    if (t + s.lookahead < tot) break;
    if (w & kTotalDone) {
      if (t < tot) break;
      return false;
    }
    // Only two tickets may claim: the one `lookahead` before the end of the
    // published tiles and the first one past it. Each belongs to exactly one
    // workgroup, so the lock is never stormed. A workgroup that has waited
    // long may also try, now and then: the designated ones may belong to
    // workgroups that are not resident yet (a grid the occupancy query
    // overestimated), and the wait must still end.
    uint32_t unlocked = 0;
    const bool overdue = spins > 4096 && (spins & 1023) == 0;
    if ((t + s.lookahead == tot || t == tot || overdue) &&
        __hip_atomic_compare_exchange_strong(&q->lock, &unlocked, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) {
      // Everything the claimer reads or writes under the lock is an
      // agent-scope atomic, performed where every XCD sees it, so the lock
      // needs no cache maintenance: its loads start after the CAS returned,
      // and the unlock waits until its stores are done.
      const uint64_t w2 = dev_load(&q->total);
      const uint64_t tot2 = max_u64(w2 & kTotalMask, s.pre_nt);
      if (!(w2 & kTotalDone) && t + s.lookahead >= tot2) {
        uint64_t g0 = 0, g1 = 0;
        bool timed_out = false;
        const uint64_t tc = now_tick();
        // slots in use: the kernel's packages plus the one claimed before the launch
        const uint32_t pre = s.pre_nt ? 1u : 0u;
        if (dev_load(&q->n_pkgs) + pre >= s.max_pkgs || !claim_package(s, &g0, &g1, &timed_out)) {
          if (timed_out || dev_load(&q->n_pkgs) + pre >= s.max_pkgs) sys_store(&s.l1->gpu_flags, 1);
          dev_store(&q->total, tot2 | kTotalDone);
        } else if (s.kind == kDynamic) {
          publish_dynamic(pay, s, tot2, g0, g1, tc);
        } else {
          publish(pay, s, tot2, g0, g1, tc);
          // A static plan fixes all of this device's bands in advance: publish
          // the rest of them now rather than one claim round trip per band.
          uint64_t tot3 = tot2 + pay.ntiles(g0, g1);
          while (s.kind == kStatic && dev_load(&q->n_pkgs) + pre < s.max_pkgs && claim_package(s, &g0, &g1, &timed_out)) {
            publish(pay, s, tot3, g0, g1, tc);
            tot3 += pay.ntiles(g0, g1);
          }
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      dev_store(&q->lock, 0u);
      continue;
    }
    if (t < tot) break;
    ++spins;
    if (waited_out(&t0, s.wait_ticks)) {
      sys_store(&s.l1->gpu_flags, 1);
      __hip_atomic_fetch_or(&q->total, kTotalDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);  // done before this workgroup counts out and the state is reset
      return false;
    }
    // waiting workgroups poll gently so the claimer's stores are not queued
    // behind their loads; those far from the published end poll least
    if (t - tot < 64)
      __builtin_amdgcn_s_sleep(4);
    else if (t - tot < 512)
      __builtin_amdgcn_s_sleep(32);
    else
      __builtin_amdgcn_s_sleep(127);
  }
  if (c.nt == 0 || t >= c.base + c.nt) {
    // Walk the publication words forward from the last package used; a
    // workgroup's tickets only grow, so it never walks back. Dynamic
    // packages all have the same tile count, so the walk starts at the
    // ticket's own package (one load instead of one per package before it).
    uint32_t p = c.nt ? c.p : 0;
    uint64_t base = c.nt ? c.base : 0;
    if (s.dyn_tiles) {
      p = (uint32_t)(t / s.dyn_tiles);
      base = (uint64_t)p * s.dyn_tiles;
    }
    for (uint64_t t1 = 0;;) {
      const uint64_t w = (p == 0 && s.pre_nt) ? pub_word(s.pre_g0, s.pre_g1 - s.pre_g0) : dev_load(&s.pub[p]);
      if (w == 0) {  // published by the claimer but not visible here yet
        if (waited_out(&t1, s.wait_ticks)) {
          sys_store(&s.l1->gpu_flags, 1);
          return false;
        }
        continue;
      }
      const uint64_t g0 = pub_g0(w), g1 = g0 + pub_size(w);
      const uint32_t nt = pay.ntiles(g0, g1);
      if (t < base + nt) {
        c.p = p;
        c.base = base;
        c.g0 = g0;
        c.g1 = g1;
        c.nt = nt;
        break;
      }
      base += nt;
      ++p;
    }
  }
  c.cur_t = t;
  *ti_out = (uint32_t)(t - c.base);
  return true;
}


// Counts this workgroup out: one atomic on the line of its blockIdx mod
// kExitLines, and one more on the shared count for the last workgroup of a
// line. True for the last workgroup of the grid.
__device__ __forceinline__ bool count_out(L2State* q) {
  const uint32_t x = blockIdx.x % kExitLines;
  const uint32_t in_line = (gridDim.x - x + kExitLines - 1) / kExitLines;
  if (dev_add(&q->exit_x[x][0], 1u) + 1 != in_line) return false;
  const uint32_t lines = gridDim.x < kExitLines ? gridDim.x : kExitLines;
  return dev_add(&q->exit_count, 1u) + 1 == lines;
}

// The last workgroup out publishes the GPU's summary to the host, clears the
// publication words and resets the level-2 state for the next run. It runs
// after every other workgroup has finished, so its loads are issued together
// and its stores drained once: each round trip here adds to the kernel.
__device__ void leave(const SchedArgs& s) {
  L2State* q = s.l2;
  // Every store of the dispenser's that the last workgroup reads or resets
  // is waited for where it is made (the claim lock, the timeout flag), so a
  // workgroup counts out without draining its tile's output stores first.
  // The last computing workgroup's end tick is read by the last gatherer:
  // with gatherers, that store is drained here.
  if (s.gather_wgs) __builtin_amdgcn_s_waitcnt(0);
  if (!count_out(q)) return;
  // without gatherers the last workgroup out is the last computing one
  const uint64_t tl = s.gather_wgs ? dev_load(&q->t_last) : now_tick();
  // with only the pre-claimed package nothing else was published; its start
  // was stamped by the workgroup of ticket 0, its end by that of its last one
  const uint64_t tf = s.pre_nt ? 0 : dev_load(&q->t_first);
  uint64_t gr = s.pre_only ? 0 : dev_load(&q->granules);
  const uint32_t np = (s.pre_only ? 0u : dev_load(&q->n_pkgs)) + (s.pre_nt ? 1u : 0u);
  const uint64_t tg = s.gather_wgs ? dev_load(&q->t_gather) : 0;
  if (s.pre_nt) {
    // the rest of the pre-claimed package's trace record
    PkgSlot* ps = &s.pkgs[0];
    ps->g0 = s.pre_g0;
    ps->g1 = s.pre_g1;
    ps->base = 0;
    ps->ntiles = s.pre_nt;
    gr += s.pre_g1 - s.pre_g0;
  } else {
    sys_store(&s.l1->gpu_t_first, tf);
  }
  // the pre-claimed package's word is never stored (workgroups build it from
  // the arguments), so with it alone there is nothing to clear
  for (uint32_t i = s.pre_only ? np : 0; i < np && i < s.max_pkgs; ++i) {
    dev_store(&s.pub[i], (uint64_t)0);
  }
  sys_store(&s.l1->gpu_t_last, tl);
  sys_store(&s.l1->gpu_granules, gr);
  sys_store(&s.l1->gpu_packages, np);
  sys_store(&s.l1->gpu_t_gather, tg);
  if (!s.pre_only) {
    dev_store(&q->ticket, (uint64_t)0);
    dev_store(&q->total, (uint64_t)0);
    dev_store(&q->n_pkgs, 0u);
    dev_store(&q->st_next, 0u);
    dev_store(&q->granules, (uint64_t)0);
    dev_store(&q->t_first, (uint64_t)0);
    dev_store(&q->lock, 0u);
  } else if (!s.stride) {
    dev_store(&q->ticket, (uint64_t)0);
  }
  if (s.gather_wgs) {
    dev_store(&q->t_last, (uint64_t)0);
    dev_store(&q->exit_compute, 0u);
    dev_store(&q->gather_next, (uint64_t)0);
    dev_store(&q->t_gather, (uint64_t)0);
  }
  for (uint32_t x = 0; x < kExitLines; ++x) dev_store(&q->exit_x[x][0], 0u);
  dev_store(&q->exit_count, 0u);
  // The host reads this word and everything else only after the kernel has
  // ended, so no store above needs to be ordered before it (a release here
  // would also write back this XCD's L2, which the end of the kernel does
  // anyway).
  sys_store(&s.l1->gpu_done, done_word(s.run_id, now_tick()));
}

// Gather (device-resident output with the host in the device set): the host
// workers publish each finished host tile as a byte range of their output
// buffer in a ring in host-coherent memory; workgroups 0 .. gather_wgs-1 read
// those ranges over PCIe and write them into the device output while the
// other workgroups compute, so no copy is left for after the kernel.
__device__ bool gather_entry(const SchedArgs& s, uint64_t* off, uint32_t* len) {
  const uint64_t j = dev_add(&s.l2->gather_next, (uint64_t)1);
  const uint64_t t0 = now_tick();
  const uint64_t want = host_final_word(s.run_id, 0) >> 40;
  for (;;) {
    if (j < s.ring_cap) {
      const uint64_t w = __hip_atomic_load(const_cast<uint64_t*>(&s.ring[j]), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
      if (w != 0) {
        *off = ring_off(w);
        *len = (uint32_t)ring_len(w);
        return true;
      }
    }
    const uint64_t f = sys_load(&s.l1->host_final);
    if ((f >> 40) == want && j >= (f & ((1ull << 40) - 1))) return false;
    if (now_tick() - t0 > s.gather_wait_ticks) {
      sys_store(&s.l1->gpu_flags, 2);
      return false;
    }
    __builtin_amdgcn_s_sleep(8);
  }
}

// Host memory is reached over PCIe with a latency of microseconds, so each
// thread issues a batch of independent loads before it stores any of them.
// The loads are system-scope atomics: a plain load could be served from a
// line this XCD cached while copying a neighbouring tile that shares it,
// before the host had written this tile's part (ragged rows share lines).
__device__ void gather_copy(const SchedArgs& s, uint64_t off, uint32_t len) {
  constexpr uint32_t kBatch = 8;
  const char* src = s.gsrc + off;
  char* dst = s.gdst + off;
  if (((off | len) & 7u) == 0) {
    uint64_t* a = reinterpret_cast<uint64_t*>(const_cast<char*>(src));
    uint64_t* b = reinterpret_cast<uint64_t*>(dst);
    const uint32_t n = len / 8;
    for (uint32_t i0 = 0; i0 < n; i0 += kBlockThreads * kBatch) {
      uint64_t v[kBatch];
#pragma unroll
      for (uint32_t k = 0; k < kBatch; ++k) {
        const uint32_t i = i0 + k * kBlockThreads + threadIdx.x;
        if (i < n) v[k] = __hip_atomic_load(a + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
#pragma unroll
      for (uint32_t k = 0; k < kBatch; ++k) {
        const uint32_t i = i0 + k * kBlockThreads + threadIdx.x;
        if (i < n) b[i] = v[k];
      }
    }
  } else {
    uint32_t* a = reinterpret_cast<uint32_t*>(const_cast<char*>(src));
    uint32_t* b = reinterpret_cast<uint32_t*>(dst);
    const uint32_t n = len / 4;
    for (uint32_t i0 = 0; i0 < n; i0 += kBlockThreads * kBatch) {
      uint32_t v[kBatch];
#pragma unroll
      for (uint32_t k = 0; k < kBatch; ++k) {
        const uint32_t i = i0 + k * kBlockThreads + threadIdx.x;
        if (i < n) v[k] = __hip_atomic_load(a + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
#pragma unroll
      for (uint32_t k = 0; k < kBatch; ++k) {
        const uint32_t i = i0 + k * kBlockThreads + threadIdx.x;
        if (i < n) b[i] = v[k];
      }
    }
  }
}

// Persistent workgroup loop. Every branch around the barriers is uniform
// across the workgroup: the claim block is entered by the whole first wave
// (readfirstlane of the thread id) and only its lane 0 touches the
// dispenser; the loop exit reads the shared flag through readfirstlane.
// With a per-lane "thread 0 only" condition instead, the compiler may
// rotate the loop so that lane 0 leaves an inner loop through an exec-mask
// update while the other lanes keep passing the barriers, which never ends.
template <class T>
__global__ __launch_bounds__(kBlockThreads, T::kMinBlocksPerCu) void k_persistent(T pay, SchedArgs s) {
  __shared__ uint32_t sh_go, sh_p, sh_ti;
  __shared__ uint64_t sh_g0, sh_g1;
  const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) == 0;
  const bool lane0 = threadIdx.x == 0;
  pay.load_constants();
  // Direct phase. The tickets of the package the host claimed before the
  // launch need nothing from the dispenser: workgroup w runs them straight
  // from the arguments (w, w + n, w + 2n ... with round-robin tickets; only
  // its first one with atomic tickets), with no cursor and no barrier of the
  // dispenser's. Only the designated claimer's ticket (lookahead before the
  // package's end, when more packages may follow) goes through the cursor,
  // so that the claim still overlaps the other workgroups' tiles; when the
  // package does not fill the grid, a workgroup left without a ticket claims
  // at once anyway, and that ticket runs directly too (a claim before it
  // would delay a tile that may be among the longest).
  const bool computing = blockIdx.x >= s.gather_wgs;
  const uint32_t n_comp = gridDim.x - s.gather_wgs;
  const uint64_t t_first = computing ? blockIdx.x - s.gather_wgs : 0;
  const bool claim_free = s.pre_only || s.pre_nt < n_comp;
  // After the direct phase the scheduler arguments are read from LDS only.
  // Kept in scalar registers across the payload they would crowd out its
  // own; and every argument the kernel names directly is loaded as it
  // starts (the compiler places those loads at the entry), where beyond the
  // few fields of the direct phase they would spill and hold up every
  // workgroup's first tile. So the lanes copy the argument block word by
  // word from the kernel-argument segment, through an address the compiler
  // cannot see through, so that it neither moves the copy to the entry nor
  // splits it into pieces staged in scratch (taking the address of the
  // argument itself would make a private copy of it). The block lies at its
  // ABI offset: the arguments are laid out in order, each at its own
  // alignment. Each lane's word is loaded here (a relaxed atomic load, which
  // the compiler keeps where it is written) and stored after the direct
  // tiles, so that its latency hides behind them instead of lengthening the
  // workgroup's end.
  static_assert(sizeof(SchedArgs) % 4 == 0 && sizeof(SchedArgs) / 4 <= kBlockThreads, "one word per lane");
  constexpr uint32_t kArgWords = sizeof(SchedArgs) / 4;
  uint32_t arg_word = 0;
  {
    constexpr size_t kOffset = (sizeof(T) + alignof(SchedArgs) - 1) / alignof(SchedArgs) * alignof(SchedArgs);
    uint64_t seg = reinterpret_cast<uint64_t>(__builtin_amdgcn_kernarg_segment_ptr());
    asm volatile("" : "+s"(seg));
    uint32_t __attribute__((address_space(1)))* src =
        reinterpret_cast<uint32_t __attribute__((address_space(1)))*>(seg + kOffset);
    if (threadIdx.x < kArgWords)
      arg_word = __hip_atomic_load(src + threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  uint64_t t_dir = t_first;  // first ticket the direct phase did not run
  if (computing && s.pre_nt) {
    if (t_first == 0 && lane0) {
      // the pre-claimed package starts with the first workgroup
      const uint64_t tp = now_tick();
      dev_store(&s.pkgs[0].t_claim, tp);
      sys_store(&s.l1->gpu_t_first, tp);
    }
    while (t_dir < s.pre_nt && (claim_free || t_dir + s.lookahead != s.pre_nt)) {
      pay.run(s.pre_g0, s.pre_g1, (uint32_t)t_dir);
      if (t_dir + 1 == s.pre_nt && lane0) dev_store(&s.pkgs[0].t_end, now_tick());  // its last ticket
      if (!s.stride) {
        t_dir = ~0ull;  // later tickets come from the counter
        break;
      }
      t_dir += n_comp;
    }
  }
  // The argument block into LDS (the barrier also ends the direct tiles' use
  // of the payload's own LDS).
  __shared__ SchedArgs sh_args;
  if (threadIdx.x < kArgWords) reinterpret_cast<uint32_t*>(&sh_args)[threadIdx.x] = arg_word;
  __syncthreads();
  const SchedArgs& sa = sh_args;
  // The next run's queue state (the other buffer) is cleared now, while
  // nothing uses it, so that no workgroup has to reset anything as it
  // leaves. Agent-scope stores: they reach memory, where the next run's
  // atomics read them, whichever XCD runs them.
  if (sa.l2_next) {
    constexpr uint32_t kStateWords = sizeof(L2State) / sizeof(uint64_t);
    uint64_t* const st = reinterpret_cast<uint64_t*>(sa.l2_next);
    const uint32_t words = kStateWords + sa.pub_next_words;
    for (uint32_t i = blockIdx.x * kBlockThreads + threadIdx.x; i < words; i += gridDim.x * kBlockThreads)
      dev_store(i < kStateWords ? &st[i] : &sa.pub_next[i - kStateWords], (uint64_t)0);
  }
  // The cursor lives in LDS too: only lane 0 of wave 0 uses it, and keeping
  // it in registers across the tile loop would cost the payload occupancy.
  __shared__ Cursor sh_cursor;
  Cursor& c = sh_cursor;
  if (wave0) {
    if (lane0) {
      c = Cursor{};
      if (t_dir == ~0ull) {
        c.t_next = c.t_end = 1;  // the next ticket comes from the counter
      } else {
        c.t_next = t_dir;  // the first ticket needs no atomic
        c.t_end = t_dir + 1;
      }
      c.tot_seen = sa.pre_nt;
    }
  }
  uint32_t prev_p = 0xFFFFFFFFu;
  if (!computing) {
    __shared__ uint64_t sh_off;
    __shared__ uint32_t sh_len;
    for (;;) {
      if (wave0) {
        if (lane0) {
          uint64_t off = 0;
          uint32_t len = 0;
          sh_go = gather_entry(sa, &off, &len) ? 1u : 0u;
          sh_off = off;
          sh_len = len;
        }
      }
      __syncthreads();
      if (__builtin_amdgcn_readfirstlane(sh_go) == 0) break;
      const uint64_t off = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(sh_off >> 32)) << 32) |
                           __builtin_amdgcn_readfirstlane((uint32_t)sh_off);
      const uint32_t len = __builtin_amdgcn_readfirstlane(sh_len);
      gather_copy(sa, off, len);
      if (wave0) {
        if (lane0) {
          sys_fetch_add(&sa.l1->gathered, (uint64_t)len);  // progress for the host's throttle
          __hip_atomic_fetch_max(&sa.l2->t_gather, now_tick(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      __syncthreads();
    }
    if (wave0) {
      if (lane0) leave(sa);
    }
    return;
  }
  for (;;) {
    if (wave0) {
      if (lane0) {
        uint32_t p = 0, ti = 0;
        uint64_t g0 = 0, g1 = 0;
        bool go;
        if (prev_p != 0xFFFFFFFFu) tile_finished(sa, c);
        go = next_tile(pay, sa, c, &ti);
        p = c.p;
        g0 = c.g0;
        g1 = c.g1;
        sh_go = go ? 1u : 0u;
        sh_p = p;
        sh_ti = ti;
        sh_g0 = g0;
        sh_g1 = g1;
      }
    }
    __syncthreads();
    const uint32_t go = __builtin_amdgcn_readfirstlane(sh_go);
    if (go == 0) break;
    const uint32_t p = __builtin_amdgcn_readfirstlane(sh_p);
    const uint32_t ti = __builtin_amdgcn_readfirstlane(sh_ti);
    const uint64_t g0 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(sh_g0 >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)sh_g0);
    const uint64_t g1 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(sh_g1 >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)sh_g1);
    // Nothing of the scheduler's may still be in flight when the payload
    // starts: its pointers come from LDS, so its accesses are flat ones,
    // which count against the LDS counter too; with one pending, every LDS
    // wait inside the payload would have to drain all of them.
    __builtin_amdgcn_s_waitcnt(0);
    pay.run(g0, g1, ti);
    prev_p = p;
    __syncthreads();  // the tile is complete and the shared slots may be reused
  }
  if (wave0) {
    if (lane0) {
      if (sa.wg_end) {
        // light exit: the loop's last barrier has seen every wave's tiles
        // done; the next run's state is already clear
        sys_store(&sa.wg_end[blockIdx.x], now_tick());
      } else {
        // the last computing workgroup out marks the end of the GPU's work
        // (gather workgroups may still be copying the host's output)
        if (sa.gather_wgs && dev_add(&sa.l2->exit_compute, 1u) + 1 == gridDim.x - sa.gather_wgs)
          dev_store(&sa.l2->t_last, now_tick());
        leave(sa);
      }
    }
  }
}

// Direct kernel: the GPU's whole share is the package the host claimed
// before the launch (a run on the GPU alone, or a Static plan that gives it
// one package) and its tiles cost alike, so workgroup w runs tickets w,
// w + n, w + 2n ... straight from the arguments. Each workgroup leaves the
// tick at which it ended; the host takes the GPU's end from these ticks and
// writes the package's trace record itself. Kept apart from the persistent
// kernel so that it carries none of the dispenser's code or registers.
template <class T>
__global__ __launch_bounds__(kBlockThreads, T::kMinBlocksPerCu) void k_direct(T pay, DirectArgs d) {
  const bool lane0 = threadIdx.x == 0;
  pay.load_constants();
  if (blockIdx.x == 0 && lane0) {
    const uint64_t tp = now_tick();
    dev_store(&d.pkgs[0].t_claim, tp);
    sys_store(&d.l1->gpu_t_first, tp);
  }
  for (uint32_t i = blockIdx.x; i < d.ntiles; i += gridDim.x) {
    // Swizzled: the hardware deals workgroup i to XCD i mod 8, so without it
    // the tiles at one position of every group of eight (escape-time: one
    // column block of every row, when a row holds eight) would all land on
    // one XCD. Within each whole group of eight the tiles are rotated by the
    // group's index instead, so every XCD meets every position in turn.
    uint32_t t = i;
    if (d.swizzle) {
      const uint32_t j = i / 8;
      if (8 * j + 8 <= d.ntiles) t = 8 * j + (i + j) % 8;
    }
    pay.run(d.g0, d.g1, t);
  }
  __syncthreads();  // every wave's tiles are done
  if (lane0) sys_store(&d.wg_end[blockIdx.x], now_tick());
}

template <class T>
__global__ __launch_bounds__(kBlockThreads) void k_bare(T pay, uint64_t G) {
  pay.load_constants();
  pay.run(0, G, blockIdx.x);
}

}  // namespace ce
