/*
 * coexec.h -- C ABI of the MI355X co-execution engine.
 *
 * One massive data-parallel kernel is co-executed over an N-dimensional index
 * space by one MI355X (a persistent HIP kernel pulling packages from a
 * dispenser) and the host CPU cores (a worker pool pulling from the same
 * dispenser). The calls follow the programming model of the paper (sections
 * 4.2 and 6): pick the devices, set the index space, pick a scheduler, bind a
 * program (kernel, inputs, outputs, output pattern), run synchronously, then
 * read statistics, the package trace and the error list.
 *
 * Conventions shared by every call:
 *  - Every function returning ce_status returns CE_OK (0) or a negative code;
 *    a failure is also appended to the engine's error list (section 6.1:
 *    errors are collected, not thrown). No C++ exception crosses the ABI and
 *    no call aborts the process.
 *  - Pointers passed in are borrowed: the caller owns host and device memory,
 *    which must stay valid and unmodified until ce_engine_run returns.
 *    "Device pointer" means HIP device memory of the engine's GPU (e.g. a
 *    PyTorch tensor's data_ptr); "host pointer" means ordinary or pinned host
 *    memory.
 *  - An engine is not thread-safe: calls on one engine must not overlap.
 *    Different engines may be used from different threads.
 */
#ifndef COEXEC_H
#define COEXEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ce_status;
#define CE_OK 0
#define CE_E_INVALID (-1)     /* bad argument, size mismatch, unbound slot      */
#define CE_E_STATE (-2)       /* call not allowed in the engine's current state */
#define CE_E_NOMEM (-3)       /* host or device allocation failed               */
#define CE_E_DEVICE (-4)      /* HIP error, or no usable GPU                    */
#define CE_E_UNSUPPORTED (-5) /* valid request the engine does not implement    */
#define CE_E_BUDGET (-6)      /* server: job larger than the HBM budget         */
#define CE_E_TIMEOUT (-7)     /* a device did not finish within the deadline    */

/* Devices (section 6: device masks). Device index order inside the engine is
 * fixed: the GPU (if used) is device 0, the host worker pool the next one. */
#define CE_DEV_GPU 1u
#define CE_DEV_HOST 2u
#define CE_MAX_DEVICES 2

/* Payload kernels: the paper's benchmark programs used on the hot path
 * (section 7.2, Table 2). */
#define CE_KERNEL_ESCAPE 1    /* escape-time fractal (Mandelbrot), 2-D, 0 in : 1 out  */
#define CE_KERNEL_BLUR5 2     /* 5x5 Gaussian blur, 2-D, 2 in (image, weights) : 1 out */
#define CE_KERNEL_NBODY_ACC 3 /* all-pairs N-body acceleration, 1-D, 1 in : 1 out      */
#define CE_KERNEL_NBODY_STEP 4 /* N-body integration step, 1-D, 2 in (pos, vel) : 2 out (pos, vel) */
#define CE_KERNEL_BINOMIAL 5    /* binomial option pricing, 1-D, 2 in (spots, leaf factors) : 1 out,
                                   out pattern 1 : steps+1                                         */
#define CE_KERNEL_RUNTIME 6     /* a payload given as HIP source at run time (ce_program_source), 1-D */

/* Schedulers (section 5.3). */
#define CE_SCHED_STATIC 0
#define CE_SCHED_DYNAMIC 1
#define CE_SCHED_HGUIDED 2
/* Static delivery order (section 7.3: "Static" puts the host's part first
 * along the index space, "Static rev" the GPU's). */
#define CE_ORDER_HOST_FIRST 0
#define CE_ORDER_GPU_FIRST 1

/* Escape-time parameters. Pixel (r, c), 0 <= r < h, 0 <= c < w, has
 * c = (x0 + c*dx) + i (y0 + r*dy); output uint32 count in [1, max_iter]. */
typedef struct {
  uint32_t w, h;
  float x0, y0, dx, dy;
  uint32_t max_iter;
} ce_escape_params;

/* Blur parameters: image w x h FP32 row-major in slot 0, 25 FP32 weights in
 * slot 1 (row-major over dy = -2..2, dx = -2..2); output w x h FP32. */
typedef struct {
  uint32_t w, h;
} ce_blur5_params;

/* N-body parameters: n bodies as float4 (x, y, z, m) in slot 0; output n
 * float4 (ax, ay, az, 0). eps2 > 0 is the squared softening. strict != 0
 * evaluates 1/sqrt by Lomont's method so that GPU and host results are
 * bitwise identical; strict == 0 uses the GPU's hardware reciprocal square
 * root and the host's correctly rounded 1/sqrtf (results then agree within a
 * tolerance, not bitwise). */
typedef struct {
  uint32_t n;
  float eps2;
  uint32_t strict;
} ce_nbody_params;

/* N-body integration step (the NBody program of section 6.2: positions and
 * velocities in, positions and velocities out, a time step and a squared
 * softening). Slot 0 in: n float4 (x, y, z, m); slot 1 in: n float4
 * (vx, vy, vz, w). With a_i the acceleration of CE_KERNEL_NBODY_ACC, each body
 * moves by the constant-acceleration step over dt, per component in FP32 as
 * h = (dt*dt)*0.5, x' = (x + v*dt) + a*h, v' = v + a*dt. Slot 0 out: n float4
 * (x', y', z', m); slot 1 out: n float4 (vx', vy', vz', w). Outputs must not
 * alias inputs (every body reads every position); time stepping swaps two
 * pairs of buffers. eps2 and strict as for CE_KERNEL_NBODY_ACC; dt finite. */
typedef struct {
  uint32_t n;
  float eps2;
  float dt;
  uint32_t strict;
} ce_nbody_step_params;

/* Binomial option pricing (the Binomial Options program of sections 6.1 and
 * 7.2): European calls priced on a Cox-Ross-Rubinstein tree of `steps`
 * steps (1..255). One work-group of steps+1 work-items prices four options
 * (one float4 of spots) and writes one float4 of prices: the index space is
 * gws = (steps+1) * n_groups with lws = steps+1, and the out pattern is one
 * output element per steps+1 work-items (section 6.1's 1:255 for 254 steps).
 * Slot 0 in: n_groups float4 spot prices; slot 1 in: steps+1 FP32 leaf
 * factors f_j = u^(2j-steps). Out: n_groups float4 prices. In FP32: leaves
 * V_j = max(S*f_j - strike, 0), then for each level L = steps-1 .. 0 and
 * j = 0..L, V_j = pu*V_{j+1} + pd*V_j (two products, then their sum); the
 * price is V_0. ce_binomial_table gives the factors, pu and pd. */
typedef struct {
  uint32_t n_groups;
  uint32_t steps;
  float strike;
  float pu;  /* discounted up probability   */
  float pd;  /* discounted down probability */
} ce_binomial_params;

/* Scheduler description (section 5.3). Arrays are indexed by engine device
 * index (GPU = 0 when used, then host).
 *  STATIC : props[0..n-2] = fraction of each device but the last, which gets
 *           the remainder (section 6.2 listing); order = CE_ORDER_*;
 *           n_packages > 0 cuts the space into that many equal bands first
 *           and hands each device whole bands (every device gets >= 1 band).
 *  DYNAMIC: equal packages of package_granules granules, or, when that is 0,
 *           ceil(G / n_packages) granules; handed in index order to whichever
 *           device asks; the last package may be short.
 *  HGUIDED: package for device i = max(min_granules[i],
 *           floor(G_r * power[i] / (k * n * sum_j power[j]))), cut to the
 *           pending granules G_r. power[i] in [1, 2^20]; k >= 1;
 *           min_granules[i] == 0 selects the default (GPU: one tile per
 *           resident workgroup; host: one host tile per worker thread). */
typedef struct {
  int32_t kind;
  int32_t order;
  uint32_t n_packages;
  uint32_t k;
  uint64_t package_granules;
  double props[CE_MAX_DEVICES];
  uint64_t power[CE_MAX_DEVICES];
  uint64_t min_granules[CE_MAX_DEVICES];
} ce_sched_desc;

/* Statistics of the last run. Times are seconds on the host's steady clock,
 * measured from the start of ce_engine_run. t_device[d] is the end of device
 * d's last package (0 if it got none). */
typedef struct {
  double t_run;                       /* whole ce_engine_run call            */
  double t_device[CE_MAX_DEVICES];    /* finish time of each device           */
  double t_gpu_kernel;                /* GPU persistent kernel, first to last package end */
  uint64_t granules[CE_MAX_DEVICES];  /* granules computed by each device     */
  uint64_t items[CE_MAX_DEVICES];     /* work-items computed by each device   */
  uint64_t packages[CE_MAX_DEVICES];  /* packages taken by each device        */
  uint32_t n_devices;
  uint32_t device_kind[CE_MAX_DEVICES]; /* CE_DEV_GPU or CE_DEV_HOST          */
  double balance;                     /* min_d t_device / max_d t_device (section 7.3) */
  uint64_t total_granules;
  uint64_t total_items;
  uint32_t gpu_workgroups;            /* persistent grid size of the last run */
  uint32_t host_threads;              /* host worker threads of the last run  */
  double t_gather;                    /* end of the GPU's last copy of host output into
                                       * the device output (0: no such copies)  */
  uint64_t gathered_bytes;            /* bytes of host output the GPU copied     */
  /* where the calling thread's time went (seconds from the start of the
   * run; 0 for phases the run did not have): the GPU kernel launched, the
   * host device's share finished, the GPU's first workgroup seen starting
   * (only in runs that re-anchor the GPU clock mapping, one every 5 ms at
   * most), the GPU's stream synchronised, the host's output copies into
   * HBM drained */
  double t_launched, t_host_done, t_gpu_seen, t_synced, t_copies_done;
} ce_run_stats;

/* One package of the last run (section 5 "Introspector"): device, granule
 * range and times (seconds from run start; GPU times mapped onto the host
 * clock by a calibration done at engine creation). */
typedef struct {
  uint32_t device;
  uint32_t pad;
  uint64_t begin, end; /* granules [begin, end) */
  double t_claim, t_end;
} ce_package_rec;

typedef struct ce_engine ce_engine;

/* Creates an engine: initialises HIP on the GPU (ordinal 0 by default), the
 * host-coherent dispenser memory, the clock calibration and the host pool.
 * Fails with CE_E_DEVICE if no gfx950 GPU is present. *out is NULL on error. */
ce_status ce_engine_create(ce_engine** out);
/* Releases every resource of the engine; NULL-safe. */
void ce_engine_destroy(ce_engine* e);

/* Device set (section 6: engine.use). dev_mask = CE_DEV_GPU | CE_DEV_HOST;
 * gpu_ordinal selects the HIP device (must match the engine's GPU, i.e. the
 * one current at creation); host_threads <= 0 uses every host core. */
ce_status ce_engine_use(ce_engine* e, uint32_t dev_mask, int gpu_ordinal, int host_threads);
/* Index space (section 6: work_items). ndim 1 or 2; gws[0] is the fastest
 * dimension. The granule -- the smallest package -- is one row (gws[0]
 * items) for 2-D spaces and lws[0] items for 1-D spaces. lws may be NULL
 * (1-D default 256). The space must match the bound kernel's parameters. */
ce_status ce_engine_work_items(ce_engine* e, uint32_t ndim, const uint64_t* gws, const uint32_t* lws);
/* Scheduler (section 6.2: engine.scheduler). The descriptor is copied. */
ce_status ce_engine_scheduler(ce_engine* e, const ce_sched_desc* s);
/* HIP stream (hipStream_t) the GPU work is ordered on; NULL = the engine's
 * own stream. The stream is borrowed. */
ce_status ce_engine_stream(ce_engine* e, void* hip_stream);

/* Program (section 6: Program::kernel / in / out / out_pattern). params is
 * copied; params_size must equal the size of the kernel's parameter struct. */
ce_status ce_program_kernel(ce_engine* e, int kernel_id, const void* params, size_t params_size);
/* Binds input slot `slot`. At least one of host_ptr / dev_ptr must be given.
 * The GPU reads dev_ptr (or a device copy the engine makes of host_ptr); the
 * host workers read host_ptr (or a host copy the engine makes of dev_ptr).
 * bytes must equal the slot's size for the bound kernel. */
ce_status ce_program_in(ce_engine* e, uint32_t slot, const void* host_ptr, const void* dev_ptr, size_t bytes);
/* Binds output slot `slot` (0, or 0 and 1 for CE_KERNEL_NBODY_STEP). After a
 * successful run the whole output is in every pointer given (host_ptr and/or
 * dev_ptr). Every output slot of the kernel must be bound before a run. */
ce_status ce_program_out(ce_engine* e, uint32_t slot, void* host_ptr, void* dev_ptr, size_t bytes);
/* Output pattern outs:items (section 4.2): each package of `items` work-items
 * writes `outs` output elements. The payloads here write one element per
 * work-item, so only 1:1 is accepted (others: CE_E_UNSUPPORTED). */
ce_status ce_program_out_pattern(ce_engine* e, uint32_t outs, uint32_t items);

/* ---- payloads supplied at run time (section 3: each device may need its own
 * kernel, given as source or binary; section 6.2: a device is declared with
 * its own kernel). The GPU's version is HIP C++ source compiled with hipRTC
 * for gfx950 when it is programmed; the host workers' version is a C
 * function. The two are separate implementations of one work-item function
 * and must agree bit for bit where the caller needs identical results.
 *
 * Arguments (the generic form of a kernel's argument list): every work-item
 * receives the buffers of the bound slots, inputs first (buf[0..n_in)), then
 * outputs (buf[n_in..n_in+n_out)), as device pointers on the GPU and host
 * pointers on the host, and a block of scalar bytes copied at programming
 * time. Work-item i (0 <= i < gws) writes out_item_bytes bytes at byte
 * offset i * out_item_bytes of each output (output pattern 1:1); it may read
 * any part of the inputs. The index space is 1-D; a granule is lws work-items. */
#define CE_RT_MAX_BUFS 4
#define CE_RT_SCALAR_BYTES 128
typedef struct {
  void* buf[CE_RT_MAX_BUFS];
  unsigned char scalars[CE_RT_SCALAR_BYTES];
} ce_rt_args;
/* Host version: computes work-items [i0, i1) and returns 0, or a nonzero
 * code if it could not. A failure is collected, not thrown (section 6.1):
 * the host device claims no further package, the other devices go on, and
 * the run returns CE_E_DEVICE with an error naming the items and the code
 * (the failed items' outputs are unspecified). */
typedef int32_t (*ce_rt_host_fn)(uint64_t i0, uint64_t i1, const ce_rt_args* a);
typedef struct {
  const char* source;         /* HIP C++ source; must define `entry` as
                               *   __device__ void entry(uint64_t i, const ce_rt_args* a)
                               * (ce_rt_args and <stdint.h> are already declared) */
  const char* entry;          /* name of that function (a C identifier)           */
  ce_rt_host_fn host;         /* host workers' version; NULL: GPU only            */
  uint32_t n_in, n_out;       /* 0..2 inputs, 1..2 outputs                        */
  uint64_t in_bytes[2];       /* size of each input buffer                        */
  uint32_t out_item_bytes;    /* bytes per work-item in every output (1..256)     */
  uint32_t scalar_bytes;      /* 0..CE_RT_SCALAR_BYTES                            */
  const void* scalars;        /* copied                                           */
} ce_rt_desc;
/* Compiles desc->source for gfx950 and binds the result as the engine's
 * payload (kernel id CE_KERNEL_RUNTIME), replacing any bound payload and
 * unbinding the slots. On a compile error returns CE_E_INVALID and writes
 * the compiler's log (NUL-terminated, truncated) into log[0..log_len) if
 * log is not NULL; the previous payload is then unbound too. Slots are then
 * bound with ce_program_in / ce_program_out as for the fixed payloads
 * (input sizes in_bytes, output sizes gws * out_item_bytes, so the index
 * space must be set before the outputs are bound). A run whose device set
 * includes the host needs desc->host; the host function is called from
 * several host worker threads at once, on disjoint item ranges. */
ce_status ce_program_source(ce_engine* e, const ce_rt_desc* desc, char* log, size_t log_len);
/* Compiles a runtime payload's source without binding it (no GPU needed):
 * CE_OK, or CE_E_INVALID with the compiler's log as above. */
ce_status ce_rt_compile_check(const char* source, const char* entry, char* log, size_t log_len);
/* As ce_rt_compile_check, and hands out the gfx950 code object (an ELF
 * shared object holding the payload's persistent and plain kernels): *size
 * receives its length; it is copied into buf when cap >= *size (buf may be
 * NULL to ask for the size). For inspecting what the GPU will run. */
ce_status ce_rt_code_object(const char* source, const char* entry, void* buf, size_t cap, size_t* size, char* log,
                            size_t log_len);
/* Plain single launch of the engine's bound runtime payload over gws
 * work-items of granule lws (the "native" side of the overhead metric):
 * device pointers, ins[] / outs[] follow its slots, on `hip_stream`. */
ce_status ce_engine_bare_run_source(ce_engine* e, uint64_t gws, uint32_t lws, const void* const* ins,
                                    void* const* outs, void* hip_stream, int sync);

/* How the host's share of a device-resident output (output bound only as a
 * device pointer, host in the device set) reaches HBM during the run
 * (section 4.2 output pattern, 1:1):
 *  CE_MERGE_DMA (default): as each host package finishes, its output range
 *    is copied host -> device by the GPU's system DMA engines (split over up
 *    to four of them), which need no compute unit and so run beside the
 *    GPU's kernel; the run returns once every copy has landed. Refused with
 *    CE_E_UNSUPPORTED if the GPU exposes no host-to-device copy engine; an
 *    engine is then created with CE_MERGE_GPU_GATHER.
 *  CE_MERGE_GPU_GATHER: a few workgroups of the GPU's kernel copy each
 *    finished host tile over PCIe into HBM while the others compute (their
 *    long PCIe loads slow the workgroups that share their compute units).
 *    Single-output kernels only: a run of a kernel with two outputs that
 *    needs this merge fails with CE_E_UNSUPPORTED.
 * Either way the host claims new packages only while less than 512 KiB of
 * its output is still waiting to be copied. */
#define CE_MERGE_DMA 0
#define CE_MERGE_GPU_GATHER 1
ce_status ce_engine_output_merge(ce_engine* e, int mode);

/* Bounds, in seconds, on the waits inside the GPU kernel for the following
 * runs (0 keeps the default): dispenser_s for a workgroup waiting on the
 * dispenser (a claim, a package to appear; default 5 s, far above the
 * microseconds these take), gather_s for a gather workgroup waiting for the
 * host's next finished tile (CE_MERGE_GPU_GATHER; default 60 s; it must
 * exceed the host's longest package). A wait that runs out ends the GPU's
 * part of the run early and the run returns CE_E_TIMEOUT, the other devices
 * having finished theirs; the kernel still ends normally and the engine is
 * ready for the next run. Errors: CE_E_INVALID for a negative value or one
 * above 3600. */
ce_status ce_engine_wait_bounds(ce_engine* e, double dispenser_s, double gather_s);

/* Number of workgroups of the GPU's persistent kernel for the following
 * runs; 0 (the default) lets the engine choose: for T tiles of the whole
 * index space, R resident workgroups (occupancy x compute units) and C
 * compute units, the largest g <= min(T, R) that minimises
 * ceil(T / g) * ceil(g / C), the tiles run by the busiest compute unit
 * (whole rounds, spread evenly over the CUs); except that a run whose GPU
 * share is one package (the direct kernel) of equal-cost tiles with at
 * least 4 R tiles, or of escape-time or runtime-payload tiles with more
 * than 4 R, and at most 65536 tiles, gets one workgroup per tile, dealt by
 * the hardware as a plain launch is (uneven tiles swizzled over the XCDs).
 * A caller's value is used as
 * given (it may exceed what fits on the GPU at once: the dispenser's
 * waits do not depend on every workgroup being resident), plus the gather
 * workgroups of CE_MERGE_GPU_GATHER. Affects speed only, never results.
 * Errors: CE_E_INVALID for a value above 2^20. */
ce_status ce_engine_gpu_workgroups(ce_engine* e, uint32_t workgroups);

/* Records the caller's HIP events (hipEvent_t handles) on the engine's
 * stream immediately before and after the GPU kernel of each following run,
 * so the caller can time the kernel with hipEventElapsedTime. NULL, NULL
 * stops recording. The events are borrowed. */
ce_status ce_engine_kernel_events(ce_engine* e, void* start_event, void* stop_event);

/* Runs the bound program synchronously (section 6: engine.run): on return
 * every output pointer holds the full result, or the call failed and outputs
 * are unspecified. */
ce_status ce_engine_run(ce_engine* e);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): runs the
 * bound program like ce_engine_run, GPU alone, without allocating. The
 * queue state, publication words and package table live in a static device
 * array of 1 MiB per GPU (held until the process ends) instead of memory the
 * engine allocates, so at most (1 MiB - queue state) / 72 B packages, about
 * 14,000, may be scheduled: a Dynamic or HGuided schedule that could need
 * more returns CE_E_INVALID before anything runs. The array is cleared by a
 * fill kernel on the engine's stream at the start of every run. Every bound
 * input and output must have a device pointer and no output a host pointer
 * (CE_E_UNSUPPORTED otherwise, as for a device set other than CE_DEV_GPU).
 * All engines on one GPU share the array: runs of this call that overlap
 * on one GPU race and give wrong results. Stats and trace work as after
 * ce_engine_run. */
ce_status ce_engine_run_noalloc(ce_engine* e);

/* Statistics of the last successful run. */
ce_status ce_engine_stats(const ce_engine* e, ce_run_stats* out);
/* Copies up to cap package records of the last run into buf (may be NULL
 * with cap 0) and returns the total number of packages. */
size_t ce_engine_trace(const ce_engine* e, ce_package_rec* buf, size_t cap);

/* Error list (section 6.1: has_errors / get_errors). The string is owned by
 * the engine and valid until the next call that changes the list. */
int ce_engine_has_errors(const ce_engine* e);
int ce_engine_error_count(const ce_engine* e);
const char* ce_engine_error(const ce_engine* e, int i);
void ce_engine_clear_errors(ce_engine* e);

/* ---- batched form ------------------------------------------------------
 * Many escape-time jobs of uneven sizes run as ONE persistent kernel launch
 * over the concatenation of their tiles, captured once in a hipGraph and
 * replayed, instead of one launch per job. The tile shape (tile_rows x
 * tile_cols, 256 pixels) and the tiles taken per workgroup request
 * (package_tiles, a Dynamic schedule inside the GPU, section 5.3) are chosen
 * by ce_batch_tune, which times every candidate on the batch itself. The
 * per-pixel arithmetic is that of CE_KERNEL_ESCAPE. GPU only. */
typedef struct ce_batch ce_batch;
typedef struct {
  uint32_t tile_rows;     /* 1, 2, 4, 8 or 16; tile_cols = 256 / tile_rows */
  uint32_t tile_cols;     /* output of ce_batch_get_config / ce_batch_tune  */
  uint32_t package_tiles; /* tiles per workgroup request, >= 1              */
} ce_batch_config;
typedef struct {
  uint32_t jobs;
  uint32_t workgroups;    /* persistent grid of the last build             */
  uint64_t items;         /* pixels over all jobs                          */
  uint64_t total_tiles;
  uint32_t tile_rows, tile_cols, package_tiles;
  uint32_t pad;
  double t_run;           /* seconds, last ce_batch_run / run_separate call */
  double t_gpu_ms;        /* GPU time of that call (HIP events)            */
  uint64_t launches;      /* graph launches so far                         */
} ce_batch_report;
/* hip_stream may be NULL (the batch creates its own stream). */
ce_status ce_batch_create(ce_batch** out, void* hip_stream);
void ce_batch_destroy(ce_batch* b);
/* Appends a job; dev_out is a device buffer of h*w uint32, owned by the
 * caller and valid while the batch uses it. At most 4096 jobs. */
ce_status ce_batch_add_escape(ce_batch* b, const ce_escape_params* p, void* dev_out, uint32_t* index);
ce_status ce_batch_clear(ce_batch* b);
ce_status ce_batch_set_config(ce_batch* b, const ce_batch_config* c);
ce_status ce_batch_get_config(const ce_batch* b, ce_batch_config* c);
/* Times every (tile shape, package size) candidate reps times on the
 * current jobs, keeps the fastest and writes it to *chosen (may be NULL).
 * Every candidate writes the outputs, so they hold a valid result after. */
ce_status ce_batch_tune(ce_batch* b, uint32_t reps, ce_batch_config* chosen);
/* One graph launch of the whole batch, synchronous. The graph is rebuilt
 * only when jobs or the configuration changed. */
ce_status ce_batch_run(ce_batch* b);
/* Baseline: one plain grid launch per job on the same stream, synchronous. */
ce_status ce_batch_run_separate(ce_batch* b);
ce_status ce_batch_stats(const ce_batch* b, ce_batch_report* s);
/* Message of the last failed call (owned by the batch). */
const char* ce_batch_error(const ce_batch* b);

/* ---- serving form -------------------------------------------------------
 * Continuous batching of jobs on one persistent serving kernel. Clients
 * submit jobs from any thread; a server thread admits them in arrival order
 * as soon as an in-flight slot and enough of the HBM budget are free (the
 * job's output, and its inputs when given as host pointers, live in one
 * device arena of hbm_budget bytes), and publishes them to the kernel, which
 * interleaves the tiles of every admitted job. A job's inputs may instead be
 * device pointers the caller keeps resident. Latency is measured from
 * ce_server_submit to the server thread seeing the job's completion word.
 * A session starts at the first submit and ends at ce_server_drain, when
 * the kernel has been idle for session_timeout_s, or when it has taken
 * max_jobs jobs; jobs submitted after that go to a new session, started by
 * the server thread (a job published just as a session ended is published
 * again in the next). While a session lasts the serving kernel occupies the
 * GPU's compute units. The per-item arithmetic is that of the CE_KERNEL_*
 * payloads. GPU only. */
#define CE_JOB_QUEUED 0
#define CE_JOB_ADMITTED 1
#define CE_JOB_DONE 2
#define CE_JOB_FAILED 3
typedef struct ce_server ce_server;
typedef struct {
  uint64_t hbm_budget;      /* bytes of device memory for job buffers (> 0)  */
  uint32_t max_inflight;    /* admitted but unfinished jobs; 0 = 64           */
  uint32_t keep_outputs;    /* 0: a job's memory is freed when it finishes   */
  uint32_t max_jobs;        /* jobs per session; 0 = 65536, at most 2^23-1  */
  uint32_t workgroups_per_cu; /* serving workgroups per CU; 0 = the occupancy
                               * limit minus one, which leaves room for copies
                               * and the caller's own kernels during a session */
  double session_timeout_s; /* the kernel leaves after this long with no new
                             * job; 0 = 300 s                                  */
} ce_server_config;
typedef struct {
  int32_t kernel_id;        /* CE_KERNEL_*                                    */
  uint32_t pad;
  ce_escape_params esc;     /* the parameters of kernel_id are used           */
  ce_blur5_params blur;
  ce_nbody_params nb;
  const void* in0_dev;      /* resident device input, or NULL                 */
  const void* in1_dev;
  const void* in0_host;     /* host input copied into HBM at admission        */
  const void* in1_host;
} ce_job;
typedef struct {
  uint64_t submitted, completed, items;
  double p50_s, p99_s, mean_s, max_s; /* latency, submit -> completion seen   */
  double wall_s;            /* first submit -> last completion               */
  double items_per_s, jobs_per_s;
  uint64_t peak_hbm;        /* largest arena use                             */
  uint64_t max_inflight_seen;
} ce_server_report;
ce_status ce_server_create(const ce_server_config* cfg, void* hip_stream, ce_server** out);
/* When a finished job ran on the GPU, in the GPU's s_memrealtime ticks (the
 * rate is hipDeviceAttributeWallClockRate kHz): the start of its first tile
 * and the end of its last. Ticks of jobs of one session compare directly, so
 * overlapping intervals show jobs sharing the device. CE_E_STATE if the job
 * is not done. */
ce_status ce_server_job_ticks(ce_server* s, uint64_t ticket, uint64_t* first_tile_tick, uint64_t* done_tick);
/* Ends the session (waits up to 30 s) and frees everything. NULL-safe. */
void ce_server_destroy(ce_server* s);
/* CE_E_BUDGET if the job alone needs more than the HBM budget. */
ce_status ce_server_submit(ce_server* s, const ce_job* job, uint64_t* ticket);
ce_status ce_server_poll(ce_server* s, uint64_t ticket, int32_t* state);
ce_status ce_server_wait(ce_server* s, uint64_t ticket, double timeout_s);
/* Device output of a finished job (keep_outputs only); valid until release. */
ce_status ce_server_output(ce_server* s, uint64_t ticket, void** dev_ptr, size_t* bytes);
/* Copies a finished job's output (keep_outputs only) into host memory on the
 * server's copy stream and waits for it; bytes must equal the output size. */
ce_status ce_server_copy_output(ce_server* s, uint64_t ticket, void* host_dst, size_t bytes);
ce_status ce_server_release(ce_server* s, uint64_t ticket);
/* Waits for every submitted job, then ends the session. */
ce_status ce_server_drain(ce_server* s, double timeout_s);
ce_status ce_server_stats(const ce_server* s, ce_server_report* r);
const char* ce_server_error(const ce_server* s);

/* ---- bandwidth reference (not part of the method): copies `bytes` (a
 * multiple of 16; both pointers 16-byte aligned device pointers, or device
 * views of pinned host memory) with one non-temporal 16-byte load and store
 * per thread, on `hip_stream` (NULL = default stream). It is the achievable
 * streaming rate the HBM-bound payloads are compared with. sync != 0 waits.
 * Errors: CE_E_INVALID for a size or alignment that does not fit,
 * CE_E_DEVICE for a launch failure. */
ce_status ce_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream, int sync);

/* ---- plain single-GPU launch (the "native" side of the overhead metric,
 * section 7.3): one grid launch of the same payload over the whole index
 * space with no dispenser, on `hip_stream` (NULL = default stream). Device
 * pointers only; ins[] follows the kernel's input slots. sync != 0 waits for
 * completion. Returns CE_E_DEVICE without a GPU. */
/* As ce_bare_run for payloads with several outputs (outs[] follows the
 * kernel's output slots; n_outs must match their count). */
ce_status ce_bare_run_outs(int kernel_id, const void* params, size_t params_size, const void* const* ins,
                           void* const* outs, uint32_t n_outs, void* hip_stream, int sync);
ce_status ce_bare_run(int kernel_id, const void* params, size_t params_size, const void* const* ins,
                      void* out, void* hip_stream, int sync);

/* ---- scheduler plan helpers (pure host logic, no GPU needed) */
/* Static plan: begin/end granule of each of n devices (section 5.3). */
ce_status ce_sched_static_plan(uint64_t G, uint32_t n, const double* props, const uint32_t* order,
                               uint32_t n_bands, uint64_t* begin, uint64_t* end);
/* HGuided package size for device i given G_r pending granules. */
uint64_t ce_sched_hguided_size(uint64_t G_r, const uint64_t* power, uint32_t n, uint32_t k, uint32_t i,
                               uint64_t min_i);

/* 5x5 Gaussian weights for sigma (normalised in double, rounded to FP32). */
ce_status ce_gauss5_weights(double sigma, float* w25);
/* Tree constants of CE_KERNEL_BINOMIAL for volatility sigma, rate r and
 * maturity T: dt = T/steps, u = exp(sigma*sqrt(dt)), d = 1/u,
 * p = (exp(r*dt) - d)/(u - d), disc = exp(-r*dt); pu = disc*p,
 * pd = disc*(1-p) and factors[j] = u^(2j-steps), j = 0..steps (steps+1
 * floats), each computed in double and rounded once. */
ce_status ce_binomial_table(uint32_t steps, double sigma, double rate, double T, float* factors, float* pu,
                            float* pd);

/* Library version string. */
const char* ce_version(void);

#ifdef __cplusplus
}
#endif
#endif /* COEXEC_H */
