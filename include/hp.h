/*
 * hp.h -- C ABI of the hierarchical nested-reduction library for MI355X (gfx950).
 *
 * The problem (Kruse, "Generalizing Hierarchical Parallelism", arXiv 2309.01906):
 * a loop nest of arbitrary depth in which every loop level is a parallel level
 * placed explicitly on one level of the hardware hierarchy (section 3.1, the
 * `level` clause, including collapsing several hardware levels into one and
 * splitting one hardware level between nested loops, section 3.8), and in which
 * a reduction is collected at every nesting level: on each level one task gathers
 * its siblings' results through that level's cheapest means of communication
 * (section 2; section 3.7 for shuffles at the warp level and the fallback through
 * memory one level up).
 *
 * Hardware levels ("scopes") of gfx950, outermost first:
 *   G  the grid: workgroups; no barrier across them (sections 1 and 3.2: teams
 *      have no barrier), so each writes a partial to global memory and a second
 *      small kernel folds the partials in index order;
 *   W  the workgroup: its wavefronts; combined through LDS and s_barrier;
 *   V  the wavefront: its 64 lanes; combined with DPP / swizzle / bpermute
 *      cross-lane moves.  V may be split between nested loops (partitions of
 *      lanes, section 3.8);
 *   L  a lane: serial iterations in registers (the private partial of 3.6).
 *
 * All functions return an hp_status, never throw and never exit.  On a non-OK
 * status hp_last_error() returns a thread-local message.
 */
#ifndef HP_H
#define HP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hp_status {
  HP_OK = 0,
  HP_EINVAL = 1,       /* malformed argument (null, extent < 1, misaligned pointer ...) */
  HP_EUNSUPPORTED = 2, /* well-formed but not supported (float MIN/MAX, unsatisfiable map ...) */
  HP_ENOMEM = 3,       /* a device or host allocation failed */
  HP_EDEVICE = 4,      /* a HIP runtime call or kernel launch failed */
  HP_EAGAIN = 5,       /* try again later (queue full) */
  HP_ETOOBIG = 6,      /* request larger than a configured budget */
  HP_ENOTREADY = 7,    /* result not ready yet */
  HP_ECANCELED = 8,    /* request dropped because its batch failed or the server shut down */
  HP_ESTATE = 9        /* call not valid in the object's current state */
} hp_status;

/* Element types.  Inputs are I32, F32 or BF16; outputs are I32, I64, F32 or F64.
 * AFFINE64 and MAT2X2_64 are the elements of ordered products (HP_OP_PROD), both
 * input and output, with arithmetic modulo 2^64:
 *   AFFINE64  : (a, b), two uint64 (16 bytes): the map x -> a x + b;
 *   MAT2X2_64 : a 2x2 matrix of uint64, row-major (32 bytes). */
typedef enum hp_dtype {
  HP_I32 = 0, HP_F32 = 1, HP_BF16 = 2, HP_I64 = 3, HP_F64 = 4, HP_AFFINE64 = 5, HP_MAT2X2_64 = 6
} hp_dtype;

/* Per-level operation.  NONE levels index the output and must form a prefix of
 * the nest.  Float nests support SUM only.  ARGMIN/ARGMAX pass the winning
 * iteration index t (first occurrence on ties) to the enclosing level. */
typedef enum hp_op {
  HP_OP_NONE = 0,
  HP_OP_SUM = 1,
  HP_OP_MIN = 2,
  HP_OP_MAX = 3,
  HP_OP_ARGMIN = 4,
  HP_OP_ARGMAX = 5,
  /* Ordered product of AFFINE64 / MAT2X2_64 elements: associative but not
   * commutative, so siblings are combined strictly in iteration order (the
   * paper notes that OpenMP reductions require commutativity, section 2):
   *   R_m = R_{m+1}(0) * R_{m+1}(1) * ... * R_{m+1}(e_m - 1).
   * Affine: (a1, b1) * (a2, b2) = (a1 a2, a2 b1 + b2), the first map applied
   * first; matrices: the matrix product.  Every reducing level of such a nest
   * is PROD; the planner chooses the map (explicit maps: HP_EUNSUPPORTED); batches
   * and the server do not take these nests. */
  HP_OP_PROD = 6
} hp_op;

/* Scope bits of a level map.  A level may use several adjacent scopes (a
 * collapse, section 3.1); L adds nothing but allows serial strips.
 * HP_SCOPE_X names the chip's 8 XCDs, a hardware level between the grid and the
 * workgroup (section 3.2's levels by property: an XCD shares one L2).  A level on
 * X gets 8 grid units, one per XCD: all workgroups of one unit run on one XCD, as
 * the dispatcher deals workgroups round-robin to the XCDs (which XCD holds unit 0
 * changes from launch to launch; hp_xcd_ids checks the partition on the device).
 * It counts as G for every other rule (X together with W is X+W), only the
 * first level that uses the grid may use it, at most one level does, and the plan
 * needs a grid of at least 16 workgroups that is a multiple of 8 with XCD
 * numbering on (no HP_FLAG_NO_XCD): else HP_EINVAL / HP_EUNSUPPORTED. */
enum { HP_SCOPE_G = 1, HP_SCOPE_W = 2, HP_SCOPE_V = 4, HP_SCOPE_L = 8, HP_SCOPE_X = 16 };
/* Axis index into hp_level_map.units[level][axis]. */
enum { HP_AXIS_G = 0, HP_AXIS_W = 1, HP_AXIS_V = 2 };

#define HP_MAX_DEPTH 8

/* A loop nest over a dense row-major array: level 0 is the outermost loop,
 * extent[depth-1] the contiguous one.  Output = the nested reduction
 *   R_d = A[i0..i_{d-1}],  R_m = OP_m over t < extent[m] of R_{m+1},
 *   out[i0..i_{p-1}] = R_p,  p = number of leading NONE levels,
 * stored row-major over the NONE levels. */
typedef struct hp_nest {
  int32_t depth;                    /* 1..HP_MAX_DEPTH */
  int32_t dtype;                    /* hp_dtype of the input */
  int32_t op[HP_MAX_DEPTH];         /* hp_op per level */
  int64_t extent[HP_MAX_DEPTH];     /* >= 1 per level */
} hp_nest;

/* Placement of each loop level on the hardware hierarchy (section 3.1's level
 * clause).  scopes[m] is a non-empty set of adjacent HP_SCOPE_* bits; the map
 * must be monotone (a level never uses a scope outer to one used by an
 * enclosing level -- the reserve rule of section 3.3).  Consecutive levels may
 * share a scope, which splits it (section 3.8): the outer level takes the high
 * part of the scope's index, the inner level the low part.  units[m][axis] asks
 * for a number of units of that axis for level m (W and V: a power of two;
 * 0: the planner chooses).  Iterations beyond the units are strip-mined
 * (section 3.4, SPMD mode) with a static cyclic schedule (3.5); units beyond the
 * extent are masked (schedule(none), 3.5). */
typedef struct hp_level_map {
  uint32_t scopes[HP_MAX_DEPTH];
  uint32_t units[HP_MAX_DEPTH][3];
} hp_level_map;

/* hp_plan flags */
#define HP_FLAG_OUT_F32 0x1u   /* float sums stored as fp32 (default fp64) */
#define HP_FLAG_SCALAR 0x2u    /* one element per load on the innermost level */
#define HP_FLAG_NO_XCD 0x4u    /* no XCD-contiguous workgroup renumbering */
/* 0x8 is reserved.  Inputs are streamed once, so every load is nontemporal. */
#define HP_FLAG_GENERIC 0x10u  /* always use the general kernel (no lean streaming variant) */

/* What the planner decided; filled by hp_plan_inspect / hp_plan_info. */
typedef struct hp_plan_info {
  int32_t depth;                   /* levels of the planned view: the nest's depth, or fewer when an
                                      automatic float plan runs its reducing levels (all SUM, so each
                                      output's block is contiguous) as one level, which it does when
                                      that view fits the lean kernel and the nested one does not */
  int32_t out_dtype;               /* HP_I32 / HP_I64 / HP_F32 / HP_F64, or the element type of an ordered product */
  int64_t n_out;                   /* number of outputs */
  size_t out_bytes;                /* n_out * size of out_dtype */
  int64_t in_elems;                /* elements of the input */
  size_t in_bytes;
  int64_t grid;                    /* workgroups per launch */
  int32_t waves;                   /* wavefronts per workgroup */
  int32_t chunk;                   /* elements per load on the innermost level */
  int64_t gsplit;                  /* workgroups whose partials form one output (1: no grid combine) */
  size_t workspace_bytes;          /* device workspace owned by the plan */
  size_t lds_bytes;                /* dynamic LDS per workgroup */
  uint32_t scopes[HP_MAX_DEPTH];   /* resolved map */
  uint32_t units[HP_MAX_DEPTH][3];
  int64_t strips[HP_MAX_DEPTH];    /* serial strips per level per unit */
  int32_t nseg;                    /* reducing segments (runs of levels combined as one) */
  int32_t kernel;                  /* hp_kernel: the kernel variant hp_run launches */
  int64_t flat_block;              /* 0, or the block length when the plan's reducing levels are the aligned
                                      interior of each output's contiguous block (a single SUM / MIN / MAX
                                      reduction whose block is not a multiple of the 16-byte vector: the
                                      planner maps the interior with 16-byte loads and spreads the elements
                                      before and after it over the output's threads); depth, scopes, units
                                      and strips then describe the interior view */
} hp_plan_info;

/* Kernel variants (hp_plan_info.kernel).  Every variant runs the same level
 * mapping; they differ in which code paths are compiled in. */
typedef enum hp_kernel {
  HP_KERNEL_LEAN = 0,     /* float, depth <= 4, at most one strided inner dim, <= 8 waves, vector chunk */
  HP_KERNEL_GENERIC4 = 1, /* float, depth <= 4 */
  HP_KERNEL_GENERIC8 = 2, /* float, depth <= 8 */
  HP_KERNEL_INT_FLAT = 3, /* int32, depth <= 4, one reducing segment */
  HP_KERNEL_INT_SEG = 4,  /* int32, depth <= 4, up to three segments */
  HP_KERNEL_INT_DEEP = 5, /* int32, anything else */
  HP_KERNEL_ORDERED = 6,  /* ordered products of AFFINE64 / MAT2X2_64 elements */
  HP_KERNEL_INT_CHAIN = 7 /* int32, two or three reducing levels with one operator each, every level
                             divided evenly by its units, innermost levels on lanes (the chain kernel) */
} hp_kernel;

typedef struct hp_plan_s* hp_plan_t;

/* Validate a nest and a level map (NULL: the planner chooses one) and lower it
 * to launch geometry, without touching any device.  Host-only: usable on a
 * machine without a GPU.  Returns HP_EINVAL for malformed nests or maps
 * (depth out of range, extent < 1, NONE after a reducing level, bad scope
 * sets, non-monotone maps, units that are not powers of two or exceed 16
 * waves / 64 lanes) and HP_EUNSUPPORTED for well-formed requests the library
 * does not implement (non-SUM ops on float inputs, ARG levels longer than
 * 2^31-1, grids beyond the launch limits). */
hp_status hp_plan_inspect(const hp_nest* nest, const hp_level_map* map, uint32_t flags,
                          hp_plan_info* info);

/* hp_plan_inspect, then allocate the plan's device workspace (zeroed) on the
 * current HIP device.  The plan owns the workspace until hp_destroy. */
hp_status hp_plan(const hp_nest* nest, const hp_level_map* map, uint32_t flags, hp_plan_t* out);

/* The planner's decisions for an existing plan. */
hp_status hp_plan_info_get(hp_plan_t plan, hp_plan_info* info);

/* Run the nest: d_in is a device pointer to the row-major input (16-byte
 * aligned, in_bytes long), d_out a device pointer to n_out outputs of
 * out_dtype (aligned to the output element: 4 or 8 bytes, 16 for ordered
 * products).  stream is a hipStream_t (NULL: the null stream).  Asynchronous:
 * allocates nothing and does not synchronise, so it may be captured in a
 * hipGraph.  A grid-split plan (gsplit > 1) launches a second, small kernel that
 * folds the workgroups' partials in a fixed order.  A plan must not run on two
 * streams at once (its workspace is shared); consecutive runs on one stream are
 * fine.
 * Errors: HP_EINVAL (null plan or pointer, misalignment), HP_EDEVICE
 * (launch failure). */
hp_status hp_run(hp_plan_t plan, const void* d_in, void* d_out, void* stream);

/* Free the plan and its workspace.  NULL is a no-op.  The caller must make
 * sure no launch using the plan is still running. */
hp_status hp_destroy(hp_plan_t plan);

/* For callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, hosts that forbid hipMalloc): hp_plan followed by hp_run
 * and hp_destroy in one call that allocates nothing.  The nest is planned on the
 * host exactly as hp_plan would plan it (same kernels, same bits as hp_run); the
 * plan, the fold tasks and the workgroup partials of a grid-split nest go into a
 * file-scope device array of HP_STATIC_SCRATCH_BYTES bytes that each GPU the
 * library runs on holds until the process ends.  The plan reaches that array
 * through a small install kernel on `stream`, then the nest kernels run there.
 * d_in, d_out and stream are as for hp_run; the call is asynchronous.
 * Every call on one GPU shares that GPU's array: calls on one stream are ordered,
 * but calls that overlap on one GPU (two streams, two threads) race and may give
 * wrong results.  Nothing in the array needs clearing: every run writes what it
 * reads.
 * Errors: as hp_plan_inspect for the nest and map; HP_EINVAL for null or
 * misaligned pointers; HP_ETOOBIG when the nest needs more workspace or fold
 * tasks than the array holds (about 7 MiB of partials, 65536 fold tasks);
 * HP_EDEVICE for launch failures. */
#define HP_STATIC_SCRATCH_BYTES (8u << 20)
hp_status hp_reduce_static(const hp_nest* nest, const hp_level_map* map, uint32_t flags, const void* d_in,
                           void* d_out, void* stream);

/* ---------------------------------------------------------------------------
 * Batches: many nests of uneven sizes in one persistent launch per kernel family.
 * Nests are planned as one-wavefront plans, and every wavefront of the persistent
 * workgroups is an independent worker: it starts on tasks dealt to it statically
 * and then takes (nest, workgroup) tasks from an atomic counter -- a dynamic
 * schedule on the grid level (section 3.5).  Tasks go largest first, each to the
 * least-loaded of 64 queues, 8 per XCD.  Grid-split nests are folded by a second
 * kernel after the persistent one, which also resets the task counters for the
 * next run.  Every nest keeps the plan it would get alone (its own shape and the
 * tuner cache decide it, never the batch), so its result is the same bits as a
 * single run of that plan.  Ordered products (HP_OP_PROD) are not batched.
 */
typedef struct hp_batch_s* hp_batch_t;

#define HP_BATCH_GRAPH 0x100u   /* hp_batch_run replays a captured hipGraph */
#define HP_BATCH_NO_TUNE 0x200u /* ignore the tuner cache: automatic maps only */

/* Plan n nests (each validated as by hp_plan_inspect; batched plans use one
 * wavefront per workgroup task) and allocate the batch's device tables, task
 * lists, counters and grid-combine workspaces.  flags: HP_BATCH_GRAPH, HP_BATCH_NO_TUNE,
 * HP_FLAG_OUT_F32.  HP_EINVAL / HP_EUNSUPPORTED name the first
 * bad nest; HP_ENOMEM if device memory runs out. */
hp_status hp_batch_plan(const hp_nest* nests, int64_t n, uint32_t flags, hp_batch_t* out);

/* Host-only: the plans hp_batch_plan would make (current tuner cache included),
 * written to infos[0..n).  No device is touched. */
hp_status hp_batch_plan_inspect(const hp_nest* nests, int64_t n, uint32_t flags, hp_plan_info* infos);

/* Planner decisions for nest i of the batch. */
hp_status hp_batch_info(hp_batch_t b, int64_t i, hp_plan_info* info);

/* Launch count (persistent kernels per run), total tasks, wavefront workers of the
 * persistent launches, and the algorithmic bytes (inputs + outputs) of one run.
 * Any output pointer may be NULL. */
hp_status hp_batch_stats(hp_batch_t b, int64_t* n_launches, int64_t* n_tasks, int64_t* n_workers, double* bytes);

/* Point the batch at its data: host arrays of n device pointers (inputs 16-byte
 * aligned, outputs aligned for their type).  Copied into the batch's device
 * table (synchronous); a captured graph stays valid across calls. */
hp_status hp_batch_set_io(hp_batch_t b, const void* const* d_in, void* const* d_out);

/* Run all nests: one persistent launch per kernel family (or one graph launch
 * with HP_BATCH_GRAPH, captured at the first call).  Asynchronous on `stream`;
 * must not overlap another run of the same batch.  HP_ESTATE before set_io. */
hp_status hp_batch_run(hp_batch_t b, void* stream);

/* Baseline: the same plans, one launch per nest (use_graph: all of those launches
 * captured once in one graph and replayed). */
hp_status hp_batch_run_each(hp_batch_t b, void* stream, int32_t use_graph);

/* Free the batch (the caller makes sure no run is in flight).  NULL is a no-op. */
hp_status hp_batch_destroy(hp_batch_t b);

/* ---------------------------------------------------------------------------
 * Autotuner (section 3.9's choice between kernel versions, made by measurement):
 * for a nest whose reducing levels fold as one reduction (SUM, MIN or MAX), time
 * candidate level maps of its size class on the current device -- the block seen
 * as (J, K) rows split between grid, waves and lane partitions, or many outputs
 * per task on lane partitions -- and store the fastest in the process-wide cache
 * that batched plans consult.  A candidate is timed as a persistent batch of
 * replicas of the nest (its throughput when it shares the device), median of
 * `reps` runs, per nest.  best_us / auto_us (may be NULL) receive the winner's
 * time and the automatic map's.  The cache is also read once from the file named
 * by the HP_TUNE_CACHE environment variable. */
hp_status hp_tune_nest(const hp_nest* nest, uint32_t flags, int32_t reps, double* best_us, double* auto_us);
hp_status hp_tune_cache_load(const char* path);
hp_status hp_tune_cache_save(const char* path);
hp_status hp_tune_cache_clear(void);
hp_status hp_tune_cache_size(int64_t* n);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of nest-reduction requests (not in the paper: the
 * serving form of the batched kernel).  Requests arrive at any time; a scheduler
 * thread admits them in arrival order while their bytes (input + output + grid
 * workspace) fit the HBM budget -- a request that does not fit may be passed by
 * later ones at most 64 times -- and launches a batch as soon as one of `streams`
 * slots is free and either max_batch requests wait, the oldest has waited
 * window_us, or the device is idle.  Batches of different slots overlap on the
 * device.  Request state (plans, task lists, fold tasks, partials) lives in the
 * slot's device arena; a request joins a batch only while its share of that arena
 * still fits (else it waits for the next batch, under the same bounded bypass), so
 * no request fails because of what it was packed with.  If a launch fails after
 * some of its work was enqueued, the slot stays busy until its stream has drained,
 * and only then are its requests failed (HP_EDEVICE).  Each request keeps the plan it would get alone, so its
 * result does not depend on the batch it ran in.  Payloads are not copied: d_in
 * and d_out must stay valid until the request completes.
 */
typedef struct hp_server_s* hp_server_t;

#define HP_SERVER_FAKE_DEVICE 0x1000u /* host-only executor for scheduler tests: no GPU work */

typedef struct hp_server_cfg {
  size_t hbm_budget;              /* bytes admitted at once */
  size_t slot_bytes;              /* device arena per slot (descriptors + workspaces of one batch) */
  int32_t streams;                /* slots = batches in flight, 1..16 */
  int32_t max_batch;              /* requests per batch */
  int32_t window_us;              /* how long a partial batch may wait while the device is busy */
  int32_t queue_cap;              /* pending requests before hp_submit returns HP_EAGAIN */
  uint32_t flags;                 /* HP_FLAG_OUT_F32, HP_SERVER_FAKE_DEVICE */
  int32_t fail_every_nth_batch;   /* test hook: every n-th batch fails (0: never) ... */
  int32_t fail_step;              /* ... before its device step fail_step: 0 the descriptor upload, then one
                                     step per persistent launch and the fold launch (clamped to the last) */
} hp_server_cfg;

typedef struct hp_req_info {
  int32_t status;      /* HP_ENOTREADY while pending / in flight, then HP_OK or the failure */
  int32_t pad;
  double t_arrival_us; /* server clock (hp_server_now_us) */
  double t_admit_us;
  double t_launch_us;
  double t_done_us;    /* when the scheduler saw the batch complete */
  int64_t bytes;       /* algorithmic bytes: input + output */
  int64_t batch_id;
} hp_req_info;

typedef struct hp_server_stats {
  int64_t submitted, completed, failed, batches, pending, max_queue;
  int64_t max_in_use_bytes, in_use_bytes;
  double bytes;                          /* input + output bytes of completed requests */
  double p50_us, p99_us, p999_us, max_us, mean_us; /* arrival -> completion latency */
  double gbps;                           /* bytes / (last completion - first arrival) */
} hp_server_stats;

/* Start a server on the current device (allocates its slots' streams, events,
 * device arenas and pinned staging).  HP_EINVAL for a bad configuration. */
hp_status hp_server_create(const hp_server_cfg* cfg, hp_server_t* out);

/* Submit one request; t_arrival_us < 0 stamps the current server time (an
 * open-loop client passes its scheduled arrival time instead).  The nest is
 * planned here (errors as hp_plan_inspect).  HP_ETOOBIG if it alone exceeds the
 * budget or its descriptors and workspace alone exceed slot_bytes, HP_EAGAIN if the
 * queue is full, HP_ESTATE after shutdown began. */
hp_status hp_submit(hp_server_t s, const hp_nest* nest, const void* d_in, void* d_out, double t_arrival_us,
                    uint64_t* ticket);

/* HP_ENOTREADY until the request completed; then HP_OK with info filled (its
 * status field holds the request's own outcome). */
hp_status hp_poll(hp_server_t s, uint64_t ticket, hp_req_info* info);

/* Block until the request completed. */
hp_status hp_wait(hp_server_t s, uint64_t ticket, hp_req_info* info);

/* Drop a completed request's record. */
hp_status hp_server_forget(hp_server_t s, uint64_t ticket);

/* Counters and latency percentiles of the completed requests. */
hp_status hp_server_get_stats(hp_server_t s, hp_server_stats* st);

/* Current server clock in microseconds. */
hp_status hp_server_now_us(hp_server_t s, double* t);

/* Open-loop client: submit request i at server time t_arrival_us[i] (ascending),
 * without waiting for completions; tickets[i] receives its ticket. */
hp_status hp_server_replay(hp_server_t s, int64_t n, const hp_nest* nests, const void* const* d_in,
                           void* const* d_out, const double* t_arrival_us, uint64_t* tickets);

/* Drain: finish every admitted and pending request, stop the scheduler, free the
 * slots.  NULL is a no-op. */
hp_status hp_server_destroy(hp_server_t s);

/* ---------------------------------------------------------------------------
 * Stencils (the paper's second class of multi-level algorithms, section 2: a
 * region whose input fits a level's local memory, repeated on every level with
 * local memory; section 4: array sections that overlap by a ghost surface).
 * `steps` five-point Jacobi sweeps of a rows x cols row-major float array,
 *   B[i][j] = c0 A[i][j] + c1 ((A[i-1][j] + A[i+1][j]) + (A[i][j-1] + A[i][j+1]))
 * for 1 <= i <= rows-2, 1 <= j <= cols-2 (fp32, in exactly this order, no fused
 * multiply-add); boundary cells keep their values.  Levels: each workgroup (8
 * threads per tile row) reads a tile_rows x 64 output tile plus a ghost surface T
 * cells wide into LDS once, runs T sweeps there and writes the tile once; each lane
 * updates column strips of 4 cells from registers; the tiles are dealt to the XCDs in bands, so ghost cells
 * that neighbouring tiles share come from HBM once into the XCD's L2.  More sweeps
 * than one launch holds (8) run as ceil(steps / T) launches, alternating between
 * d_out and a rows x cols buffer the plan allocates, so that the last writes d_out.
 * hp_stencil_plan: rows, cols >= 1, steps >= 1 (HP_EINVAL); at most 8 sweeps per
 *   launch, spread evenly over the launches; 64-row tiles from 6 sweeps per launch
 *   when they fit the workgroup level's local memory and the array gives the fill
 *   target of workgroups (both from hp_level_table), else 32-row tiles.
 * hp_stencil_plan_ex: the same with tile_rows (0: choose, 32 or 64), sweeps per
 *   launch (0: choose, 1..8) and flags (HP_STENCIL_NO_XCD: tile b on workgroup b);
 *   HP_EINVAL for other values, HP_EUNSUPPORTED when the tile does not fit LDS or
 *   the array needs more tiles than one launch holds.  The plan remembers the
 *   current device when it allocates its buffer; run it there (HP_EINVAL).
 * hp_stencil_info: the tile rows and columns, sweeps per launch and launches.
 * hp_stencil_run: d_in and d_out are caller-owned device arrays of rows*cols
 *   floats, 4-byte aligned, not overlapping (HP_EINVAL); asynchronous on `stream`.
 *   Calls that share a plan of several launches must not overlap (they share its
 *   buffer).
 * hp_stencil_destroy frees the plan and its buffer (call it once the plan's last
 *   run has finished); NULL is a no-op.
 */
enum { HP_STENCIL_NO_XCD = 1 };
typedef struct hp_stencil_s* hp_stencil_t;
hp_status hp_stencil_plan(int64_t rows, int64_t cols, int32_t steps, float c0, float c1, hp_stencil_t* out);
hp_status hp_stencil_plan_ex(int64_t rows, int64_t cols, int32_t steps, float c0, float c1, int32_t tile_rows,
                             int32_t sweeps_per_launch, uint32_t flags, hp_stencil_t* out);
hp_status hp_stencil_info(hp_stencil_t s, int32_t* tile_rows, int32_t* tile_cols, int32_t* sweeps_per_launch,
                          int32_t* launches);
hp_status hp_stencil_run(hp_stencil_t s, const float* d_in, float* d_out, void* stream);
hp_status hp_stencil_destroy(hp_stencil_t s);

/* ---------------------------------------------------------------------------
 * Calibration (not part of the method): a plain streaming read of `bytes` bytes
 * at d_in -- 16-byte nontemporal loads, four in flight per thread, each workgroup
 * reading 16 KiB blocks block-cyclically, added up -- on `grid` workgroups of 256
 * threads.  It writes one float per workgroup to d_out
 * (grid floats, caller-owned), only to keep the loads.  Its bandwidth is the read
 * ceiling the reduction kernels are compared with.  d_in and bytes must be
 * multiples of 16; asynchronous on `stream`. */
hp_status hp_stream_read(const void* d_in, size_t bytes, float* d_out, int32_t grid, void* stream);

/* The device's hardware levels and their properties -- the build's analogue of
 * the paper's Table 2 (section 3.2 selects levels by property).  The automatic
 * map reads it: a reduction on a level needs a way to combine its units' values,
 * so reducing levels go first to the level with HP_LP_SHUFFLE (the wavefront's
 * lanes), then to the level with HP_LP_BARRIER and HP_LP_LOCALMEM (a workgroup's
 * waves, through LDS), and last to the grid, which has neither (a second kernel
 * folds its partials); the unit counts bound the lanes and waves it hands out;
 * `fill_workgroups` sets the grid split: a nest with fewer outputs than half of it
 * also splits its outermost reducing level over workgroups, to about twice that
 * many workgroups for float inputs and that many for int32.  HP_LP_SHARED_CACHE (an XCD's L2) pays only when
 * several workgroups read the same data; a nested reduction reads every element
 * once, so the automatic map never places a level on X (explicit maps may).
 * hp_level_table copies the rows, outermost first (G, X, W, V, L), into out
 * (cap rows at most) and sets *n to the number of rows and *fill_workgroups.
 * Host only.  Errors: HP_EINVAL for null pointers or cap < 1. */
#define HP_LP_BARRIER 0x1u      /* the level's units can wait for each other */
#define HP_LP_SHUFFLE 0x2u      /* they exchange registers directly (DPP, permlane, bpermute) */
#define HP_LP_LOCALMEM 0x4u     /* they share an addressable scratch memory (LDS) */
#define HP_LP_ATOMIC 0x8u       /* they have atomics on memory they share */
#define HP_LP_DYNAMIC 0x10u     /* work can be handed to them dynamically (a counter) */
#define HP_LP_LOCKSTEP 0x20u    /* they run in lockstep */
#define HP_LP_SHARED_CACHE 0x40u /* they share a cache that is not addressable */
typedef struct hp_level_props {
  uint32_t scope;       /* HP_SCOPE_* bit of the level */
  int32_t units;        /* units inside one unit of the next level out; 0: as many as the work needs */
  uint32_t props;       /* HP_LP_* bits */
  int64_t shared_bytes; /* memory the units share: LDS per workgroup, L2 per XCD; 0: none */
} hp_level_props;
hp_status hp_level_table(hp_level_props* out, int32_t cap, int32_t* n, int64_t* fill_workgroups);

/* Diagnostic of the XCD scope: launches `grid` workgroups of `threads` threads
 * (a multiple of 64, at most 1024) with `lds_bytes` of dynamic LDS (at most
 * 64 KiB), and thread 0 of workgroup b writes to d_out[b] the XCD it runs on, as
 * the hardware reports it (register XCC_ID).  The XCD-aware numbering assumes the
 * dispatcher deals workgroups round-robin to the XCDs, so that workgroups b and b'
 * share an XCD exactly when b = b' mod 8 (which XCD takes workgroup 0 depends on
 * where the previous launch stopped); this checks it for a launch shape.
 * d_out: device array of `grid` int32.  Errors: HP_EINVAL for bad arguments,
 * HP_EDEVICE for a launch failure. */
hp_status hp_xcd_ids(int32_t* d_out, int32_t grid, int32_t threads, size_t lds_bytes, void* stream);

/* Thread-local text for the last non-OK status returned on this thread. */
const char* hp_last_error(void);

/* Name of a status code. */
const char* hp_status_str(hp_status s);

#ifdef __cplusplus
}
#endif
#endif /* HP_H */
