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
 *   G  the grid: workgroups; no barrier across them, combined through global
 *      memory with an atomic ticket (sections 1 and 3.2: teams have no barrier);
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

/* Element types.  Inputs are I32, F32 or BF16; outputs are I32, I64, F32 or F64. */
typedef enum hp_dtype { HP_I32 = 0, HP_F32 = 1, HP_BF16 = 2, HP_I64 = 3, HP_F64 = 4 } hp_dtype;

/* Per-level operation.  NONE levels index the output and must form a prefix of
 * the nest.  Float nests support SUM only.  ARGMIN/ARGMAX pass the winning
 * iteration index t (first occurrence on ties) to the enclosing level. */
typedef enum hp_op {
  HP_OP_NONE = 0,
  HP_OP_SUM = 1,
  HP_OP_MIN = 2,
  HP_OP_MAX = 3,
  HP_OP_ARGMIN = 4,
  HP_OP_ARGMAX = 5
} hp_op;

/* Scope bits of a level map.  A level may use several adjacent scopes (a
 * collapse, section 3.1); L adds nothing but allows serial strips. */
enum { HP_SCOPE_G = 1, HP_SCOPE_W = 2, HP_SCOPE_V = 4, HP_SCOPE_L = 8 };
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
#define HP_FLAG_TEMPORAL 0x8u  /* plain (cached) loads instead of nontemporal ones */

/* What the planner decided; filled by hp_plan_inspect / hp_plan_info. */
typedef struct hp_plan_info {
  int32_t depth;
  int32_t out_dtype;               /* HP_I32 / HP_I64 / HP_F32 / HP_F64 */
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
} hp_plan_info;

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
 * out_dtype (8-byte aligned).  stream is a hipStream_t (NULL: the null
 * stream).  Asynchronous: allocates nothing and does not synchronise, so it
 * may be captured in a hipGraph.  A plan must not run on two streams at once
 * (its workspace is shared); consecutive runs on one stream are fine.
 * Errors: HP_EINVAL (null plan or pointer, misalignment), HP_EDEVICE
 * (launch failure). */
hp_status hp_run(hp_plan_t plan, const void* d_in, void* d_out, void* stream);

/* Free the plan and its workspace.  NULL is a no-op.  The caller must make
 * sure no launch using the plan is still running. */
hp_status hp_destroy(hp_plan_t plan);

/* Thread-local text for the last non-OK status returned on this thread. */
const char* hp_last_error(void);

/* Name of a status code. */
const char* hp_status_str(hp_status s);

#ifdef __cplusplus
}
#endif
#endif /* HP_H */
