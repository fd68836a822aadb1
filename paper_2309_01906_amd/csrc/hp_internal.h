// Internal structures shared by the planner (host) and the kernels (device).
//
// The planner lowers a nest + level map into a DevPlan: for every loop level the
// number of units it gets on each hardware axis (grid G, workgroup W, wavefront V),
// where those units sit in the workgroup / wave / lane index, its static chunk and
// how many serial strips each unit walks; and the reducing levels grouped into
// "segments" (maximal runs of levels whose operator lets them be combined as one
// reduction: SUM, MIN, MAX; every ARG level is a segment of its own).  The kernel
// then walks the strips of the reducing levels as one flat odometer and combines a
// segment's partials across its lanes, waves and workgroups when its last strip is
// done.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "hp.h"

namespace hp {

constexpr int kMaxDepth = HP_MAX_DEPTH;
constexpr int kWave = 64;
constexpr int kMaxWaves = 16;
constexpr int kSlotBytes = 16;  // one LDS / workspace slot: an int carrier {i64 v; i32 idx} or a float pair

enum OutKind : int32_t { OUT_I32 = HP_I32, OUT_I64 = HP_I64, OUT_F32 = HP_F32, OUT_F64 = HP_F64 };

enum GMode : int32_t {
  GCOMB_NONE = 0,     // no reducing level spans workgroups
  GCOMB_UNIFORM = 1,  // all workgroup-spanning reducing levels are in one segment
  GCOMB_NESTED = 2    // several segments span workgroups (outer ones have one strip)
};

// Division by a plan constant d of a dividend 0 <= n < 2^31 as one 64-bit product
// and a shift: q = (n * m) >> s with s = 31 + ceil(log2 d), m = ceil(2^s / d)
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994: m d = 2^s + e with 0 <= e < d <= 2^(s - 31), so the
// error term n e / (d 2^s) stays below 1/d and never reaches the next integer).
// m = 0 marks a divisor whose dividends may not fit 31 bits: plain division.
struct FastDiv {
  uint32_t m, s;
};

struct DevLevel {
  int64_t e;        // extent
  int64_t stride;   // elements between consecutive iterations
  int64_t span;     // iterations covered by one strip of all units = units * chunk
  int64_t strips;   // ceil(e / span)
  int64_t sstride;  // element offset of one strip = span * stride
  int64_t ostride;  // output-index stride (NONE levels only)
  uint32_t gdiv;    // divisor of this level's digit in the workgroup's G coordinate
  uint32_t gf;      // units on G
  int32_t wf, wsh;  // units on W (power of two) and lowest wave-index bit
  int32_t vf, vsh;  // units on V (power of two) and lowest lane-index bit
  int32_t op;
  int32_t chunk;    // consecutive iterations per unit per strip
  int32_t seg;      // segment index, -1 for NONE levels
  int32_t ragged;   // some unit may see t >= e on some strip
  FastDiv fd_gdiv;  // divisions by gdiv and gf (workgroup digits, always < 2^31)
  FastDiv fd_gf;
  FastDiv fd_span;  // division by span for the strips in bounds (m = 0 when e + span >= 2^31)
  int32_t csh;      // log2(chunk)
  int32_t pad_;
};

struct DevSeg {
  int32_t first, last;   // levels [first, last]
  int32_t op;
  int32_t wlo;           // lowest wave bit of the segment
  uint32_t vmask;        // lane bits of the segment's levels
  uint32_t wmask;        // wave bits of the segment's levels
  uint32_t lds_lanes;    // lane bits that belong to levels outside the segment
  int32_t nwu;           // wave units combined by the segment (2^popcount(wmask))
  uint32_t gunits;       // product of the G units of the segment's levels
  uint32_t ufast;        // lane bits b of vmask whose butterfly step may take a mirror or
                         // permlane-swap partner: every lower lane bit is already reduced
};

struct alignas(16) DevPlan {
  int32_t depth, p, nseg, dtype;
  int32_t out_kind, nw, flags, chunk;
  int64_t n_out;
  int64_t grid;
  int64_t gsplit;       // product of G units over reducing levels
  int64_t none_iters;   // product of strips over NONE levels
  int64_t red_iters;    // product of strips over reducing levels
  int64_t in_elems;
  int32_t gmode;
  int32_t xcd;          // renumber workgroups so each XCD gets a contiguous range
  uint32_t red_vmask, red_wmask;    // lane / wave bits of reducing levels
  uint32_t idle_vmask, idle_wmask;  // lane / wave bits assigned to no level
  int32_t lds_slot_lanes;           // 64 if a segment keeps per-lane LDS slots, else 1
  int32_t gq;                       // innermost segment spanning workgroups (0 if none)
  int32_t vlane32;                  // the lanes of a wave lie within 2^31 bytes of lane 0
  int32_t pad3;
  int64_t ord_block;                // ordered products: elements per output
  int64_t ord_span;                 // ordered products: elements per chunk (gsplit chunks per output)
  // Contiguous blocks at any element offset (a single reduction whose block length
  // is not a multiple of the 16-byte vector): output o's block is the flat_b
  // elements at s = o * flat_b.  The reducing levels of the plan cover its aligned
  // interior, flat_e elements from s + h, h = (-s) mod chunk; the other elements
  // (h before it, flat_b - h - flat_e after it) are spread over the flat_units
  // threads that share the output and added before the combine.  0: off.
  int64_t flat_b;
  int64_t flat_e;
  int64_t flat_units;
  // innermost segment, walked as one batched stream: its levels with more than one
  // strip, outer to inner ("inner dims")
  int32_t a;                        // first level of the innermost segment
  int32_t nid;                      // number of inner dims
  int32_t last_dim_is_last_level;   // the innermost inner dim is level depth-1
  int32_t kernel;                   // hp_kernel variant
  int64_t inner_iters;              // product of strips over the innermost segment
  int64_t outer_iters;              // product of strips over reducing levels before it
  int64_t id_strips[kMaxDepth];
  int64_t id_sstride[kMaxDepth];
  int32_t id_level[kMaxDepth];
  int32_t id_ragged[kMaxDepth];
  DevLevel lv[kMaxDepth];
  DevSeg seg[kMaxDepth];
};

// Host-side result of planning (no device resources).
struct Lowered {
  DevPlan dp;
  hp_plan_info info;
};

// Fill `out` from nest + map; sets the thread-local error text on failure.
// force_nw > 0 (batched plans): the plan must use exactly that many waves per
// workgroup; the automatic map gives them to its wave level.
// flat_block > 0: the nest's reducing levels are the aligned interior of blocks of
// flat_block contiguous elements (see DevPlan::flat_b); the planner and the tuner
// make such views of single-reduction nests whose blocks are not vector multiples.
hp_status lower(const hp_nest* nest, const hp_level_map* map, uint32_t flags, Lowered* out, int force_nw = 0,
                int64_t flat_block = 0);

// Whether a nest may be viewed as flat blocks: one reduction (SUM, MIN or MAX over
// every reducing level) of int32 / float elements whose block is long enough to
// hold an aligned interior; *block receives the block length and *p the number of
// output levels.  vec = elements per 16-byte vector.
bool flat_candidate(const hp_nest* nest, int* p, int64_t* block, int* vec);
// The aligned interior of such a block of b elements: the largest multiple of
// `unit` (a multiple of vec) that fits after the up to vec - 1 elements before the
// block's first aligned vector.
int64_t flat_interior(int64_t b, int vec, int64_t unit);

// Thread-local error text.
hp_status fail(hp_status s, const char* fmt, ...);
void clear_error();

}  // namespace hp
