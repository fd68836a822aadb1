// Autotuner for the level map of single-segment nests, and the batch planner that
// consults it.
#pragma once

#include "hp_internal.h"

namespace hp {

constexpr int kBatchWaves = 1;          // waves per task of every batched plan (wave tasks)
constexpr int kBatchGroupWaves = 4;     // wavefronts per workgroup of a persistent launch

// How a tuned plan is built for every nest of one size class (single-segment nests:
// one operator that folds as one reduction, so the block may be reshaped).
//   mode 0: the planner's automatic map;
//   mode 1: the block viewed as (J, K) rows: NONE levels on the grid, J on the grid
//           (gj units) x waves x lane partitions (vj), K on the remaining lanes;
//   mode 2: many outputs per task: the block as one level on pw lanes, the
//           innermost NONE level on 64/pw lane partitions x waves, opt outputs per
//           task (the rest of the outputs on the grid).
struct Recipe {
  int32_t mode;
  int64_t k;
  int32_t vj;
  int32_t gj;
  int32_t pw;
  int32_t opt;
  double us;  // measured time of the winner on the class representative
};

// Default recipe for a batched nest when the cache has none.
Recipe default_recipe(const hp_nest* nest, int nw);

// Size class of a nest: input type, operator signature, output count and block
// length (log2 buckets).
std::string tune_key(const hp_nest* nest);

// Plan one nest of a batch: the tuned map of its class if the cache has one and
// use_tuner is set, else the automatic map; always `nw` waves per workgroup.
hp_status plan_for_batch(const hp_nest* nest, uint32_t flags, bool use_tuner, int nw, Lowered* out);

// Build the nest and map a recipe stands for (false if the recipe does not apply).
// *flat_block receives 0, or the block length when `shaped` is the aligned interior
// of blocks that are not a multiple of the row length (see DevPlan::flat_b).
bool apply_recipe(const hp_nest* nest, const Recipe& r, int nw, hp_nest* shaped, hp_level_map* map,
                  int64_t* flat_block);

}  // namespace hp
