// Autotuner for the level map of single-segment nests, and the batch planner that
// consults it.
#pragma once

#include "hp_internal.h"

namespace hp {

constexpr int kBatchWaves = 4;  // waves per workgroup of every batched plan

// How a tuned plan is built for every nest of one size class.  The reduced block
// of a single-segment nest (one operator that folds as one reduction) is viewed as
// (J, K): K contiguous elements, J = block / K; NONE levels stay on the grid,
// J goes to the grid (g units) x waves (all of them) x lane partitions (vj), K to
// the remaining lanes.  k == 0 means: the planner's automatic map.
struct Recipe {
  int64_t k;
  int32_t vj;
  int32_t gj;
  double us;  // measured time of the winner on the class representative
};

// Size class of a nest: input type, operator signature, output count and block
// length (log2 buckets).
std::string tune_key(const hp_nest* nest);

// Plan one nest of a batch: the tuned map of its class if the cache has one and
// use_tuner is set, else the automatic map; always `nw` waves per workgroup.
hp_status plan_for_batch(const hp_nest* nest, uint32_t flags, bool use_tuner, int nw, Lowered* out);

// Build the nest and map a recipe stands for (false if the recipe does not apply).
bool apply_recipe(const hp_nest* nest, const Recipe& r, int nw, hp_nest* shaped, hp_level_map* map);

}  // namespace hp
