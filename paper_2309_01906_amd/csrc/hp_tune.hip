// Autotuner: picks, per size class, how the reduced block of a single-segment nest
// is split between the grid, the waves and the lanes (and how it is viewed as
// (J, K) rows), by timing candidate plans on the device.  The paper's section 3.9
// selects kernel versions per hardware; here the versions are level maps of one
// kernel, chosen by measurement on the gfx950 at hand and kept in a cache file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hp_internal.h"
#include "hp_batch_dev.h"
#include "hp_tune.h"

struct hp_batch_s;
namespace hp {
hp_status batch_from_plans(const std::vector<Lowered>& plans, uint32_t flags, hp_batch_s** out);
}

namespace {

std::mutex g_mu;
std::map<std::string, hp::Recipe> g_cache;
bool g_env_loaded = false;

int lb(int64_t x) {
  int r = 0;
  while ((int64_t(1) << (r + 1)) <= x) ++r;
  return r;
}

int elem_bytes(int dt) { return dt == HP_BF16 ? 2 : 4; }

// one segment of SUM, MIN or MAX: the block is one flat reduction and may be reshaped
bool single_segment(const hp_nest* n, int* p_out, int64_t* block) {
  int p = n->depth;
  for (int l = 0; l < n->depth; ++l)
    if (n->op[l] != HP_OP_NONE) {
      p = l;
      break;
    }
  if (p == n->depth) return false;
  const int op = n->op[p];
  if (op == HP_OP_ARGMIN || op == HP_OP_ARGMAX) return false;
  int64_t b = 1;
  for (int l = p; l < n->depth; ++l) {
    if (n->op[l] != op) return false;
    b *= n->extent[l];
  }
  *p_out = p;
  *block = b;
  return true;
}

hp_status load_file_locked(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return hp::fail(HP_EINVAL, "cannot open tuner cache %s", path);
  char key[256];
  long long k;
  int mode, vj, gj, pw, opt;
  double us;
  while (fscanf(f, "%255s %d %lld %d %d %d %d %lf", key, &mode, &k, &vj, &gj, &pw, &opt, &us) == 8)
    g_cache[key] = hp::Recipe{mode, k, vj, gj, pw, opt, us};
  fclose(f);
  return HP_OK;
}

void load_env_locked() {
  if (g_env_loaded) return;
  g_env_loaded = true;
  const char* p = getenv("HP_TUNE_CACHE");
  if (p && *p) (void)load_file_locked(p);
}

}  // namespace

namespace hp {

std::string tune_key(const hp_nest* n) {
  int p = 0;
  int64_t block = 1, outs = 1;
  char ops[HP_MAX_DEPTH + 1] = {0};
  for (int l = 0; l < n->depth; ++l) {
    ops[l] = "NSmMaA"[n->op[l] < 6 && n->op[l] >= 0 ? n->op[l] : 0];
    if (n->op[l] == HP_OP_NONE) {
      outs *= n->extent[l];
      ++p;
    } else {
      block *= n->extent[l];
    }
  }
  char buf[96];
  snprintf(buf, sizeof buf, "gfx950:%d:%s:o%d:b%d", n->dtype, ops, lb(outs), lb(block));
  return buf;
}

bool apply_recipe(const hp_nest* n, const Recipe& r, int nw, hp_nest* shaped, hp_level_map* map,
                  int64_t* flat_block) {
  int p;
  int64_t block;
  *flat_block = 0;
  if (r.mode == 0 || !single_segment(n, &p, &block)) return false;
  const int op = n->op[p];
  const int c = 16 / elem_bytes(n->dtype);
  memset(shaped, 0, sizeof *shaped);
  memset(map, 0, sizeof *map);
  shaped->dtype = n->dtype;
  for (int l = 0; l < p; ++l) {
    shaped->extent[l] = n->extent[l];
    shaped->op[l] = HP_OP_NONE;
    map->scopes[l] = HP_SCOPE_G;
  }
  if (r.mode == 1) {
    if (r.k <= 0 || p + 2 > HP_MAX_DEPTH) return false;
    if (r.vj < 1 || r.vj > 64 || (r.vj & (r.vj - 1)) || r.gj < 1) return false;
    // rows of k elements; a block that is not a whole number of rows keeps its
    // aligned interior of whole rows and spreads the rest over its threads
    int64_t rows = block / r.k;
    if (block % r.k != 0) {
      if (r.k % c != 0) return false;
      rows = flat_interior(block, c, r.k) / r.k;
      if (rows < 1) return false;
      *flat_block = block;
    }
    shaped->extent[p] = rows;
    shaped->op[p] = op;
    shaped->extent[p + 1] = r.k;
    shaped->op[p + 1] = op;
    shaped->depth = p + 2;
    uint32_t sj = HP_SCOPE_W;
    if (r.gj > 1) sj |= HP_SCOPE_G;
    if (r.vj > 1) sj |= HP_SCOPE_V;
    map->scopes[p] = sj;
    map->units[p][HP_AXIS_W] = (uint32_t)nw;
    if (r.gj > 1) map->units[p][HP_AXIS_G] = (uint32_t)r.gj;
    if (r.vj > 1) map->units[p][HP_AXIS_V] = (uint32_t)r.vj;
    map->scopes[p + 1] = HP_SCOPE_V;
    map->units[p + 1][HP_AXIS_V] = (uint32_t)(64 / r.vj);
    return true;
  }
  if (r.mode == 2) {
    if (p < 1 || r.pw < 1 || r.pw > 64 || (r.pw & (r.pw - 1)) || r.opt < 1) return false;
    const int64_t eo = n->extent[p - 1];
    shaped->extent[p] = block;
    if (block % c != 0 && flat_interior(block, c, c) >= c) {  // vector loads on the aligned interior
      shaped->extent[p] = flat_interior(block, c, c);
      *flat_block = block;
    }
    shaped->op[p] = op;
    shaped->depth = p + 1;
    const int64_t parts = 64 / r.pw;
    int64_t g = (eo + r.opt - 1) / r.opt;
    if (g < 1) g = 1;
    map->scopes[p - 1] = HP_SCOPE_G | HP_SCOPE_W | (parts > 1 ? HP_SCOPE_V : 0u);
    map->units[p - 1][HP_AXIS_G] = (uint32_t)g;
    map->units[p - 1][HP_AXIS_W] = (uint32_t)nw;
    if (parts > 1) map->units[p - 1][HP_AXIS_V] = (uint32_t)parts;
    map->scopes[p] = HP_SCOPE_V;
    map->units[p][HP_AXIS_V] = (uint32_t)r.pw;
    return true;
  }
  return false;
}

Recipe default_recipe(const hp_nest* n, int nw) {
  Recipe r{0, 0, 1, 1, 64, 1, 0.0};
  int p;
  int64_t block;
  if (!single_segment(n, &p, &block) || p < 1) return r;
  const int es = elem_bytes(n->dtype);
  const int64_t bytes = block * es;
  if (bytes >= (16 << 10)) return r;  // large blocks: the automatic map splits them
  // a block that is not a vector multiple is mapped as its aligned interior (vector
  // loads) plus a few elements spread over its lanes
  const int c = (block % (16 / es) == 0 || flat_interior(block, 16 / es, 16 / es) >= 16 / es) ? 16 / es : 1;
  int64_t lanes = (block + c - 1) / c;
  int pw = 1;
  while (pw < lanes && pw < 64) pw *= 2;
  const int64_t per_pass = (64 / pw) * (int64_t)nw;
  int64_t opt = ((32 << 10) / (bytes > 0 ? bytes : 1)) / per_pass * per_pass;
  if (opt < per_pass) opt = per_pass;
  const int64_t eo = n->extent[p - 1];
  if (opt > eo) opt = (eo + per_pass - 1) / per_pass * per_pass;
  r.mode = 2;
  r.pw = pw;
  r.opt = (int32_t)(opt > 0x7FFFFFFF ? 0x7FFFFFFF : opt);
  return r;
}

hp_status plan_for_batch(const hp_nest* nest, uint32_t flags, bool use_tuner, int nw, Lowered* out) {
  if (!nest) return fail(HP_EINVAL, "null nest");
  Recipe r = default_recipe(nest, nw);
  if (use_tuner) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    auto it = g_cache.find(tune_key(nest));
    if (it != g_cache.end()) r = it->second;
  }
  hp_nest shaped;
  hp_level_map m;
  int64_t fb = 0;
  if (apply_recipe(nest, r, nw, &shaped, &m, &fb) && lower(&shaped, &m, flags, out, nw, fb) == HP_OK) return HP_OK;
  return lower(nest, nullptr, flags, out, nw);
}

}  // namespace hp

// ---------------------------------------------------------------------------
// C API

extern "C" hp_status hp_tune_cache_load(const char* path) {
  if (!path) return hp::fail(HP_EINVAL, "null path");
  std::lock_guard<std::mutex> lk(g_mu);
  g_env_loaded = true;
  return load_file_locked(path);
}

extern "C" hp_status hp_tune_cache_save(const char* path) {
  if (!path) return hp::fail(HP_EINVAL, "null path");
  std::lock_guard<std::mutex> lk(g_mu);
  FILE* f = fopen(path, "w");
  if (!f) return hp::fail(HP_EINVAL, "cannot write %s", path);
  for (const auto& kv : g_cache)
    fprintf(f, "%s %d %lld %d %d %d %d %.3f\n", kv.first.c_str(), kv.second.mode, (long long)kv.second.k,
            kv.second.vj, kv.second.gj, kv.second.pw, kv.second.opt, kv.second.us);
  fclose(f);
  return HP_OK;
}

extern "C" hp_status hp_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
  g_env_loaded = true;
  return HP_OK;
}

extern "C" hp_status hp_tune_cache_size(int64_t* n) {
  if (!n) return hp::fail(HP_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g_mu);
  *n = (int64_t)g_cache.size();
  return HP_OK;
}

namespace {

struct Timed {
  hp::Recipe r;
  double us;
};

// Throughput of a candidate inside a batch: R replicas of the plan (distinct input
// and output slots) as one persistent launch; returns the median time per nest.
// This is the figure that matters when the nest shares the device with others.
hp_status time_candidate_batch(const hp::Lowered& L, int R, unsigned char* in, size_t in_stride, unsigned char* out,
                               size_t out_stride, int reps, hipStream_t st, double* us) {
  std::vector<hp::Lowered> plans((size_t)R, L);
  hp_batch_s* b = nullptr;
  hp_status s = hp::batch_from_plans(plans, 0, &b);
  if (s != HP_OK) return s;
  std::vector<const void*> ins((size_t)R);
  std::vector<void*> outs((size_t)R);
  for (int i = 0; i < R; ++i) {
    ins[(size_t)i] = in + (size_t)i * in_stride;
    outs[(size_t)i] = out + (size_t)i * out_stride;
  }
  s = hp_batch_set_io(b, ins.data(), outs.data());
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  std::vector<float> t;
  for (int r = 0; r < reps + 2 && s == HP_OK; ++r) {
    (void)hipEventRecord(e0, st);
    s = hp_batch_run(b, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) s = hp::fail(HP_EDEVICE, "tuner batch run failed");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (r >= 2) t.push_back(ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hp_batch_destroy(b);
  if (s != HP_OK) return s;
  std::sort(t.begin(), t.end());
  *us = t.empty() ? 0.0 : 1e3 * (double)t[t.size() / 2] / (double)R;
  return HP_OK;
}

}  // namespace

extern "C" hp_status hp_tune_nest(const hp_nest* nest, uint32_t flags, int32_t reps, double* best_us,
                                  double* auto_us) {
  using namespace hp;
  if (!nest || reps < 1) return fail(HP_EINVAL, "bad argument");
  int p;
  int64_t block;
  Lowered L0;
  hp_status s = plan_for_batch(nest, flags, false, kBatchWaves, &L0);
  if (s != HP_OK) return s;
  const bool tunable = single_segment(nest, &p, &block);
  // device buffers for R replicas of the nest (values do not change the kernels' timing)
  const size_t in_stride = (L0.info.in_bytes + 255) / 256 * 256;
  const size_t out_stride = (L0.info.out_bytes + 255) / 256 * 256;
  int R = (int)((size_t)(64 << 20) / in_stride);
  if (R < 1) R = 1;
  if (R > 2048) R = 2048;
  unsigned char* in = nullptr;
  unsigned char* out = nullptr;
  if (hipMalloc((void**)&in, in_stride * (size_t)R) != hipSuccess) return fail(HP_ENOMEM, "tuner input allocation");
  if (hipMemset(in, 0, in_stride * (size_t)R) != hipSuccess ||
      hipMalloc((void**)&out, out_stride * (size_t)R) != hipSuccess) {
    (void)hipFree(in);
    return fail(HP_ENOMEM, "tuner output allocation");
  }
  hipStream_t st;
  if (hipStreamCreate(&st) != hipSuccess) {
    (void)hipFree(in);
    (void)hipFree(out);
    return fail(HP_EDEVICE, "tuner stream");
  }
  double t_auto = 0;
  s = time_candidate_batch(L0, R, in, in_stride, out, out_stride, reps, st, &t_auto);
  Recipe best{0, 0, 1, 1, 64, 1, t_auto};
  auto consider = [&](const Recipe& r) {
    hp_nest shaped;
    hp_level_map m;
    Lowered L;
    int64_t fb = 0;
    if (!apply_recipe(nest, r, kBatchWaves, &shaped, &m, &fb)) return;
    if (lower(&shaped, &m, flags, &L, kBatchWaves, fb) != HP_OK) return;
    double us = 0;
    if (time_candidate_batch(L, R, in, in_stride, out, out_stride, reps, st, &us) != HP_OK) return;
    if (us < best.us * 0.98) {
      best = r;
      best.us = us;
    }
  };
  if (s == HP_OK && tunable) {
    const int c = 16 / elem_bytes(nest->dtype);
    int64_t outs = 1;
    for (int l = 0; l < p; ++l) outs *= nest->extent[l];
    // default recipe first, so a tie keeps it
    const Recipe d = default_recipe(nest, kBatchWaves);
    if (d.mode != 0) consider(d);
    // mode 1: (J, K) rows
    for (int64_t k = c; k <= block && k <= (int64_t)c * 1024; k *= 2) {
      if (block % k != 0 && flat_interior(block, c, k) < k) continue;
      for (int vj = 1; vj <= 16; vj *= 2) {
        if ((64 / vj) * c > 4 * k) continue;  // most lanes of a row would idle
        const int64_t J = block / k;
        if (vj > J) continue;
        for (int gj = 1; gj <= 512; gj *= 2) {
          if ((int64_t)gj * kBatchWaves * vj > J) break;
          if (outs * gj > 65536) break;
          consider(Recipe{1, k, vj, gj, 64, 1, 0.0});
        }
      }
    }
    // mode 2: many outputs per task
    if (p >= 1) {
      for (int pw = 1; pw <= 64; pw *= 2) {
        if ((int64_t)pw * c > 4 * block && pw > 1) break;
        const int64_t per_pass = (64 / pw) * (int64_t)kBatchWaves;
        for (int64_t mult = 1; mult <= 64; mult *= 2) {
          const int64_t opt = per_pass * mult;
          if (opt > 2 * nest->extent[p - 1] && mult > 1) break;
          consider(Recipe{2, 0, 1, 1, pw, (int32_t)opt, 0.0});
        }
      }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    load_env_locked();
    g_cache[tune_key(nest)] = best;
  }
  (void)hipStreamDestroy(st);
  (void)hipFree(in);
  (void)hipFree(out);
  if (s != HP_OK) return s;
  if (best_us) *best_us = best.us;
  if (auto_us) *auto_us = t_auto;
  return HP_OK;
}
