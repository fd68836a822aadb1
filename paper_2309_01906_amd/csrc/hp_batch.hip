// Batches of nests: one persistent launch per kernel family, optionally replayed
// from a hipGraph, and the one-launch-per-nest baseline over the same plans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hp_internal.h"
#include "hp_batch_dev.h"
#include "hp_fold.h"
#include "hp_tune.h"

namespace hp {

hp_status batch_f32_launch(int, int, const BatchArgs&, int, int, size_t, hipStream_t);
hp_status batch_bf16_launch(int, int, const BatchArgs&, int, int, size_t, hipStream_t);
hp_status batch_i32_launch(int, int, const BatchArgs&, int, int, size_t, hipStream_t);
hp_status batch_i32_deep_launch(int, int, const BatchArgs&, int, int, size_t, hipStream_t);
int batch_f32_occupancy(int, int, int, size_t);
int batch_bf16_occupancy(int, int, int, size_t);
int batch_i32_occupancy(int, int, int, size_t);
int batch_i32_deep_occupancy(int, int, int, size_t);

hp_status launch_batch(int family, int chunk, const BatchArgs& B, int grid, int nw, size_t lds, hipStream_t st) {
  switch (family) {
    case FAM_F32_4: case FAM_F32_8: return batch_f32_launch(family, chunk, B, grid, nw, lds, st);
    case FAM_BF16_4: case FAM_BF16_8: return batch_bf16_launch(family, chunk, B, grid, nw, lds, st);
    case FAM_I32_FLAT: case FAM_I32_SEG: return batch_i32_launch(family, chunk, B, grid, nw, lds, st);
    default: return batch_i32_deep_launch(family, chunk, B, grid, nw, lds, st);
  }
}

int batch_occupancy(int family, int chunk, int nw, size_t lds) {
  switch (family) {
    case FAM_F32_4: case FAM_F32_8: return batch_f32_occupancy(family, chunk, nw, lds);
    case FAM_BF16_4: case FAM_BF16_8: return batch_bf16_occupancy(family, chunk, nw, lds);
    case FAM_I32_FLAT: case FAM_I32_SEG: return batch_i32_occupancy(family, chunk, nw, lds);
    default: return batch_i32_deep_occupancy(family, chunk, nw, lds);
  }
}

__global__ void k_clear_counters(unsigned int* p, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = 0u;
}

hp_status launch_clear(unsigned int* ctr, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_counters, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ctr, n);
  if (hipGetLastError() != hipSuccess) return fail(HP_EDEVICE, "counter clear launch failed");
  return HP_OK;
}

// Fold tasks: one wave each, grid-stride over the list.
template <bool ONE>
__device__ __forceinline__ void fold_body(const DevPlan* plans, const FoldTask* tasks, int n, void* const* outs,
                                          unsigned char* const* wss, void* out1, const unsigned char* ws1) {
  const int lane = (int)(threadIdx.x & 63);
  const int nwv = (int)(gridDim.x * (blockDim.x >> 6));
  for (int t = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); t < n; t += nwv) {
    const FoldTask ft = tasks[t];
    if (ONE) fold_task(plans[0], ft, out1, ws1, lane);
    else fold_task(plans[ft.nest], ft, outs[ft.nest], wss[ft.nest], lane);
  }
}

__global__ void __launch_bounds__(256) k_fold(const DevPlan* plans, const FoldTask* tasks, int n, void* const* outs,
                                              unsigned char* const* wss, unsigned int* ctr, int n_ctr) {
  // the persistent launches before this one on the stream have finished: nothing
  // reads their task counters any more
  for (int i = (int)(blockIdx.x * blockDim.x + threadIdx.x); i < n_ctr; i += (int)(gridDim.x * blockDim.x)) ctr[i] = 0u;
  fold_body<false>(plans, tasks, n, outs, wss, nullptr, nullptr);
}

__global__ void __launch_bounds__(256) k_fold_one(const DevPlan* plan, const FoldTask* tasks, int n, void* out,
                                                  const unsigned char* ws) {
  fold_body<true>(plan, tasks, n, nullptr, nullptr, out, ws);
}

static unsigned fold_grid(int n) {
  const int g = (n + 3) / 4;
  return (unsigned)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

hp_status launch_fold(const DevPlan* plans, const FoldTask* tasks, int n, void* const* outs,
                      unsigned char* const* wss, hipStream_t st, unsigned int* ctr, int n_ctr) {
  if (n <= 0 && n_ctr <= 0) return HP_OK;
  hipLaunchKernelGGL(k_fold, dim3(fold_grid(n)), dim3(256), 0, st, plans, tasks, n, outs, wss, ctr, n_ctr);
  if (hipGetLastError() != hipSuccess) return fail(HP_EDEVICE, "fold launch failed");
  return HP_OK;
}

hp_status launch_fold_one(const DevPlan* plan, const FoldTask* tasks, int n, void* out, const unsigned char* ws,
                          hipStream_t st) {
  if (n <= 0) return HP_OK;
  hipLaunchKernelGGL(k_fold_one, dim3(fold_grid(n)), dim3(256), 0, st, plan, tasks, n, out, ws);
  if (hipGetLastError() != hipSuccess) return fail(HP_EDEVICE, "fold launch failed");
  return HP_OK;
}

hp_status warm_batch_kernels(hipStream_t st) {
  BatchArgs A;
  memset(&A, 0, sizeof A);  // empty queues: every worker exits at once, nothing is read
  A.per_pop = 1;
  const size_t lds = (size_t)kBatchGroupWaves * kWaveLdsBytes;
  const int fams[][2] = {{FAM_F32_4, 4}, {FAM_F32_4, 1}, {FAM_F32_8, 4}, {FAM_F32_8, 1},
                         {FAM_BF16_4, 8}, {FAM_BF16_4, 1}, {FAM_BF16_8, 8}, {FAM_BF16_8, 1},
                         {FAM_I32_FLAT, 4}, {FAM_I32_FLAT, 1}, {FAM_I32_SEG, 4}, {FAM_I32_SEG, 1},
                         {FAM_I32_DEEP, 4}, {FAM_I32_DEEP, 1}};
  for (const auto& f : fams) {
    hp_status s = launch_batch(f[0], f[1], A, 1, kBatchGroupWaves, lds, st);
    if (s != HP_OK) return s;
  }
  hipLaunchKernelGGL(k_fold, dim3(1), dim3(64), 0, st, (const DevPlan*)nullptr, (const FoldTask*)nullptr, 0,
                     (void* const*)nullptr, (unsigned char* const*)nullptr, (unsigned int*)nullptr, 0);
  hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, st, (unsigned int*)nullptr, 0);
  if (hipGetLastError() != hipSuccess) return fail(HP_EDEVICE, "warm-up launch failed");
  return HP_OK;
}

// The SimpleDesc of a plan, if it has that form (see hp_batch_dev.h).
bool simple_desc_of(const DevPlan& P, SimpleDesc* D) {
  if (P.dtype != HP_F32 && P.dtype != HP_BF16) return false;
  const int c = P.dtype == HP_BF16 ? 8 : 4;
  if (P.depth != 2 || P.p != 1 || P.nseg != 1 || P.seg[0].op != HP_OP_SUM || P.gmode != GCOMB_NONE) return false;
  const DevLevel& L0 = P.lv[0];
  const DevLevel& L1 = P.lv[1];
  if (L1.gf != 1 || L1.wf != 1 || L1.vsh != 0 || L1.chunk != c || L1.ragged || L1.stride != 1) return false;
  if (L0.wf != 1 || L0.chunk != 1 || L0.ostride != 1 || (L0.vf > 1 && (1 << L0.vsh) != L1.vf)) return false;
  const int64_t lim = 0x7fffffffLL;
  if (L0.e > lim || L0.strips > lim || L1.strips > lim || L0.stride > lim || P.flat_b > lim) return false;
  if (L0.gdiv != 1 || (int64_t)L0.gf != P.grid) return false;
  memset(D, 0, sizeof *D);
  D->block = (int32_t)L0.stride;
  D->flat_b = (int32_t)P.flat_b;
  D->flat_e = (int32_t)P.flat_e;
  D->e0 = (int32_t)L0.e;
  D->g0 = (int32_t)L0.gf;
  D->v0 = L0.vf;
  D->v1 = L1.vf;
  D->strips1 = (int32_t)L1.strips;
  D->strips0 = (int32_t)L0.strips;
  D->bits = (uint32_t)(L0.vf > 1 ? L0.vsh : 0) | (P.out_kind == OUT_F64 ? 0x100u : 0u) |
            ((P.seg[0].ufast & 0x3Fu) << 16);
  return true;
}

void deal_tasks(const int2* ordered, const double* weight, int n, int grid, int2* out, BatchArgs* B) {
  const int nq = grid < kQueues ? (grid < 1 ? 1 : grid) : kQueues;
  // queue q is served by the workgroups b < grid with b % kQueues == q; a task goes
  // to the queue with the least cost per serving workgroup so far (ties: the lowest
  // queue), found with a min-heap
  double load[kQueues] = {};
  int cnt[kQueues] = {};
  double groups[kQueues] = {};
  for (int q = 0; q < nq; ++q) groups[q] = (double)((grid - q + kQueues - 1) / kQueues);
  typedef std::pair<double, int> Key;
  std::vector<Key> heap;
  heap.reserve((size_t)nq);
  for (int q = 0; q < nq; ++q) heap.push_back(Key(0.0, q));
  std::vector<int> qof((size_t)n);
  for (int j = 0; j < n; ++j) {
    std::pop_heap(heap.begin(), heap.end(), std::greater<Key>());
    const int q = heap.back().second;
    qof[(size_t)j] = q;
    load[q] += weight[j];
    ++cnt[q];
    heap.back() = Key(load[q] / groups[q], q);
    std::push_heap(heap.begin(), heap.end(), std::greater<Key>());
  }
  int pos = 0, fill[kQueues];
  for (int q = 0; q < kQueues; ++q) {
    B->qbeg[q] = pos;
    fill[q] = pos;
    pos += cnt[q];
  }
  B->qbeg[kQueues] = pos;
  for (int j = 0; j < n; ++j) out[fill[qof[(size_t)j]]++] = ordered[j];
  // several tasks per atomic when every worker has many to do
  const long long workers = (long long)grid * kBatchGroupWaves;
  long long k = (long long)n / (workers * 8);
  B->per_pop = (int)(k < 1 ? 1 : (k > 8 ? 8 : k));
}

hp_status launch_single(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds,
                        hipStream_t st) {
  switch (P.dtype) {
    case HP_F32: return launch_nest_f32(P, dP, in, out, ws, lds, st);
    case HP_BF16: return launch_nest_bf16(P, dP, in, out, ws, lds, st);
    default: return launch_nest_i32(P, dP, in, out, ws, lds, st);
  }
}

}  // namespace hp

namespace {

struct Group {  // nests of one kernel family and chunk: one persistent launch
  int family, chunk;
  long long n_tasks;
  hp::BatchArgs args;  // pointers into the batch's device memory
  int grid;
  size_t lds;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct hp_batch_s {
  int64_t n;
  uint32_t flags;
  int device;
  int nw;
  std::vector<hp::DevPlan> plans;
  std::vector<hp_plan_info> infos;
  hp::DevPlan* d_plans = nullptr;
  const void** d_in = nullptr;
  void** d_out = nullptr;
  unsigned char** d_ws = nullptr;
  std::vector<unsigned char*> ws_ptrs;
  void* arena = nullptr;  // tasks, counters, fold tasks, workspaces
  std::vector<Group> groups;
  hp::FoldTask* d_fold = nullptr;  // in the arena
  int n_fold = 0;
  std::vector<int> fold_beg;      // nest i's fold tasks: [fold_beg[i], fold_beg[i + 1])
  std::vector<hp::SimpleDesc> simple;  // host copy of the compact descriptors (pointers set by set_io)
  std::vector<char> is_simple;
  hp::SimpleDesc* d_simple = nullptr;  // in the arena
  bool io_set = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph_each = nullptr;
  hipGraphExec_t exec_each = nullptr;
  double bytes = 0;
};

static void batch_free(hp_batch_s* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->exec_each) (void)hipGraphExecDestroy(b->exec_each);
  if (b->graph_each) (void)hipGraphDestroy(b->graph_each);
  if (b->arena) (void)hipFree(b->arena);
  if (b->d_plans) (void)hipFree(b->d_plans);
  if (b->d_in) (void)hipFree(b->d_in);
  delete b;
}

namespace hp {

// Build a batch from plans made by the caller (batched plans: kBatchWaves waves).
hp_status batch_from_plans(const std::vector<Lowered>& plans, uint32_t flags, hp_batch_s** out);

}  // namespace hp

extern "C" hp_status hp_batch_plan(const hp_nest* nests, int64_t n, uint32_t flags, hp_batch_t* out) {
  using namespace hp;
  if (!out || !nests || n < 1) return fail(HP_EINVAL, "null argument or empty batch");
  *out = nullptr;
  if (flags & ~(uint32_t)(HP_BATCH_GRAPH | HP_FLAG_OUT_F32 | HP_BATCH_NO_TUNE))
    return fail(HP_EINVAL, "unknown batch flag bits 0x%x", flags);
  std::vector<Lowered> plans((size_t)n);
  const uint32_t pflags = flags & HP_FLAG_OUT_F32;
  for (int64_t i = 0; i < n; ++i) {
    hp_status s = plan_for_batch(&nests[i], pflags, !(flags & HP_BATCH_NO_TUNE), kBatchWaves, &plans[(size_t)i]);
    if (s != HP_OK) {
      char msg[512];
      snprintf(msg, sizeof msg, "%s", hp_last_error());
      return fail(s, "nest %lld: %s", (long long)i, msg);
    }
  }
  return batch_from_plans(plans, flags, out);
}

extern "C" hp_status hp_batch_plan_inspect(const hp_nest* nests, int64_t n, uint32_t flags, hp_plan_info* infos) {
  using namespace hp;
  if (!nests || !infos || n < 1) return fail(HP_EINVAL, "null argument or empty batch");
  const uint32_t pflags = flags & HP_FLAG_OUT_F32;
  for (int64_t i = 0; i < n; ++i) {
    Lowered L;
    hp_status s = plan_for_batch(&nests[i], pflags, !(flags & HP_BATCH_NO_TUNE), kBatchWaves, &L);
    if (s != HP_OK) return s;
    infos[i] = L.info;
  }
  return HP_OK;
}

hp_status hp::batch_from_plans(const std::vector<Lowered>& plans, uint32_t flags, hp_batch_s** out) {
  const int64_t n = (int64_t)plans.size();
  hp_batch_s* b = new (std::nothrow) hp_batch_s;
  if (!b) return fail(HP_ENOMEM, "host allocation failed");
  b->n = n;
  b->flags = flags;
  b->nw = kBatchWaves;
  if (hipGetDevice(&b->device) != hipSuccess) {
    batch_free(b);
    return fail(HP_EDEVICE, "no HIP device");
  }
  b->plans.resize((size_t)n);
  b->infos.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    b->plans[(size_t)i] = plans[(size_t)i].dp;
    b->infos[(size_t)i] = plans[(size_t)i].info;
    b->bytes += (double)plans[(size_t)i].info.in_bytes + (double)plans[(size_t)i].info.out_bytes;
  }
  // groups by (family, chunk); tasks largest first inside a group
  std::vector<std::vector<int64_t>> members;
  std::vector<std::pair<int, int>> keys;
  for (int64_t i = 0; i < n; ++i) {
    const DevPlan& P = b->plans[(size_t)i];
    std::pair<int, int> k(family_of(P), P.chunk);
    size_t g = 0;
    while (g < keys.size() && keys[g] != k) ++g;
    if (g == keys.size()) {
      keys.push_back(k);
      members.emplace_back();
    }
    members[g].push_back(i);
  }
  // device memory: plans, pointer tables, then one arena for tasks, counters and workspaces
  // the task counters of every group sit together at the start (zero after the
  // upload; each run leaves them at zero again), then each group's task list
  size_t arena_bytes = align_up(keys.size() * kCtrWords * sizeof(unsigned int), 256);
  std::vector<size_t> task_off(keys.size()), ctr_off(keys.size());
  std::vector<long long> ntask(keys.size(), 0);
  for (size_t g = 0; g < keys.size(); ++g) {
    for (int64_t i : members[g]) ntask[g] += b->plans[(size_t)i].grid;
    ctr_off[g] = g * kCtrWords * sizeof(unsigned int);
    task_off[g] = arena_bytes;
    arena_bytes = align_up(arena_bytes + (size_t)ntask[g] * sizeof(int2), 256);
    if (ntask[g] > 0x7fffffffLL) {
      batch_free(b);
      return fail(HP_ETOOBIG, "batch group has %lld tasks, more than 2^31 - 1", ntask[g]);
    }
  }
  // compact descriptors of the nests whose plans have the simple form (float
  // families of depth <= 4 only: those kernels hold the simple path)
  const size_t simple_off = arena_bytes;
  arena_bytes = align_up(arena_bytes + (size_t)n * sizeof(SimpleDesc), 256);
  std::vector<SimpleDesc> simple((size_t)n);
  std::vector<char> is_simple((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const DevPlan& P = b->plans[(size_t)i];
    const int fam = family_of(P);
    if ((fam == FAM_F32_4 || fam == FAM_BF16_4) && simple_desc_of(P, &simple[(size_t)i])) is_simple[(size_t)i] = 1;
  }
  std::vector<hp::FoldTask> folds;
  b->fold_beg.assign((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    b->fold_beg[(size_t)i] = (int)folds.size();
    fold_tasks_of(b->plans[(size_t)i], (int)i, folds);
  }
  b->fold_beg[(size_t)n] = (int)folds.size();
  b->n_fold = (int)folds.size();
  const size_t fold_off = arena_bytes;
  arena_bytes = align_up(arena_bytes + folds.size() * sizeof(hp::FoldTask), 256);
  std::vector<size_t> ws_off((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const size_t wb = b->infos[(size_t)i].workspace_bytes;
    if (wb) {
      ws_off[(size_t)i] = arena_bytes;
      arena_bytes = align_up(arena_bytes + wb, 256);
    }
  }
  if (hipMalloc(&b->d_plans, sizeof(DevPlan) * (size_t)n) != hipSuccess ||
      hipMalloc((void**)&b->d_in, 3 * sizeof(void*) * (size_t)n) != hipSuccess ||
      hipMalloc(&b->arena, arena_bytes) != hipSuccess) {
    batch_free(b);
    return fail(HP_ENOMEM, "batch device allocation failed");
  }
  b->d_out = reinterpret_cast<void**>(const_cast<void**>(b->d_in + n));
  b->d_ws = reinterpret_cast<unsigned char**>(const_cast<void**>(b->d_in + 2 * n));
  std::vector<unsigned char> host_arena(arena_bytes, 0);
  memcpy(host_arena.data() + simple_off, simple.data(), (size_t)n * sizeof(SimpleDesc));
  b->d_simple = reinterpret_cast<SimpleDesc*>((unsigned char*)b->arena + simple_off);
  b->simple.swap(simple);
  b->is_simple.swap(is_simple);
  if (!folds.empty()) memcpy(host_arena.data() + fold_off, folds.data(), folds.size() * sizeof(hp::FoldTask));
  b->d_fold = reinterpret_cast<hp::FoldTask*>((unsigned char*)b->arena + fold_off);
  b->ws_ptrs.assign((size_t)n, nullptr);
  for (int64_t i = 0; i < n; ++i)
    if (b->infos[(size_t)i].workspace_bytes) b->ws_ptrs[(size_t)i] = (unsigned char*)b->arena + ws_off[(size_t)i];
  for (size_t g = 0; g < keys.size(); ++g) {
    std::vector<int64_t>& mem = members[g];
    // largest work per task first
    std::stable_sort(mem.begin(), mem.end(), [&](int64_t a, int64_t c) {
      const double wa = (double)b->infos[(size_t)a].in_bytes / (double)b->plans[(size_t)a].grid;
      const double wc = (double)b->infos[(size_t)c].in_bytes / (double)b->plans[(size_t)c].grid;
      return wa > wc;
    });
    std::vector<int2> ordered((size_t)ntask[g]);
    std::vector<double> weight((size_t)ntask[g]);
    long long k = 0;
    for (int64_t i : mem) {
      const double wt = task_cost((double)b->infos[(size_t)i].in_bytes / (double)b->plans[(size_t)i].grid);
      for (long long w = 0; w < b->plans[(size_t)i].grid; ++w) {
        weight[(size_t)k] = wt;
        ordered[(size_t)k++] = make_int2((int)i, (int)w | (b->is_simple[(size_t)i] ? kSimpleTask : 0));
      }
    }
    Group G;
    G.family = keys[g].first;
    G.chunk = keys[g].second;
    G.n_tasks = ntask[g];
    // wave tasks: every wavefront of a persistent workgroup runs tasks on its own
    G.lds = (size_t)kBatchGroupWaves * kWaveLdsBytes;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess || cus < 1)
      cus = 256;
    int occ = batch_occupancy(G.family, G.chunk, kBatchGroupWaves, G.lds);
    if (occ < 1) occ = 1;
    long long grid = (long long)cus * occ;
    const long long need = (G.n_tasks + kBatchGroupWaves - 1) / kBatchGroupWaves;
    if (grid > need) grid = need;
    G.grid = (int)grid;
    deal_tasks(ordered.data(), weight.data(), (int)ntask[g], G.grid,
               reinterpret_cast<int2*>(host_arena.data() + task_off[g]), &G.args);
    G.args.tasks = reinterpret_cast<const int2*>((unsigned char*)b->arena + task_off[g]);
    G.args.simple = b->d_simple;
    G.args.ctr = reinterpret_cast<unsigned int*>((unsigned char*)b->arena + ctr_off[g]);
    b->groups.push_back(G);
  }
  std::vector<unsigned char*> wsv(b->ws_ptrs);
  if (hipMemcpy(b->d_plans, b->plans.data(), sizeof(DevPlan) * (size_t)n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->arena, host_arena.data(), arena_bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_ws, wsv.data(), sizeof(void*) * (size_t)n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(b->d_in, 0, 2 * sizeof(void*) * (size_t)n) != hipSuccess) {
    batch_free(b);
    return fail(HP_EDEVICE, "batch upload failed");
  }
  *out = b;
  return HP_OK;
}

extern "C" hp_status hp_batch_info(hp_batch_t b, int64_t i, hp_plan_info* info) {
  if (!b || !info || i < 0 || i >= b->n) return hp::fail(HP_EINVAL, "bad batch, index or info pointer");
  *info = b->infos[(size_t)i];
  return HP_OK;
}

extern "C" hp_status hp_batch_stats(hp_batch_t b, int64_t* n_launches, int64_t* n_tasks, int64_t* n_workers,
                                    double* bytes) {
  if (!b) return hp::fail(HP_EINVAL, "null batch");
  long long t = 0, w = 0;
  for (const Group& g : b->groups) {
    t += g.n_tasks;
    w += (long long)g.grid * hp::kBatchGroupWaves;
  }
  if (n_launches) *n_launches = (int64_t)b->groups.size();
  if (n_tasks) *n_tasks = t;
  if (n_workers) *n_workers = w;
  if (bytes) *bytes = b->bytes;
  return HP_OK;
}

extern "C" hp_status hp_batch_set_io(hp_batch_t b, const void* const* d_in, void* const* d_out) {
  if (!b || !d_in || !d_out) return hp::fail(HP_EINVAL, "null argument");
  for (int64_t i = 0; i < b->n; ++i) {
    if (!d_in[i] || !d_out[i]) return hp::fail(HP_EINVAL, "nest %lld: null pointer", (long long)i);
    if (reinterpret_cast<uintptr_t>(d_in[i]) & 15u)
      return hp::fail(HP_EINVAL, "nest %lld: input not 16-byte aligned", (long long)i);
    const int od = b->infos[(size_t)i].out_dtype;
    const uintptr_t al = (od == HP_I64 || od == HP_F64) ? 7u : 3u;
    if (reinterpret_cast<uintptr_t>(d_out[i]) & al)
      return hp::fail(HP_EINVAL, "nest %lld: output misaligned", (long long)i);
  }
  if (b->exec_each) {  // that graph holds the old pointers as launch arguments
    (void)hipGraphExecDestroy(b->exec_each);
    (void)hipGraphDestroy(b->graph_each);
    b->exec_each = nullptr;
    b->graph_each = nullptr;
  }
  bool any_simple = false;
  for (int64_t i = 0; i < b->n; ++i)
    if (b->is_simple[(size_t)i]) {
      b->simple[(size_t)i].in = d_in[i];
      b->simple[(size_t)i].out = d_out[i];
      any_simple = true;
    }
  if (hipMemcpy(b->d_in, d_in, sizeof(void*) * (size_t)b->n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_out, d_out, sizeof(void*) * (size_t)b->n, hipMemcpyHostToDevice) != hipSuccess ||
      (any_simple && hipMemcpy(b->d_simple, b->simple.data(), sizeof(hp::SimpleDesc) * (size_t)b->n,
                               hipMemcpyHostToDevice) != hipSuccess))
    return hp::fail(HP_EDEVICE, "pointer table upload failed");
  b->io_set = true;
  return HP_OK;
}

static hp_status launch_groups(hp_batch_s* b, hipStream_t st) {
  for (const Group& G : b->groups) {
    hp::BatchArgs A = G.args;
    A.plans = b->d_plans;
    A.ins = b->d_in;
    A.outs = b->d_out;
    A.wss = b->d_ws;
    // With fold tasks, the fold kernel that ends the run clears the counters for
    // the next one; without, each group clears its own before it starts.
    hp_status s = b->n_fold > 0 ? HP_OK : hp::launch_clear(A.ctr, hp::kCtrWords, st);
    if (s == HP_OK) s = hp::launch_batch(G.family, G.chunk, A, G.grid, hp::kBatchGroupWaves, G.lds, st);
    if (s != HP_OK) return s;
  }
  if (b->n_fold <= 0) return HP_OK;
  return hp::launch_fold(b->d_plans, b->d_fold, b->n_fold, b->d_out, b->d_ws, st,
                         reinterpret_cast<unsigned int*>(b->arena), (int)(b->groups.size() * hp::kCtrWords));
}

static hp_status capture(hp_batch_s* b, bool each, hipGraph_t* graph, hipGraphExec_t* exec);

extern "C" hp_status hp_batch_run(hp_batch_t b, void* stream) {
  if (!b) return hp::fail(HP_EINVAL, "null batch");
  if (!b->io_set) return hp::fail(HP_ESTATE, "hp_batch_set_io has not been called");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
    return hp::fail(HP_EINVAL, "batch was made on device %d, current device is %d", b->device, dev);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (b->flags & HP_BATCH_GRAPH) {
    if (!b->exec) {
      hp_status s = capture(b, false, &b->graph, &b->exec);
      if (s != HP_OK) return s;
    }
    if (hipGraphLaunch(b->exec, st) != hipSuccess) return hp::fail(HP_EDEVICE, "graph launch failed");
    return HP_OK;
  }
  return launch_groups(b, st);
}

// The fold kernel of nest i alone (what hp_run launches after a grid-split nest).
static hp_status launch_fold_of(hp_batch_s* b, int64_t i, hipStream_t st) {
  const int f0 = b->fold_beg[(size_t)i], f1 = b->fold_beg[(size_t)i + 1];
  if (f1 == f0) return HP_OK;
  return hp::launch_fold(b->d_plans, b->d_fold + f0, f1 - f0, b->d_out, b->d_ws, st);
}

// Baseline: the same plans, one single-nest launch per nest (optionally replayed
// from one graph holding all of those launches).
static hp_status launch_each(hp_batch_s* b, hipStream_t st) {
  std::vector<const void*> in((size_t)b->n);
  std::vector<void*> out((size_t)b->n);
  if (hipMemcpy(in.data(), b->d_in, sizeof(void*) * (size_t)b->n, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(out.data(), b->d_out, sizeof(void*) * (size_t)b->n, hipMemcpyDeviceToHost) != hipSuccess)
    return hp::fail(HP_EDEVICE, "pointer table download failed");
  for (int64_t i = 0; i < b->n; ++i) {
    hp_status s = hp::launch_single(b->plans[(size_t)i], b->d_plans + i, in[(size_t)i], out[(size_t)i],
                                    b->ws_ptrs[(size_t)i], b->infos[(size_t)i].lds_bytes, st);
    if (s == HP_OK) s = launch_fold_of(b, i, st);
    if (s != HP_OK) return s;
  }
  return HP_OK;
}

static hp_status capture(hp_batch_s* b, bool each, hipGraph_t* graph, hipGraphExec_t* exec) {
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return hp::fail(HP_EDEVICE, "capture stream creation failed");
  hp_status s = HP_OK;
  if (each) {
    // the host-side pointer copies must not be captured: fetch them first
    std::vector<const void*> ins((size_t)b->n);
    std::vector<void*> outs((size_t)b->n);
    if (hipMemcpy(ins.data(), b->d_in, sizeof(void*) * (size_t)b->n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(outs.data(), b->d_out, sizeof(void*) * (size_t)b->n, hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return hp::fail(HP_EDEVICE, "pointer table download failed");
    }
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return hp::fail(HP_EDEVICE, "begin capture failed");
    }
    for (int64_t i = 0; i < b->n && s == HP_OK; ++i) {
      s = hp::launch_single(b->plans[(size_t)i], b->d_plans + i, ins[(size_t)i], outs[(size_t)i],
                            b->ws_ptrs[(size_t)i], b->infos[(size_t)i].lds_bytes, cs);
      if (s == HP_OK) s = launch_fold_of(b, i, cs);
    }
  } else {
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return hp::fail(HP_EDEVICE, "begin capture failed");
    }
    s = launch_groups(b, cs);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  (void)hipStreamDestroy(cs);
  if (s != HP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess || !g) return hp::fail(HP_EDEVICE, "end capture failed");
  if (hipGraphInstantiate(exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hp::fail(HP_EDEVICE, "graph instantiation failed");
  }
  *graph = g;
  return HP_OK;
}

extern "C" hp_status hp_batch_run_each(hp_batch_t b, void* stream, int32_t use_graph) {
  if (!b) return hp::fail(HP_EINVAL, "null batch");
  if (!b->io_set) return hp::fail(HP_ESTATE, "hp_batch_set_io has not been called");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (use_graph) {
    if (!b->exec_each) {
      hp_status s = capture(b, true, &b->graph_each, &b->exec_each);
      if (s != HP_OK) return s;
    }
    if (hipGraphLaunch(b->exec_each, st) != hipSuccess) return hp::fail(HP_EDEVICE, "graph launch failed");
    return HP_OK;
  }
  return launch_each(b, st);
}

extern "C" hp_status hp_batch_destroy(hp_batch_t b) {
  batch_free(b);
  return HP_OK;
}
