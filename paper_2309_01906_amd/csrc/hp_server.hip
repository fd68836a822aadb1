// Serving loop: continuous batching of nest-reduction requests.
//
// Clients submit requests (a nest plus device input/output pointers) at any time.
// One scheduler thread admits pending requests in arrival order while their bytes
// (input + output + grid-combine workspace) fit in the HBM budget, forms a batch as
// soon as one of K in-flight slots is free, uploads the batch's plans / task list /
// pointer tables into that slot's device arena with one asynchronous copy, launches
// the persistent kernels of the batch on the slot's stream, and polls the slots'
// completion events.  Batches on different slots overlap on the device.  Every
// request keeps the plan it would get alone, so its result does not depend on what
// it was batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hp_internal.h"
#include "hp_batch_dev.h"
#include "hp_fold.h"
#include "hp_tune.h"

namespace {

using Clock = std::chrono::steady_clock;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Request {
  uint64_t id;
  hp_nest nest;
  const void* in;
  void* out;
  hp::Lowered L;
  size_t bytes;  // budget charge
  hp_req_info info;
  int bypassed;
  // what the request adds to a slot arena (see Tally)
  std::pair<int, int> key;  // kernel family and chunk: one persistent launch per key
  long long ntask;          // workgroup tasks
  long long nfold;          // fold tasks
  size_t ws;                // grid-combine workspace, 256-byte aligned
};

size_t A256(size_t x) { return align_up(x, 256); }

// Bytes of slot arena a batch needs: plans, the pointer tables, per kernel family
// its task list and queue counters, the fold tasks and the workspaces, each region
// 256-byte aligned.  layout_batch lays the regions out in this order; Tally keeps
// the same sum up to date while a batch is packed, one request at a time, so a
// batch never outgrows its slot.
struct Tally {
  int64_t n = 0;
  long long nfold = 0;
  size_t ws = 0;
  std::vector<std::pair<int, int>> keys;
  std::vector<long long> ntask;

  size_t total() const {
    size_t t = A256(sizeof(hp::DevPlan) * (size_t)n) + A256(3 * sizeof(void*) * (size_t)n);
    for (long long k : ntask) t += A256((size_t)k * sizeof(int2)) + A256(hp::kCtrWords * sizeof(unsigned int));
    return t + A256((size_t)nfold * sizeof(hp::FoldTask)) + ws;
  }
  void add(const Request& r) {
    ++n;
    nfold += r.nfold;
    ws += r.ws;
    size_t g = 0;
    while (g < keys.size() && keys[g] != r.key) ++g;
    if (g == keys.size()) {
      keys.push_back(r.key);
      ntask.push_back(0);
    }
    ntask[g] += r.ntask;
  }
  size_t total_with(const Request& r) const {
    Tally t = *this;
    t.add(r);
    return t.total();
  }
};

struct Layout {
  size_t plans_off = 0, ptr_off = 0, fold_off = 0, ws_begin = 0, total = 0;
  std::vector<std::pair<int, int>> keys;
  std::vector<std::vector<int64_t>> members;
  std::vector<size_t> task_off, ctr_off;
  std::vector<long long> ntask;
  std::vector<hp::FoldTask> folds;
  std::vector<size_t> ws_off;
};

void layout_batch(const std::vector<Request*>& rs, Layout& Lo) {
  using namespace hp;
  const int64_t n = (int64_t)rs.size();
  size_t off = 0;
  Lo.plans_off = off;
  off = align_up(off + sizeof(DevPlan) * (size_t)n, 256);
  Lo.ptr_off = off;
  off = align_up(off + 3 * sizeof(void*) * (size_t)n, 256);
  for (int64_t i = 0; i < n; ++i) {
    size_t g = 0;
    while (g < Lo.keys.size() && Lo.keys[g] != rs[(size_t)i]->key) ++g;
    if (g == Lo.keys.size()) {
      Lo.keys.push_back(rs[(size_t)i]->key);
      Lo.members.emplace_back();
    }
    Lo.members[g].push_back(i);
  }
  Lo.task_off.resize(Lo.keys.size());
  Lo.ctr_off.resize(Lo.keys.size());
  Lo.ntask.assign(Lo.keys.size(), 0);
  for (size_t g = 0; g < Lo.keys.size(); ++g) {
    for (int64_t i : Lo.members[g]) Lo.ntask[g] += rs[(size_t)i]->ntask;
    Lo.task_off[g] = off;
    off = align_up(off + (size_t)Lo.ntask[g] * sizeof(int2), 256);
    Lo.ctr_off[g] = off;
    off = align_up(off + kCtrWords * sizeof(unsigned int), 256);
  }
  for (int64_t i = 0; i < n; ++i) fold_tasks_of(rs[(size_t)i]->L.dp, (int)i, Lo.folds);
  Lo.fold_off = off;
  off = align_up(off + Lo.folds.size() * sizeof(FoldTask), 256);
  Lo.ws_begin = off;
  Lo.ws_off.assign((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (rs[(size_t)i]->ws) {
      Lo.ws_off[(size_t)i] = off;
      off += rs[(size_t)i]->ws;
    }
  }
  Lo.total = off;
}

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  unsigned char* d_arena = nullptr;
  unsigned char* h_stage = nullptr;
  size_t cap = 0;
  bool busy = false;
  std::vector<uint64_t> reqs;
  size_t charged = 0;
  double t_launch = 0;
  double fake_done = 0;  // fake executor: completion time
  int64_t batch_id = 0;
  // a launch failed after work was enqueued: the slot stays busy until its stream
  // has drained (the event of the last enqueued step), then its requests fail with err
  int32_t err = HP_OK;
};

}  // namespace

struct hp_server_s {
  hp_server_cfg cfg;
  int device = 0;
  bool fake = false;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_done;
  std::condition_variable cv_work;
  std::deque<uint64_t> pending;              // arrival order
  std::unordered_map<uint64_t, Request> reqs;
  std::vector<Slot> slots;
  std::atomic<bool> stop{false};
  std::thread th;
  uint64_t next_id = 1;
  size_t in_use = 0;
  int64_t batches = 0;
  // stats
  std::vector<double> lat;  // completed latencies (us)
  int64_t submitted = 0, completed = 0, failed = 0;
  double bytes_done = 0, first_arrival = -1, last_done = 0;
  int64_t max_queue = 0;
  size_t max_in_use = 0;
  int64_t fail_every = 0;  // test hook: fail every n-th batch
  // persistent grid per (family, chunk)
  std::unordered_map<int, int> occ;
  int cus = 256;

  double now() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }
};

namespace {

int occ_key(int fam, int chunk) { return fam * 16 + chunk; }

// Lay out a batch in the slot's staging buffer, copy it to the device arena and
// launch one persistent kernel per (family, chunk) group, then the fold kernel.
// These device steps go onto the slot's stream in order.  On failure, *drain says
// whether some of them were already enqueued: then the slot must stay busy until
// its stream has finished with the staging buffer and the arena.  The fake executor
// (host-only tests) runs the same layout and steps without touching a device.
hp_status launch_slot(hp_server_s* S, Slot& slot, std::vector<Request*>& rs, bool* drain) {
  using namespace hp;
  *drain = false;
  const int64_t n = (int64_t)rs.size();
  Layout Lo;
  layout_batch(rs, Lo);
  if (Lo.total > slot.cap)
    return fail(HP_ETOOBIG, "batch needs %zu bytes of slot arena, capacity %zu", Lo.total, slot.cap);
  const size_t lds = (size_t)kBatchGroupWaves * kWaveLdsBytes;
  const int n_steps = 1 + (int)Lo.keys.size() + (Lo.folds.empty() ? 0 : 1);
  // test hook: this batch fails before device step fail_step (0: before the upload)
  int fail_at = -1;
  if (S->fail_every > 0 && slot.batch_id % S->fail_every == 0)
    fail_at = S->cfg.fail_step < n_steps ? S->cfg.fail_step : n_steps;
  double work = 0;  // fake executor: bytes the enqueued steps read
  auto hook = [&](int step) -> hp_status {
    if (step != fail_at) return HP_OK;
    *drain = step > 0;
    return fail(HP_EDEVICE, "injected failure before device step %d", step);
  };
  if (S->fake) {
    for (int step = 0; step <= n_steps; ++step) {
      hp_status s = hook(step);
      if (s != HP_OK) {
        slot.fake_done = S->now() + 5.0 + work / 4.0e3;
        return s;
      }
      if (step > 0 && step <= (int)Lo.keys.size())
        for (int64_t i : Lo.members[(size_t)step - 1]) work += (double)rs[(size_t)i]->L.info.in_bytes;
    }
    slot.fake_done = S->now() + 5.0 + work / 4.0e3;  // a 4 GB/s pretend device
    return HP_OK;
  }
  unsigned char* h = slot.h_stage;
  unsigned char* d = slot.d_arena;
  DevPlan* hp_ = reinterpret_cast<DevPlan*>(h + Lo.plans_off);
  const void** hin = reinterpret_cast<const void**>(h + Lo.ptr_off);
  void** hout = reinterpret_cast<void**>(h + Lo.ptr_off) + n;
  unsigned char** hws = reinterpret_cast<unsigned char**>(h + Lo.ptr_off) + 2 * n;
  for (int64_t i = 0; i < n; ++i) {
    hp_[i] = rs[(size_t)i]->L.dp;
    hin[i] = rs[(size_t)i]->in;
    hout[i] = rs[(size_t)i]->out;
    hws[i] = Lo.ws_off[(size_t)i] ? d + Lo.ws_off[(size_t)i] : nullptr;
  }
  std::vector<BatchArgs> args(Lo.keys.size());
  std::vector<int> grid(Lo.keys.size());
  for (size_t g = 0; g < Lo.keys.size(); ++g) {
    std::vector<int64_t>& mem = Lo.members[g];
    std::stable_sort(mem.begin(), mem.end(), [&](int64_t a, int64_t c) {
      const double wa = (double)rs[(size_t)a]->L.info.in_bytes / (double)rs[(size_t)a]->L.dp.grid;
      const double wc = (double)rs[(size_t)c]->L.info.in_bytes / (double)rs[(size_t)c]->L.dp.grid;
      return wa > wc;
    });
    std::vector<int2> ordered((size_t)Lo.ntask[g]);
    std::vector<double> weight((size_t)Lo.ntask[g]);
    long long k = 0;
    for (int64_t i : mem) {
      const double wt = task_cost((double)rs[(size_t)i]->L.info.in_bytes / (double)rs[(size_t)i]->L.dp.grid);
      for (long long w = 0; w < rs[(size_t)i]->L.dp.grid; ++w) {
        weight[(size_t)k] = wt;
        ordered[(size_t)k++] = make_int2((int)i, (int)w);
      }
    }
    const int key = occ_key(Lo.keys[g].first, Lo.keys[g].second);
    auto it = S->occ.find(key);
    int o;
    if (it == S->occ.end()) {
      o = batch_occupancy(Lo.keys[g].first, Lo.keys[g].second, kBatchGroupWaves, lds);
      if (o < 1) o = 1;
      S->occ[key] = o;
    } else {
      o = it->second;
    }
    long long gr = (long long)S->cus * o;
    const long long need = (Lo.ntask[g] + kBatchGroupWaves - 1) / kBatchGroupWaves;
    if (gr > need) gr = need;
    grid[g] = (int)gr;
    deal_tasks(ordered.data(), weight.data(), (int)Lo.ntask[g], grid[g], reinterpret_cast<int2*>(h + Lo.task_off[g]),
               &args[g]);
    memset(h + Lo.ctr_off[g], 0, kCtrWords * sizeof(unsigned int));
  }
  if (!Lo.folds.empty()) memcpy(h + Lo.fold_off, Lo.folds.data(), Lo.folds.size() * sizeof(FoldTask));
  // step 0: upload the descriptors; the workspaces need no clearing (every partial
  // is written before the fold kernel reads it)
  hp_status s = hook(0);
  if (s != HP_OK) return s;
  if (hipMemcpyAsync(d, h, Lo.ws_begin, hipMemcpyHostToDevice, slot.st) != hipSuccess)
    return fail(HP_EDEVICE, "batch upload failed");
  int step = 1;
  // after the first enqueued step, any failure leaves work on the stream
  for (size_t g = 0; g < Lo.keys.size(); ++g, ++step) {
    if ((s = hook(step)) != HP_OK) return s;
    BatchArgs A = args[g];
    A.plans = reinterpret_cast<const DevPlan*>(d + Lo.plans_off);
    A.tasks = reinterpret_cast<const int2*>(d + Lo.task_off[g]);
    A.ctr = reinterpret_cast<unsigned int*>(d + Lo.ctr_off[g]);
    A.ins = reinterpret_cast<const void* const*>(d + Lo.ptr_off);
    A.outs = reinterpret_cast<void* const*>(d + Lo.ptr_off) + n;
    A.wss = reinterpret_cast<unsigned char* const*>(d + Lo.ptr_off) + 2 * n;
    s = launch_batch(Lo.keys[g].first, Lo.keys[g].second, A, grid[g], kBatchGroupWaves, lds, slot.st);
    if (s != HP_OK) {
      *drain = true;
      return s;
    }
  }
  if (!Lo.folds.empty()) {
    if ((s = hook(step)) != HP_OK) return s;
    s = launch_fold(reinterpret_cast<const DevPlan*>(d + Lo.plans_off),
                    reinterpret_cast<const FoldTask*>(d + Lo.fold_off), (int)Lo.folds.size(),
                    reinterpret_cast<void* const*>(d + Lo.ptr_off) + n,
                    reinterpret_cast<unsigned char* const*>(d + Lo.ptr_off) + 2 * n, slot.st);
    if (s != HP_OK) {
      *drain = true;
      return s;
    }
    ++step;
  }
  if ((s = hook(step)) != HP_OK) return s;
  if (hipEventRecord(slot.ev, slot.st) != hipSuccess) {
    *drain = true;
    return fail(HP_EDEVICE, "event record failed");
  }
  return HP_OK;
}

void finish_slot(hp_server_s* S, Slot& slot, int32_t status) {
  const double t = S->now();
  for (uint64_t id : slot.reqs) {
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) continue;
    Request& r = it->second;
    r.info.status = status;
    r.info.t_done_us = t;
    if (status == HP_OK) {
      ++S->completed;
      S->lat.push_back(t - r.info.t_arrival_us);
      S->bytes_done += (double)(r.L.info.in_bytes + r.L.info.out_bytes);
      S->last_done = t;
    } else {
      ++S->failed;
    }
  }
  S->in_use -= slot.charged;
  slot.charged = 0;
  slot.reqs.clear();
  slot.busy = false;
  slot.err = HP_OK;
}

// A launch failed after some of its steps were enqueued on the slot's stream: keep
// the slot busy until that work has finished (its staging buffer and arena are in
// use until then), and fail its requests only at that point.
void drain_failed_slot(hp_server_s* S, Slot& slot, int32_t status) {
  slot.err = status;
  if (S->fake) return;  // fake_done was set by the executor
  if (hipEventRecord(slot.ev, slot.st) != hipSuccess) {
    (void)hipStreamSynchronize(slot.st);  // cannot poll: wait here
    finish_slot(S, slot, status);
  }
}

void scheduler(hp_server_s* S) {
  if (!S->fake) (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    // completions
    bool any_busy = false;
    for (Slot& sl : S->slots) {
      if (!sl.busy) continue;
      if (S->fake) {
        if (S->now() >= sl.fake_done) finish_slot(S, sl, sl.err);
      } else {
        const hipError_t q = hipEventQuery(sl.ev);
        if (q == hipSuccess) finish_slot(S, sl, sl.err);
        else if (q != hipErrorNotReady) finish_slot(S, sl, HP_EDEVICE);
      }
      any_busy = any_busy || sl.busy;
    }
    S->cv_done.notify_all();
    if (S->stop.load() && S->pending.empty() && !any_busy) break;
    // form a batch when a slot is free
    Slot* free_slot = nullptr;
    for (Slot& sl : S->slots)
      if (!sl.busy) {
        free_slot = &sl;
        break;
      }
    bool launched = false;
    if (free_slot && !S->pending.empty()) {
      const double t = S->now();
      const Request& head = S->reqs[S->pending.front()];
      const bool full = (int64_t)S->pending.size() >= S->cfg.max_batch;
      const bool waited = t - head.info.t_arrival_us >= S->cfg.window_us;
      if (full || waited || !any_busy || S->stop.load()) {
        std::vector<Request*> rs;
        size_t charge = 0;
        Tally tally;
        for (auto it = S->pending.begin(); it != S->pending.end() && (int64_t)rs.size() < S->cfg.max_batch;) {
          Request& r = S->reqs[*it];
          // a request joins when its bytes fit the HBM budget and its descriptors and
          // workspace fit what is left of the slot arena; otherwise it stays pending
          if (S->in_use + charge + r.bytes <= S->cfg.hbm_budget && tally.total_with(r) <= free_slot->cap) {
            r.info.t_admit_us = t;
            rs.push_back(&r);
            charge += r.bytes;
            tally.add(r);
            it = S->pending.erase(it);
          } else {
            // bounded bypass: later requests may pass a request that does not fit
            // only a limited number of times, so large requests are not starved
            if (++r.bypassed > 64) break;
            ++it;
          }
        }
        if (!rs.empty()) {
          Slot& sl = *free_slot;
          sl.busy = true;
          sl.charged = charge;
          sl.batch_id = ++S->batches;
          sl.err = HP_OK;
          S->in_use += charge;
          S->max_in_use = std::max(S->max_in_use, S->in_use);
          sl.reqs.clear();
          for (Request* r : rs) {
            sl.reqs.push_back(r->id);
            r->info.t_launch_us = t;
            r->info.batch_id = sl.batch_id;
          }
          bool drain = false;
          lk.unlock();
          hp_status s = launch_slot(S, sl, rs, &drain);
          lk.lock();
          if (s != HP_OK) {
            const int32_t st = s == HP_ETOOBIG ? HP_ETOOBIG : HP_EDEVICE;
            if (drain) drain_failed_slot(S, sl, st);
            else finish_slot(S, sl, st);
          }
          launched = true;
        }
      }
    }
    if (!launched) {
      // nothing to launch now: sleep briefly (woken by submissions)
      S->cv_work.wait_for(lk, std::chrono::microseconds(any_busy ? 5 : 50));
    }
  }
}

}  // namespace

extern "C" hp_status hp_server_create(const hp_server_cfg* cfg, hp_server_t* out) {
  using namespace hp;
  if (!cfg || !out) return fail(HP_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->streams < 1 || cfg->streams > 16 || cfg->max_batch < 1 || cfg->max_batch > 65536 ||
      cfg->window_us < 0 || cfg->queue_cap < 1 || cfg->hbm_budget == 0 || cfg->slot_bytes < 4096 ||
      cfg->fail_every_nth_batch < 0 || cfg->fail_step < 0)
    return fail(HP_EINVAL, "bad server configuration");
  hp_server_s* S = new (std::nothrow) hp_server_s;
  if (!S) return fail(HP_ENOMEM, "host allocation failed");
  S->cfg = *cfg;
  S->fake = (cfg->flags & HP_SERVER_FAKE_DEVICE) != 0;
  S->fail_every = cfg->fail_every_nth_batch;
  S->t0 = Clock::now();
  S->slots.resize((size_t)cfg->streams);
  for (Slot& sl : S->slots) sl.cap = cfg->slot_bytes;
  if (!S->fake) {
    if (hipGetDevice(&S->device) != hipSuccess) {
      delete S;
      return fail(HP_EDEVICE, "no HIP device");
    }
    if (hipDeviceGetAttribute(&S->cus, hipDeviceAttributeMultiprocessorCount, S->device) != hipSuccess)
      S->cus = 256;
    for (Slot& sl : S->slots) {
      if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
          hipMalloc(&sl.d_arena, sl.cap) != hipSuccess || hipHostMalloc(&sl.h_stage, sl.cap) != hipSuccess) {
        for (Slot& q : S->slots) {
          if (q.st) (void)hipStreamDestroy(q.st);
          if (q.ev) (void)hipEventDestroy(q.ev);
          if (q.d_arena) (void)hipFree(q.d_arena);
          if (q.h_stage) (void)hipHostFree(q.h_stage);
        }
        delete S;
        return fail(HP_ENOMEM, "slot allocation failed");
      }
    }
  }
  if (!S->fake) {
    // load the kernels and learn their occupancy now, not on the first requests
    const size_t lds = (size_t)kBatchGroupWaves * kWaveLdsBytes;
    for (int fam = 0; fam < FAM_COUNT; ++fam)
      for (int chunk : {1, 4, 8}) {
        const bool ok = chunk == 1 || (chunk == 8) == (fam == FAM_BF16_4 || fam == FAM_BF16_8);
        if (!ok) continue;
        int o = batch_occupancy(fam, chunk, kBatchGroupWaves, lds);
        S->occ[occ_key(fam, chunk)] = o < 1 ? 1 : o;
      }
    if (warm_batch_kernels(S->slots[0].st) != HP_OK || hipStreamSynchronize(S->slots[0].st) != hipSuccess) {
      for (Slot& q : S->slots) {
        (void)hipStreamDestroy(q.st);
        (void)hipEventDestroy(q.ev);
        (void)hipFree(q.d_arena);
        (void)hipHostFree(q.h_stage);
      }
      delete S;
      return fail(HP_EDEVICE, "kernel warm-up failed");
    }
  }
  S->th = std::thread(scheduler, S);
  *out = S;
  return HP_OK;
}

extern "C" hp_status hp_server_now_us(hp_server_t S, double* t) {
  if (!S || !t) return hp::fail(HP_EINVAL, "null argument");
  *t = S->now();
  return HP_OK;
}

extern "C" hp_status hp_submit(hp_server_t S, const hp_nest* nest, const void* d_in, void* d_out,
                               double t_arrival_us, uint64_t* ticket) {
  using namespace hp;
  if (!S || !nest || !ticket) return fail(HP_EINVAL, "null argument");
  if (!S->fake && (!d_in || !d_out)) return fail(HP_EINVAL, "null device pointer");
  if (reinterpret_cast<uintptr_t>(d_in) & 15u) return fail(HP_EINVAL, "input not 16-byte aligned");
  if (S->stop.load()) return fail(HP_ESTATE, "server is shutting down");
  Request r;
  memset(&r.info, 0, sizeof r.info);
  hp_status s = plan_for_batch(nest, (uint32_t)(S->cfg.flags & HP_FLAG_OUT_F32), true,
                               kBatchWaves, &r.L);
  if (s != HP_OK) return s;
  const uintptr_t al = (r.L.info.out_dtype == HP_I64 || r.L.info.out_dtype == HP_F64) ? 7u : 3u;
  if (reinterpret_cast<uintptr_t>(d_out) & al) return fail(HP_EINVAL, "output misaligned");
  r.bytes = r.L.info.in_bytes + r.L.info.out_bytes + r.L.info.workspace_bytes;
  if (r.bytes > S->cfg.hbm_budget)
    return fail(HP_ETOOBIG, "request needs %zu bytes, budget is %zu", r.bytes, (size_t)S->cfg.hbm_budget);
  r.key = std::make_pair(family_of(r.L.dp), (int)r.L.dp.chunk);
  r.ntask = r.L.dp.grid;
  r.nfold = fold_task_count(r.L.dp);
  r.ws = align_up(r.L.info.workspace_bytes, 256);
  {
    const size_t arena = Tally().total_with(r);
    if (arena > S->cfg.slot_bytes)
      return fail(HP_ETOOBIG, "request needs %zu bytes of slot arena, slot_bytes is %zu", arena,
                  (size_t)S->cfg.slot_bytes);
  }
  r.nest = *nest;
  r.in = d_in;
  r.out = d_out;
  r.bypassed = 0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if ((int64_t)S->pending.size() >= S->cfg.queue_cap) return fail(HP_EAGAIN, "queue full");
    r.id = S->next_id++;
    r.info.status = HP_ENOTREADY;
    r.info.t_arrival_us = t_arrival_us >= 0 ? t_arrival_us : S->now();
    r.info.bytes = (int64_t)(r.L.info.in_bytes + r.L.info.out_bytes);
    if (S->first_arrival < 0 || r.info.t_arrival_us < S->first_arrival) S->first_arrival = r.info.t_arrival_us;
    *ticket = r.id;
    S->pending.push_back(r.id);
    S->reqs.emplace(r.id, r);
    ++S->submitted;
    S->max_queue = std::max(S->max_queue, (int64_t)S->pending.size());
  }
  S->cv_work.notify_one();
  return HP_OK;
}

extern "C" hp_status hp_poll(hp_server_t S, uint64_t ticket, hp_req_info* info) {
  if (!S) return hp::fail(HP_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return hp::fail(HP_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (info) *info = it->second.info;
  return it->second.info.status == HP_ENOTREADY ? HP_ENOTREADY : HP_OK;
}

extern "C" hp_status hp_wait(hp_server_t S, uint64_t ticket, hp_req_info* info) {
  if (!S) return hp::fail(HP_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return hp::fail(HP_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  S->cv_done.wait(lk, [&] { return it->second.info.status != HP_ENOTREADY; });
  if (info) *info = it->second.info;
  return HP_OK;
}

extern "C" hp_status hp_server_get_stats(hp_server_t S, hp_server_stats* st) {
  if (!S || !st) return hp::fail(HP_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  memset(st, 0, sizeof *st);
  st->submitted = S->submitted;
  st->completed = S->completed;
  st->failed = S->failed;
  st->batches = S->batches;
  st->pending = (int64_t)S->pending.size();
  st->max_queue = S->max_queue;
  st->max_in_use_bytes = (int64_t)S->max_in_use;
  st->in_use_bytes = (int64_t)S->in_use;
  st->bytes = S->bytes_done;
  std::vector<double> v(S->lat);
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto q = [&](double f) {
      size_t k = (size_t)std::ceil(f * (double)v.size());
      if (k < 1) k = 1;
      if (k > v.size()) k = v.size();
      return v[k - 1];
    };
    st->p50_us = q(0.50);
    st->p99_us = q(0.99);
    st->p999_us = q(0.999);
    st->max_us = v.back();
    double sum = 0;
    for (double x : v) sum += x;
    st->mean_us = sum / (double)v.size();
  }
  const double span = S->last_done - (S->first_arrival < 0 ? 0 : S->first_arrival);
  st->gbps = span > 0 ? S->bytes_done / (span * 1e3) : 0;
  return HP_OK;
}

extern "C" hp_status hp_server_forget(hp_server_t S, uint64_t ticket) {
  if (!S) return hp::fail(HP_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return hp::fail(HP_EINVAL, "unknown ticket");
  if (it->second.info.status == HP_ENOTREADY) return hp::fail(HP_ESTATE, "request still in flight");
  S->reqs.erase(it);
  return HP_OK;
}

extern "C" hp_status hp_server_destroy(hp_server_t S) {
  if (!S) return HP_OK;
  S->stop.store(true);
  S->cv_work.notify_all();
  if (S->th.joinable()) S->th.join();
  if (!S->fake) {
    for (Slot& q : S->slots) {
      if (q.st) (void)hipStreamSynchronize(q.st);
      if (q.st) (void)hipStreamDestroy(q.st);
      if (q.ev) (void)hipEventDestroy(q.ev);
      if (q.d_arena) (void)hipFree(q.d_arena);
      if (q.h_stage) (void)hipHostFree(q.h_stage);
    }
  }
  delete S;
  return HP_OK;
}

// Open-loop load generator: submit request i at server time t_arrival_us[i]
// (busy-waiting until then, never waiting for completions), from this thread.
extern "C" hp_status hp_server_replay(hp_server_t S, int64_t n, const hp_nest* nests, const void* const* d_in,
                                      void* const* d_out, const double* t_arrival_us, uint64_t* tickets) {
  if (!S || n < 0 || (n > 0 && (!nests || !d_in || !d_out || !t_arrival_us || !tickets)))
    return hp::fail(HP_EINVAL, "bad argument");
  for (int64_t i = 0; i < n; ++i) {
    while (S->now() < t_arrival_us[i]) {
    }
    hp_status s;
    do {
      s = hp_submit(S, &nests[i], d_in[i], d_out[i], t_arrival_us[i], &tickets[i]);
      if (s == HP_EAGAIN) std::this_thread::yield();
    } while (s == HP_EAGAIN);
    if (s != HP_OK) return s;
  }
  return HP_OK;
}
