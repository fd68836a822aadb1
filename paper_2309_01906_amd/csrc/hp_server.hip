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
};

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
// launch one persistent kernel per (family, chunk) group.
hp_status launch_slot(hp_server_s* S, Slot& slot, std::vector<Request*>& rs) {
  using namespace hp;
  const int64_t n = (int64_t)rs.size();
  size_t off = 0;
  const size_t plans_off = off;
  off = align_up(off + sizeof(DevPlan) * (size_t)n, 256);
  const size_t ptr_off = off;
  off = align_up(off + 3 * sizeof(void*) * (size_t)n, 256);
  // groups
  std::vector<std::pair<int, int>> keys;
  std::vector<std::vector<int64_t>> members;
  for (int64_t i = 0; i < n; ++i) {
    std::pair<int, int> k(family_of(rs[(size_t)i]->L.dp), rs[(size_t)i]->L.dp.chunk);
    size_t g = 0;
    while (g < keys.size() && keys[g] != k) ++g;
    if (g == keys.size()) {
      keys.push_back(k);
      members.emplace_back();
    }
    members[g].push_back(i);
  }
  std::vector<size_t> task_off(keys.size()), ctr_off(keys.size());
  std::vector<long long> ntask(keys.size(), 0);
  for (size_t g = 0; g < keys.size(); ++g) {
    for (int64_t i : members[g]) ntask[g] += rs[(size_t)i]->L.dp.grid;
    task_off[g] = off;
    off = align_up(off + (size_t)ntask[g] * sizeof(int2), 256);
    ctr_off[g] = off;
    off = align_up(off + kCtrWords * sizeof(unsigned int), 256);
  }
  std::vector<FoldTask> folds;
  for (int64_t i = 0; i < n; ++i) fold_tasks_of(rs[(size_t)i]->L.dp, (int)i, folds);
  const size_t fold_off = off;
  off = align_up(off + folds.size() * sizeof(FoldTask), 256);
  const size_t ws_begin = off;
  std::vector<size_t> ws_off((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const size_t wb = rs[(size_t)i]->L.info.workspace_bytes;
    if (wb) {
      ws_off[(size_t)i] = off;
      off = align_up(off + wb, 256);
    }
  }
  if (off > slot.cap) return fail(HP_ETOOBIG, "batch needs %zu bytes of slot arena, capacity %zu", off, slot.cap);
  unsigned char* h = slot.h_stage;
  unsigned char* d = slot.d_arena;
  DevPlan* hp_ = reinterpret_cast<DevPlan*>(h + plans_off);
  const void** hin = reinterpret_cast<const void**>(h + ptr_off);
  void** hout = reinterpret_cast<void**>(h + ptr_off) + n;
  unsigned char** hws = reinterpret_cast<unsigned char**>(h + ptr_off) + 2 * n;
  for (int64_t i = 0; i < n; ++i) {
    hp_[i] = rs[(size_t)i]->L.dp;
    hin[i] = rs[(size_t)i]->in;
    hout[i] = rs[(size_t)i]->out;
    hws[i] = ws_off[(size_t)i] ? d + ws_off[(size_t)i] : nullptr;
  }
  const size_t lds = (size_t)kBatchGroupWaves * kWaveLdsBytes;
  std::vector<BatchArgs> args(keys.size());
  std::vector<int> grid(keys.size());
  for (size_t g = 0; g < keys.size(); ++g) {
    std::vector<int64_t>& mem = members[g];
    std::stable_sort(mem.begin(), mem.end(), [&](int64_t a, int64_t c) {
      const double wa = (double)rs[(size_t)a]->L.info.in_bytes / (double)rs[(size_t)a]->L.dp.grid;
      const double wc = (double)rs[(size_t)c]->L.info.in_bytes / (double)rs[(size_t)c]->L.dp.grid;
      return wa > wc;
    });
    std::vector<int2> ordered((size_t)ntask[g]);
    long long k = 0;
    for (int64_t i : mem)
      for (long long w = 0; w < rs[(size_t)i]->L.dp.grid; ++w) ordered[(size_t)k++] = make_int2((int)i, (int)w);
    const int key = occ_key(keys[g].first, keys[g].second);
    auto it = S->occ.find(key);
    int o;
    if (it == S->occ.end()) {
      o = batch_occupancy(keys[g].first, keys[g].second, kBatchGroupWaves, lds);
      if (o < 1) o = 1;
      S->occ[key] = o;
    } else {
      o = it->second;
    }
    long long gr = (long long)S->cus * o;
    const long long need = (ntask[g] + kBatchGroupWaves - 1) / kBatchGroupWaves;
    if (gr > need) gr = need;
    grid[g] = (int)gr;
    deal_tasks(ordered.data(), (int)ntask[g], grid[g], reinterpret_cast<int2*>(h + task_off[g]), &args[g]);
    memset(h + ctr_off[g], 0, kCtrWords * sizeof(unsigned int));
  }
  if (!folds.empty()) memcpy(h + fold_off, folds.data(), folds.size() * sizeof(FoldTask));
  // upload the descriptors; the workspaces need no clearing (every partial is written
  // before the fold kernel reads it)
  if (hipMemcpyAsync(d, h, ws_begin, hipMemcpyHostToDevice, slot.st) != hipSuccess)
    return fail(HP_EDEVICE, "batch upload failed");
  for (size_t g = 0; g < keys.size(); ++g) {
    BatchArgs A = args[g];
    A.plans = reinterpret_cast<const DevPlan*>(d + plans_off);
    A.tasks = reinterpret_cast<const int2*>(d + task_off[g]);
    A.ctr = reinterpret_cast<unsigned int*>(d + ctr_off[g]);
    A.ins = reinterpret_cast<const void* const*>(d + ptr_off);
    A.outs = reinterpret_cast<void* const*>(d + ptr_off) + n;
    A.wss = reinterpret_cast<unsigned char* const*>(d + ptr_off) + 2 * n;
    hp_status s = launch_batch(keys[g].first, keys[g].second, A, grid[g], kBatchGroupWaves, lds, slot.st);
    if (s != HP_OK) return s;
  }
  if (!folds.empty()) {
    hp_status s = launch_fold(reinterpret_cast<const DevPlan*>(d + plans_off),
                              reinterpret_cast<const FoldTask*>(d + fold_off), (int)folds.size(),
                              reinterpret_cast<void* const*>(d + ptr_off) + n,
                              reinterpret_cast<unsigned char* const*>(d + ptr_off) + 2 * n, slot.st);
    if (s != HP_OK) return s;
  }
  if (hipEventRecord(slot.ev, slot.st) != hipSuccess) return fail(HP_EDEVICE, "event record failed");
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
        if (S->now() >= sl.fake_done) finish_slot(S, sl, HP_OK);
      } else {
        const hipError_t q = hipEventQuery(sl.ev);
        if (q == hipSuccess) finish_slot(S, sl, HP_OK);
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
        for (auto it = S->pending.begin(); it != S->pending.end() && (int64_t)rs.size() < S->cfg.max_batch;) {
          Request& r = S->reqs[*it];
          if (S->in_use + charge + r.bytes <= S->cfg.hbm_budget) {
            r.info.t_admit_us = t;
            rs.push_back(&r);
            charge += r.bytes;
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
          S->in_use += charge;
          S->max_in_use = std::max(S->max_in_use, S->in_use);
          sl.reqs.clear();
          for (Request* r : rs) {
            sl.reqs.push_back(r->id);
            r->info.t_launch_us = t;
            r->info.batch_id = sl.batch_id;
          }
          hp_status s = HP_OK;
          if (S->fail_every > 0 && sl.batch_id % S->fail_every == 0) {
            s = HP_EDEVICE;  // test hook: this batch fails before launch
          } else if (S->fake) {
            double work = 0;
            for (Request* r : rs) work += (double)r->L.info.in_bytes;
            sl.fake_done = t + 5.0 + work / 4.0e3;  // 4 GB/s-ish pretend device
          } else {
            lk.unlock();
            s = launch_slot(S, sl, rs);
            lk.lock();
          }
          if (s != HP_OK) finish_slot(S, sl, s == HP_ETOOBIG ? HP_ETOOBIG : HP_EDEVICE);
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
      cfg->window_us < 0 || cfg->queue_cap < 1 || cfg->hbm_budget == 0 || cfg->slot_bytes < 4096)
    return fail(HP_EINVAL, "bad server configuration");
  hp_server_s* S = new (std::nothrow) hp_server_s;
  if (!S) return fail(HP_ENOMEM, "host allocation failed");
  S->cfg = *cfg;
  S->fake = (cfg->flags & HP_SERVER_FAKE_DEVICE) != 0;
  S->fail_every = cfg->fail_every_nth_batch;
  S->t0 = Clock::now();
  S->slots.resize((size_t)cfg->streams);
  if (!S->fake) {
    if (hipGetDevice(&S->device) != hipSuccess) {
      delete S;
      return fail(HP_EDEVICE, "no HIP device");
    }
    if (hipDeviceGetAttribute(&S->cus, hipDeviceAttributeMultiprocessorCount, S->device) != hipSuccess)
      S->cus = 256;
    for (Slot& sl : S->slots) {
      sl.cap = cfg->slot_bytes;
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
