// Persistent batched kernels: device code shared by the per-type batch units.
#pragma once

#include "hp_nest.h"

namespace hp {

// Persistent batched kernels: workers pop (nest, workgroup) tasks with atomic
// counters -- a dynamic schedule on the grid level.  The tasks are dealt, largest
// first, into kQueues queues with one counter each; workgroup b takes from queue
// b % kQueues, which is the XCD the hardware places it on, so the counters are
// contended by one XCD each instead of the whole chip.  Every run leaves the
// counters at zero for the next one, so a run can be replayed from a graph: the
// fold kernel that ends a run with grid-split nests clears them (the persistent
// launches before it on the stream have finished), and a batch without fold tasks
// clears them with a small kernel before each persistent launch.
constexpr int kQueues = 8;
constexpr int kCtrStride = 64;  // counters 256 bytes apart

struct BatchArgs {
  const DevPlan* plans;        // one plan per nest
  const int2* tasks;           // (nest, logical workgroup), queue by queue
  unsigned int* ctr;           // kQueues counters, kCtrStride apart
  const void* const* ins;      // per nest
  void* const* outs;           // per nest
  unsigned char* const* wss;   // per nest (grid-combine workspace, may be null)
  int qbeg[kQueues + 1];       // queue q holds tasks [qbeg[q], qbeg[q+1])
  int per_pop;                 // tasks taken per atomic
};

// Wave tasks: every wavefront of the workgroup is an independent worker running
// one-wave plans (no workgroup barrier), with its own small slice of LDS.  The next
// task index is taken before the current task runs, so the atomic's latency
// overlaps it.
constexpr int kWaveLdsBytes = 256;

template <class T, int C, int NS, int U, int KD, bool PF = true>
__device__ __forceinline__ void batch_run_waves(const BatchArgs& B, char* lds) {
  const int w = (int)(threadIdx.x >> 6);
  const int lane = (int)(threadIdx.x & 63);
  char* scratch = lds + w * kWaveLdsBytes;
  const int q = (int)(blockIdx.x % kQueues);
  const int qb = B.qbeg[q], qe = B.qbeg[q + 1];
  const int k = B.per_pop;
  // Workers of queue q: the waves of workgroups q, q + 8, ...  Worker r starts on
  // tasks [qb + r k, qb + r k + k) without touching the counter; the counter hands
  // out what follows the static part.
  const int nblk = ((int)gridDim.x - q + kQueues - 1) / kQueues;
  const int nwq = nblk * (int)(blockDim.x >> 6);
  const int r = (int)(blockIdx.x / kQueues) * (int)(blockDim.x >> 6) + w;
  const long long dyn0 = (long long)qb + (long long)nwq * k;
  unsigned int* ctr = B.ctr + q * kCtrStride;
  // The atomic's result is only needed after the current task, so the wave does not
  // wait for it here.
  auto pop = [&]() -> int {
    unsigned int v = 0;
    if (lane == 0) v = __hip_atomic_fetch_add(ctr, (unsigned int)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long t = dyn0 + (unsigned int)__builtin_amdgcn_readfirstlane((int)v);
    return t < qe ? (int)t : qe;
  };
  // Plans and task entries do not change while the kernel runs: read them through
  // the constant address space, so they arrive in scalar registers by scalar loads
  // and never queue behind the data stream's vector loads.
  typedef const __attribute__((address_space(4))) DevPlan CPlan;
  typedef const __attribute__((address_space(4))) int CInt;
  CPlan* plans = (CPlan*)(B.plans);
  CInt* tasks = (CInt*)(B.tasks);  // (nest, workgroup) pairs
  long long t0 = (long long)qb + (long long)r * k;
  int t = t0 < qe ? (int)t0 : qe;
  int t_end = t0 + k < qe ? (int)(t0 + k) : qe;
  while (t < t_end) {
    const int x = __builtin_amdgcn_readfirstlane(tasks[2 * (long long)t]);
    const int y = __builtin_amdgcn_readfirstlane(tasks[2 * (long long)t + 1]);
    int u = t + 1, u_end = t_end;
    if (u == t_end) {
      u = pop();
      u_end = u + k < qe ? u + k : qe;
    }
    wg_run<T, C, NS, U, KD, false, true, PF>(*(const DevPlan*)(plans + x),
                                             reinterpret_cast<const typename T::Raw*>(B.ins[x]), B.outs[x],
                                             B.wss[x], (uint32_t)y, scratch);
    group_sync(true);  // the scratch slice is reused by the next task
    t = u;
    t_end = u_end;
  }
}

// Kernel families.  Every nest of one persistent launch belongs to one family.
enum Family : int32_t {
  FAM_F32_4 = 0, FAM_F32_8, FAM_BF16_4, FAM_BF16_8, FAM_I32_FLAT, FAM_I32_SEG, FAM_I32_DEEP, FAM_COUNT
};
__host__ __device__ inline int family_of(const DevPlan& P) {
  if (P.dtype == HP_F32) return P.depth <= 4 ? FAM_F32_4 : FAM_F32_8;
  if (P.dtype == HP_BF16) return P.depth <= 4 ? FAM_BF16_4 : FAM_BF16_8;
  if (P.depth <= 4 && P.nseg <= 1) return FAM_I32_FLAT;
  if (P.depth <= 4 && P.nseg <= 3) return FAM_I32_SEG;
  return FAM_I32_DEEP;
}

// Launch a persistent batch of one family / chunk on `grid` workgroups of nw waves.
hp_status launch_batch(int family, int chunk, const BatchArgs& B, int grid, int nw, size_t lds, hipStream_t st);
// Launch every persistent kernel once with no tasks (and the counter and fold
// kernels), so that code objects are loaded before the first real batch.
hp_status warm_batch_kernels(hipStream_t st);
// Clear n counters (a kernel, so that it can sit in a captured graph).
hp_status launch_clear(unsigned int* ctr, int n, hipStream_t st);
// Deal n tasks, given largest first, round-robin into the queues that a grid of
// `grid` workgroups serves; writes them queue by queue to `out` and fills B->qbeg
// and B->per_pop.
void deal_tasks(const int2* ordered, int n, int grid, int2* out, BatchArgs* B);
// Counter words one batch launch uses (cleared before each launch).
constexpr int kCtrWords = kQueues * kCtrStride;
// Resident workgroups per CU for that kernel.
int batch_occupancy(int family, int chunk, int nw, size_t lds);

}  // namespace hp
