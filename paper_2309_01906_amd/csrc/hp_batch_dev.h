// Persistent batched kernels: device code shared by the per-type batch units.
#pragma once

#include "hp_nest.h"

namespace hp {

// Persistent batched kernels: workers pop (nest, workgroup) tasks with atomic
// counters -- a dynamic schedule on the grid level.  The tasks are dealt, largest
// first, into kQueues queues with one counter each; workgroup b takes from queue
// b % kQueues, which is the XCD the hardware places it on, so the counters are
// contended by one XCD each instead of the whole chip.  The counters are cleared by
// a separate small kernel before every run, so a run can be replayed from a graph.
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
// one-wave plans (no workgroup barrier), with its own slice of LDS.  The task's
// plan is first copied into that slice, so the kernel reads it from LDS instead of
// with vector loads that would queue behind the data stream.  The next task index
// is taken before the current task runs, so the atomic's latency overlaps it.
constexpr int kPlanLdsBytes = (int)((sizeof(DevPlan) + 255) / 256 * 256);
constexpr int kWaveLdsBytes = kPlanLdsBytes + 256;
static_assert(sizeof(DevPlan) % 16 == 0, "plans are copied in 16-byte words");

template <class T, int C, int NS, int U, int KD, bool PF = true>
__device__ __forceinline__ void batch_run_waves(const BatchArgs& B, char* lds) {
  const int w = (int)(threadIdx.x >> 6);
  const int lane = (int)(threadIdx.x & 63);
  char* mine = lds + w * kWaveLdsBytes;
  DevPlan* plan = reinterpret_cast<DevPlan*>(mine);
  char* scratch = mine + kPlanLdsBytes;
  const int q = (int)(blockIdx.x % kQueues);
  const int qb = B.qbeg[q], qe = B.qbeg[q + 1];
  const int k = B.per_pop;
  unsigned int* ctr = B.ctr + q * kCtrStride;
  auto pop = [&]() -> int {
    unsigned int v = 0;
    if (lane == 0) v = __hip_atomic_fetch_add(ctr, (unsigned int)k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return qb + __builtin_amdgcn_readfirstlane((int)v);
  };
  int first = pop();
  while (first < qe) {
    const int next = pop();
    const int last = first + k < qe ? first + k : qe;
    for (int t = first; t < last; ++t) {
      const int2 te = B.tasks[t];
      const int x = __builtin_amdgcn_readfirstlane(te.x);
      const int y = __builtin_amdgcn_readfirstlane(te.y);
      const i32x4* src = reinterpret_cast<const i32x4*>(B.plans + x);
      i32x4* dst = reinterpret_cast<i32x4*>(plan);
      for (int i = lane; i < (int)(sizeof(DevPlan) / 16); i += 64) dst[i] = src[i];
      group_sync(true);
      wg_run<T, C, NS, U, KD, false, true, PF>(*plan, reinterpret_cast<const typename T::Raw*>(B.ins[x]),
                                               B.outs[x], B.wss[x], (uint32_t)y, scratch);
      group_sync(true);  // the plan slice is rewritten by the next task
    }
    first = next;
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
