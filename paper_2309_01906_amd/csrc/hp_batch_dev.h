// Persistent batched kernels: device code shared by the per-type batch units.
#pragma once

#include "hp_nest.h"

namespace hp {

// Persistent batched kernels: workers pop (nest, workgroup) tasks with atomic
// counters -- a dynamic schedule on the grid level.  The tasks are dealt, largest
// first, each to the queue with the least estimated work so far, into kQueues
// queues with one counter each; workgroup b takes from queue
// b % kQueues, which sits on one XCD (workgroups are dealt round-robin to the 8
// XCDs).  Atomics on one address are serialised in the L2 (some 20 ns apiece), so
// a batch of tens of thousands of small tasks needs many counters: 64 queues, 8
// per XCD, each shared by an eighth of an XCD's workers.  Every run leaves the
// counters at zero for the next one, so a run can be replayed from a graph: the
// fold kernel that ends a run with grid-split nests clears them (the persistent
// launches before it on the stream have finished), and a batch without fold tasks
// clears them with a small kernel before each persistent launch.
constexpr int kQueues = 64;
constexpr int kCtrStride = 64;  // counters 256 bytes apart

// Compact form of the most common batched plan -- one float SUM over each output's
// contiguous block, the block on lanes of one wave (16-byte chunks, whole strips,
// possibly the aligned interior of a flat block), the outputs on the grid and on
// the remaining lanes -- so a task reads one 64-byte line (the nest's input and
// output pointers included, written when the batch's pointers are set) instead of
// the plan's fields and the pointer tables.  The arithmetic, and its order, is the
// general path's: the same chunk folds, the same flat-block rest, the same
// butterfly, so the bits are those of the nest's own plan run alone.
struct alignas(64) SimpleDesc {
  const void* in;
  void* out;
  int32_t block;     // elements between consecutive outputs' blocks
  int32_t flat_b;    // 0, or the flat block length (the interior is flat_e elements)
  int32_t flat_e;
  int32_t e0;        // outputs
  int32_t g0;        // grid units of the output level
  int32_t v0;        // output lane groups per wave
  int32_t v1;        // lanes per output
  int32_t strips1;   // interior chunks per lane
  int32_t strips0;   // output strips
  uint32_t bits;     // v0sh (bits 0-7: lane bit of the output level), fp64 output (bit 8),
                     // butterfly steps that may take the uniform form (bits 16-21)
};

struct BatchArgs {
  const DevPlan* plans;        // one plan per nest
  const int2* tasks;           // (nest, logical workgroup), queue by queue
  unsigned int* ctr;           // kQueues counters, kCtrStride apart
  const void* const* ins;      // per nest
  void* const* outs;           // per nest
  unsigned char* const* wss;   // per nest (grid-combine workspace, may be null)
  int qbeg[kQueues + 1];       // queue q holds tasks [qbeg[q], qbeg[q+1])
  int per_pop;                 // tasks taken per atomic
  const SimpleDesc* simple;    // per nest; read for tasks marked kSimpleTask (may be null)
};
constexpr int kSimpleTask = (int)0x80000000;  // task's workgroup field: the nest has a SimpleDesc

// One task of a SimpleDesc nest: output strip s0 of this task's outputs, each lane
// a unit of the output level (bits >= v0sh) and of the block (bits < v0sh).  The
// first elements of a flat block's rest are loaded before the interior, so their
// round trip to memory overlaps the stream; they are added after it, as the
// general path adds them.
constexpr int kRestVecPre = 2, kRestOnePre = 2;

template <class T, int C>
__device__ __forceinline__ void simple_task(const SimpleDesc& D, uint32_t g, int lane) {
  using V = typename Chunk<typename T::Raw, C>::V;
  using Raw = typename T::Raw;
  const Raw* __restrict__ in = reinterpret_cast<const Raw*>(D.in);
  const int v1 = D.v1;
  const int v0sh = (int)(D.bits & 0xFFu);
  const int uv1 = lane & (v1 - 1);
  const int uv0 = (lane >> v0sh) & (D.v0 - 1);
  const bool real = lane < D.v0 * v1;  // lanes beyond both levels' units are idle
  const long long span1 = (long long)v1 * C;
  DevSeg S;
  S.vmask = (uint32_t)(v1 - 1);
  S.ufast = (D.bits >> 16) & 0x3Fu;
  S.op = HP_OP_SUM;
  for (int s0 = 0; s0 < D.strips0; ++s0) {
    const long long o = ((long long)g * D.v0 + uv0) + (long long)s0 * D.g0 * D.v0;
    const bool valid = o < D.e0;
    const long long sb = (valid ? o : 0) * D.block;  // an invalid lane reads output 0's block
    const long long h = D.flat_b ? ((-sb) & (long long)(C - 1)) : 0;
    const Raw* __restrict__ p = in + sb + h + (long long)uv1 * C;
    // the rest of a flat block: whole vectors of its tail, then single elements
    long long tail = 0, nv = 0, ns = 0, tv = 0;
    V rv[kRestVecPre];
    Raw r1[kRestOnePre];
    if (D.flat_b) {
      tail = sb + h + D.flat_e;
      const long long tl = D.flat_b - h - D.flat_e;
      nv = tl / C;
      ns = h + (tl - nv * C);
      tv = tail + nv * C;
#pragma unroll
      for (int i = 0; i < kRestVecPre; ++i) {
        const long long j = uv1 + (long long)i * v1;
        if (j < nv) rv[i] = load_chunk<V>(in + tail + j * C);
      }
#pragma unroll
      for (int i = 0; i < kRestOnePre; ++i) {
        const long long k = uv1 + (long long)i * v1;
        if (k < ns) r1[i] = in[k < h ? sb + k : tv + (k - h)];
      }
    }
    FAcc a = T::identity(0);
    // the interior: strips1 chunks, four loads in flight
    int f = 0;
    for (; f + 4 <= D.strips1; f += 4) {
      V x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = load_chunk<V>(p + (long long)(f + u) * span1);
#pragma unroll
      for (int u = 0; u < 4; ++u) AddChunk<T, C, HP_OP_SUM>::run(a, x[u], 0, true);
    }
    for (; f < D.strips1; ++f) AddChunk<T, C, HP_OP_SUM>::run(a, load_chunk<V>(p + (long long)f * span1), 0, true);
    if (D.flat_b) {  // in flat_rest's order
#pragma unroll
      for (int i = 0; i < kRestVecPre; ++i)
        if (uv1 + (long long)i * v1 < nv) AddChunk<T, C, HP_OP_SUM>::run(a, rv[i], 0, true);
      for (long long j = uv1 + (long long)kRestVecPre * v1; j < nv; j += v1)
        RestVec<T, C>::run(a, in + tail + j * C, HP_OP_SUM);
#pragma unroll
      for (int i = 0; i < kRestOnePre; ++i)
        if (uv1 + (long long)i * v1 < ns) RestAdd<T>::run(a, r1[i], HP_OP_SUM);
      for (long long k = uv1 + (long long)kRestOnePre * v1; k < ns; k += v1)
        RestAdd<T>::run(a, in[k < h ? sb + k : tv + (k - h)], HP_OP_SUM);
    }
    a = lane_combine<T>(a, S, lane);
    if (valid && real && uv1 == 0) {
      const double v = (double)a.s + (double)a.c;
      if (D.bits & 0x100u) reinterpret_cast<double*>(D.out)[o] = v;
      else reinterpret_cast<float*>(D.out)[o] = (float)v;
    }
  }
}

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
  typedef const __attribute__((address_space(4))) SimpleDesc CSimple;
  while (t < t_end) {
    const int x = __builtin_amdgcn_readfirstlane(tasks[2 * (long long)t]);
    const int y = __builtin_amdgcn_readfirstlane(tasks[2 * (long long)t + 1]);
    int u = t + 1, u_end = t_end;
    if (u == t_end) {
      u = pop();
      u_end = u + k < qe ? u + k : qe;
    }
    if constexpr (T::kFloat && KD == 4) {
      if (y & kSimpleTask) {
        simple_task<T, C>(*(const SimpleDesc*)((CSimple*)B.simple + x), (uint32_t)(y & ~kSimpleTask), lane);
        t = u;
        t_end = u_end;
        continue;
      }
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
// Deal n tasks, given largest first with their estimated costs (weight[j], e.g.
// input bytes plus a per-task overhead), into the queues that a grid of `grid`
// workgroups serves: each task goes to the queue with the least cost so far
// (longest-processing-time-first), so the queues end together; a queue keeps its
// tasks largest first.  Writes them queue by queue to `out` and fills B->qbeg and
// B->per_pop.
void deal_tasks(const int2* ordered, const double* weight, int n, int grid, int2* out, BatchArgs* B);
// estimated cost of one task of `bytes` input bytes, in bytes: the data plus the
// fixed latency of starting a task (descriptor, first loads, combine, write)
inline double task_cost(double bytes) { return bytes + 4096.0; }
// Counter words one batch launch uses (cleared before each launch).
constexpr int kCtrWords = kQueues * kCtrStride;
// Resident workgroups per CU for that kernel.
int batch_occupancy(int family, int chunk, int nw, size_t lds);

}  // namespace hp
