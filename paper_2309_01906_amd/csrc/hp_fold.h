// Grid combine of grid-split nests: the fold kernel's device code and its tasks.
#pragma once

#include <vector>

#include "hp_nest.h"

namespace hp {

// The grid combine.  Every workgroup of a grid-split nest writes its partial (one
// slot per workgroup digit of the reducing levels) and a second, small kernel folds
// the partials of each output once all workgroups are done.  The kernel boundary
// makes the partials visible across the XCDs' L2 caches; an in-kernel "last
// arriver" fold would need an agent-scope release and acquire per workgroup, which
// write back and invalidate the whole L2 of an XCD each time.
//
// The fold order is fixed by the partial count G alone, never by how many threads
// run it, so every launch form of a plan gives the same bits:
//   floats, G <= kSeqFold: one lane adds s then c of partials 0, 1, ..., G-1 into
//     an fp64 pair;
//   floats, G > kSeqFold: lane k adds partials k, k+64, ... the same way and the 64
//     pairs merge in a xor butterfly;
//   integers: the operators are exact, associative and commutative (ARG keeps the
//     smaller index on ties), so any order gives the same result.  One grid-spanning
//     segment: up to kSeqFold partials on one lane, more on a whole wave (lane k
//     takes partials k, k+64, ..., then a xor butterfly); several grid-spanning
//     segments are folded by one lane, digits in index order.
constexpr long long kSeqFold = 16;

// Partials are read kFoldBatch at a time, all loads issued before the first is
// used, so a fold of up to kFoldBatch partials waits for memory once rather than
// once per partial; the order of the additions is unchanged.
constexpr int kFoldBatch = 16;

__device__ __forceinline__ double fold_flt_seq(const char* part, long long G) {
  DPair a{0.0, 0.0};
  for (long long k0 = 0; k0 < G; k0 += kFoldBatch) {
    FAcc v[kFoldBatch];
#pragma unroll
    for (int u = 0; u < kFoldBatch; ++u)
      if (k0 + u < G) v[u] = FloatT<float>::get(part, k0 + u);
#pragma unroll
    for (int u = 0; u < kFoldBatch; ++u)
      if (k0 + u < G) {
        dpair_add(a, (double)v[u].s);
        dpair_add(a, (double)v[u].c);
      }
  }
  return a.s + a.c;
}

// whole wave; every lane returns the result
__device__ __forceinline__ double fold_flt_wave(const char* part, long long G, int lane) {
  DPair a{0.0, 0.0};
  constexpr int B = kFoldBatch / 2;
  for (long long k0 = lane; k0 < G; k0 += (long long)B * kWave) {
    FAcc v[B];
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (k0 + (long long)u * kWave < G) v[u] = FloatT<float>::get(part, k0 + (long long)u * kWave);
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (k0 + (long long)u * kWave < G) {
        dpair_add(a, (double)v[u].s);
        dpair_add(a, (double)v[u].c);
      }
  }
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    const DPair o{xor_move_d(a.s, 1 << b, lane), xor_move_d(a.c, 1 << b, lane)};
    a = dpair_merge(a, o);
  }
  return a.s + a.c;
}

__device__ __forceinline__ long long fold_int_uniform_seq(const char* part, long long G, int op) {
  IAcc a = IntT::identity(op);
  for (long long k0 = 0; k0 < G; k0 += kFoldBatch) {
    IAcc v[kFoldBatch];
#pragma unroll
    for (int u = 0; u < kFoldBatch; ++u)
      if (k0 + u < G) v[u] = IntT::get(part, k0 + u);
#pragma unroll
    for (int u = 0; u < kFoldBatch; ++u)
      if (k0 + u < G) a = IntT::merge(a, v[u], op);
  }
  return IntT::emit(a, op);
}

// whole wave, one grid-spanning segment; every lane returns the result
__device__ __forceinline__ long long fold_int_uniform_wave(const char* part, long long G, int op, int lane) {
  IAcc a = IntT::identity(op);
  constexpr int B = kFoldBatch / 2;
  for (long long k0 = lane; k0 < G; k0 += (long long)B * kWave) {
    IAcc v[B];
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (k0 + (long long)u * kWave < G) v[u] = IntT::get(part, k0 + (long long)u * kWave);
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (k0 + (long long)u * kWave < G) a = IntT::merge(a, v[u], op);
  }
#pragma unroll
  for (int b = 0; b < 6; ++b) a = IntT::merge(a, IntT::shfl(a, 1 << b, lane), op);
  return IntT::emit(a, op);
}

// Several segments span workgroups: fold segment gq's partials, then apply the
// outer segments' operators in nest order.  Outer segments are pure grid levels
// with one iteration per workgroup, so their iteration index is the workgroup digit.
template <int KD>
__device__ __forceinline__ long long fold_int_nested(const DevPlan& P, const char* part) {
  const int q = P.gq;
  IAcc A[KD];
  long long dg[KD];
#pragma unroll
  for (int j = 0; j < KD; ++j) {
    A[j] = IntT::identity(j <= q ? P.seg[j].op : 0);
    dg[j] = 0;
  }
  for (long long idx = 0; idx < P.gsplit; ++idx) {
    const IAcc pv = IntT::get(part, idx);
#pragma unroll
    for (int j = 0; j < KD; ++j)
      if (j == q) A[j] = IntT::merge(A[j], pv, P.seg[j].op);
    bool carry = true;
#pragma unroll
    for (int j = KD - 1; j >= 0; --j) {
      if (j <= q && carry) {
        const DevSeg& S = P.seg[j];
        if (dg[j] == (long long)S.gunits - 1) {
          if (j > 0) {
            const DevSeg& Sp = P.seg[j - 1];
            long long rem = dg[j - 1];
            bool valid = true;
            long long t_last = 0;
            for (int l = Sp.last; l >= Sp.first; --l) {
              const long long gfl = P.lv[l].gf;
              const long long t = rem % gfl;
              rem /= gfl;
              if (t >= P.lv[l].e) valid = false;
              if (l == Sp.last) t_last = t;
            }
            if (valid) IntT::add(A[j - 1], IntT::emit(A[j], S.op), t_last, Sp.op);
            A[j] = IntT::identity(S.op);
          }
          dg[j] = 0;
        } else {
          dg[j] += 1;
          carry = false;
        }
      }
    }
  }
  return IntT::emit(A[0], P.seg[0].op);
}

// A fold task covers outputs [o0, o0 + n) of one nest: with one lane per output
// (n <= 64) when every output folds on one lane, else one output per wave.
struct FoldTask {
  int nest;
  int o0;
  int n;
  int wave;  // 1: the whole wave folds output o0
};

// Whether outputs of plan P fold on one lane each.
__host__ __device__ inline bool fold_on_lane(const DevPlan& P) {
  const bool flt = P.dtype == HP_F32 || P.dtype == HP_BF16;
  return P.gsplit <= kSeqFold || (!flt && P.gmode != GCOMB_UNIFORM);
}

// One wave runs one fold task.
__device__ __forceinline__ void fold_task(const DevPlan& P, const FoldTask& t, void* out, const unsigned char* ws,
                                          int lane) {
  const bool flt = P.dtype == HP_F32 || P.dtype == HP_BF16;
  if (t.wave) {
    const long long o = t.o0;
    const char* part = reinterpret_cast<const char*>(ws) + o * P.gsplit * kSlotBytes;
    if (flt) {
      const double v = fold_flt_wave(part, P.gsplit, lane);
      if (lane == 0) store_flt(P, out, o, v);
    } else {
      const long long v = fold_int_uniform_wave(part, P.gsplit, P.seg[0].op, lane);
      if (lane == 0) store_int(P, out, o, v);
    }
    return;
  }
  if (lane >= t.n) return;
  const long long o = (long long)t.o0 + lane;
  const char* part = reinterpret_cast<const char*>(ws) + o * P.gsplit * kSlotBytes;
  if (flt) store_flt(P, out, o, fold_flt_seq(part, P.gsplit));
  else if (P.gmode == GCOMB_UNIFORM) store_int(P, out, o, fold_int_uniform_seq(part, P.gsplit, P.seg[0].op));
  else store_int(P, out, o, fold_int_nested<kMaxDepth>(P, part));
}

// Host side: how many fold tasks fold_tasks_of appends for plan P.
inline long long fold_task_count(const DevPlan& P) {
  if (P.gmode == GCOMB_NONE || P.gsplit <= 1) return 0;
  return fold_on_lane(P) ? (P.n_out + kWave - 1) / kWave : P.n_out;
}

// Host side: the fold tasks of one plan (appended to v).
inline void fold_tasks_of(const DevPlan& P, int nest, std::vector<FoldTask>& v) {
  if (P.gmode == GCOMB_NONE || P.gsplit <= 1) return;
  if (fold_on_lane(P)) {
    for (long long o = 0; o < P.n_out; o += kWave) {
      const long long n = P.n_out - o < kWave ? P.n_out - o : kWave;
      v.push_back(FoldTask{nest, (int)o, (int)n, 0});
    }
  } else {
    for (long long o = 0; o < P.n_out; ++o) v.push_back(FoldTask{nest, (int)o, 1, 1});
  }
}

// Fold the grid-split outputs: n fold tasks over a pointer table of nests.  When
// ctr is given, the kernel also sets its n_ctr words to zero (the task counters of
// the persistent launches that ran before it, ready for the next run).
hp_status launch_fold(const DevPlan* plans, const FoldTask* tasks, int n, void* const* outs,
                      unsigned char* const* wss, hipStream_t st, unsigned int* ctr = nullptr, int n_ctr = 0);
// The same for a single plan.
hp_status launch_fold_one(const DevPlan* plan, const FoldTask* tasks, int n, void* out, const unsigned char* ws,
                          hipStream_t st);

}  // namespace hp
