// Nested multi-level reduction: device templates for gfx950 (CDNA4, wave64).
//
// One kernel template executes any planned nest.  Every loop level owns a slice of
// the hardware: a factor of the workgroup index (G), of the wave index (W) and of
// the lane index (V); the rest of its iterations are serial strips (L).  Inside a
// workgroup the reducing levels are walked in two loops whose counters are the same
// for every thread (so they live in scalar registers):
//   - the innermost segment (a run of levels with one operator that can be folded
//     as a single reduction) is a stream: U chunks are loaded back to back, each
//     one 16-byte load per lane at thread_base + strip_offset, then folded into the
//     lane's private partial (section 3.6's private partial sum);
//   - the levels outside it form an odometer; each time a segment's last strip is
//     done its partials are combined and fed to the enclosing level's operator.
// Combines follow the paper's recursive reduction (section 2: every level collects
// its siblings' results through its cheapest means):
//   lanes       xor butterfly: DPP quad_perm / mirrors / row shifts and gfx950's
//               permlane16 / permlane32 swaps (hp_lanes.h; section 3.7's shuffle; a
//               wave64 runs in lockstep, so no masks or warp syncs are needed);
//   waves       one LDS slot per wave, s_barrier, every wave folds its group's slots
//               in wave order (section 3.7's fallback through memory one level up);
//   workgroups  a partial per workgroup in global memory; a second, small kernel
//               folds each output's partials in index order (the grid has no
//               barrier across its units, sections 1 and 3.2).
// Float sums keep an fp32 (sum, error) pair per lane, extended by TwoSum for every
// element, and use fp64 only when partials of several workgroups are folded and for
// the output.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "hp_internal.h"
#include "hp_lanes.h"

namespace hp {

// clang vector types (nontemporal loads need native vectors, not HIP's wrappers)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// cross-lane moves: the value held by lane (lane ^ mask), mask in {1,2,4,8,16,32}

__device__ __forceinline__ int xor_move(int v, int mask, int lane) {
  if (mask == 1) return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  if (mask == 2) return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  if (mask == 4) {
    const int dn = __builtin_amdgcn_update_dpp(v, v, 0x114, 0xF, 0xF, false);  // row_shr:4, from lane-4
    const int up = __builtin_amdgcn_update_dpp(v, v, 0x104, 0xF, 0xF, false);  // row_shl:4, from lane+4
    return (lane & 4) ? dn : up;
  }
  if (mask == 8) {
    const int dn = __builtin_amdgcn_update_dpp(v, v, 0x118, 0xF, 0xF, false);  // row_shr:8
    const int up = __builtin_amdgcn_update_dpp(v, v, 0x108, 0xF, 0xF, false);  // row_shl:8
    return (lane & 8) ? dn : up;
  }
  if (mask == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);  // bitmask mode: and 0x1F, xor 0x10
  return __builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, v);
}

__device__ __forceinline__ float xor_move_f(float v, int mask, int lane) {
  return __int_as_float(xor_move(__float_as_int(v), mask, lane));
}
__device__ __forceinline__ long long xor_move_l(long long v, int mask, int lane) {
  const int lo = xor_move((int)(uint32_t)(unsigned long long)v, mask, lane);
  const int hi = xor_move((int)(uint32_t)((unsigned long long)v >> 32), mask, lane);
  return (long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double xor_move_d(double v, int mask, int lane) {
  return __longlong_as_double(xor_move_l(__double_as_longlong(v), mask, lane));
}

// Error-free sum (Knuth's TwoSum): s + e == a + b exactly, s = fl(a + b).
template <class F>
__device__ __forceinline__ void two_sum(F a, F b, F& s, F& e) {
  s = a + b;
  const F bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// n / d by the plan's FastDiv of d (plain division when it has none)
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f, uint32_t d) {
  return f.m ? (uint32_t)(((unsigned long long)n * f.m) >> f.s) : n / d;
}
// the digit of a level in the workgroup's G coordinate: (g / gdiv) % gf
__device__ __forceinline__ uint32_t g_digit(uint32_t g, const DevLevel& L) {
  const uint32_t q = fdiv(g, L.fd_gdiv, L.gdiv);
  return q - fdiv(q, L.fd_gf, L.gf) * L.gf;
}

// ---------------------------------------------------------------------------
// carriers

struct FAcc {
  float s, c;  // value = s + c; c collects the exact rounding errors of s
};
struct IAcc {
  long long v;
  int i;  // ARG levels: iteration index of v
  int pad;
};

template <class RawT>
struct FloatT {
  using Raw = RawT;
  using Acc = FAcc;
  static constexpr bool kFloat = true;
  static constexpr bool kKey = false;
  __device__ static __forceinline__ Acc identity(int) { return Acc{0.f, 0.f}; }
  // TwoSum per element, its exact error added to c.  (Kahan's four-operation step
  // rounds x + c before it adds, which loses about u |x| per element: on a 2^20-element
  // sum of N(0,1) values that is 2e-6 relative to the result, above the 1e-6 rule.)
  __device__ static __forceinline__ void add(Acc& a, float x, long long, int) {
    float s, e;
    two_sum(a.s, x, s, e);
    a.s = s;
    a.c += e;
  }
  // symmetric in (a, b), so both partners of a butterfly step get identical bits
  __device__ static __forceinline__ Acc merge(Acc a, Acc b, int) {
    float s, e;
    two_sum(a.s, b.s, s, e);
    const float c = (a.c + b.c) + e;
    const float s2 = s + c;
    return Acc{s2, c - (s2 - s)};
  }
  __device__ static __forceinline__ Acc shfl(Acc a, int mask, int lane) {
    return Acc{xor_move_f(a.s, mask, lane), xor_move_f(a.c, mask, lane)};
  }
  __device__ static __forceinline__ void put(char* base, long long slot, Acc a) {
    f32x2 v;
    v.x = a.s;
    v.y = a.c;
    *reinterpret_cast<f32x2*>(base + slot * kSlotBytes) = v;
  }
  __device__ static __forceinline__ Acc get(const char* base, long long slot) {
    const f32x2 v = *reinterpret_cast<const f32x2*>(base + slot * kSlotBytes);
    return Acc{v.x, v.y};
  }
};

struct IntT {
  using Raw = int32_t;
  using Acc = IAcc;
  static constexpr bool kFloat = false;
  static constexpr bool kKey = false;
  __device__ static __forceinline__ Acc identity(int op) {
    switch (op) {
      case HP_OP_MIN: return Acc{0x7FFFFFFFFFFFFFFFll, 0, 0};
      case HP_OP_MAX: return Acc{(long long)0x8000000000000000ull, 0, 0};
      case HP_OP_ARGMIN: return Acc{0x7FFFFFFFFFFFFFFFll, 0x7FFFFFFF, 0};
      case HP_OP_ARGMAX: return Acc{(long long)0x8000000000000000ull, 0x7FFFFFFF, 0};
      default: return Acc{0, 0, 0};
    }
  }
  // Merge carrier b into a.  Written without branches on op: op is uniform, and in
  // the combine code a switch per call multiplies the scalar work and the code size;
  // with a constant op (the element folds) the selects fold away.
  // ARG: lexicographic (value, index), so ties keep the smaller index.
  __device__ static __forceinline__ Acc merge(Acc a, Acc b, int op) {
    const bool sum = op == HP_OP_SUM;
    const bool keep = op == HP_OP_NONE;
    const bool minlike = op == HP_OP_MIN || op == HP_OP_ARGMIN;
    const bool arg = op == HP_OP_ARGMIN || op == HP_OP_ARGMAX;
    const bool lt = b.v < a.v, gt = b.v > a.v;
    const bool take = !sum && !keep && ((minlike ? lt : gt) || (arg && b.v == a.v && b.i < a.i));
    Acc r;
    r.v = sum ? (long long)((unsigned long long)a.v + (unsigned long long)b.v) : (take ? b.v : a.v);
    r.i = take ? b.i : a.i;
    r.pad = 0;
    return r;
  }
  // fold child value x with iteration index t into the carrier
  __device__ static __forceinline__ void add(Acc& a, long long x, long long t, int op) {
    a = merge(a, Acc{x, (int)t, 0}, op);
  }
  __device__ static __forceinline__ long long emit(Acc a, int op) {
    return (op == HP_OP_ARGMIN || op == HP_OP_ARGMAX) ? (long long)a.i : a.v;
  }
  __device__ static __forceinline__ Acc shfl(Acc a, int mask, int lane) {
    Acc r;
    r.v = xor_move_l(a.v, mask, lane);
    r.i = xor_move(a.i, mask, lane);
    r.pad = 0;
    return r;
  }
  __device__ static __forceinline__ void put(char* base, long long slot, Acc a) {
    long long* q = reinterpret_cast<long long*>(base + slot * kSlotBytes);
    q[0] = a.v;
    q[1] = (long long)(uint32_t)a.i;
  }
  __device__ static __forceinline__ Acc get(const char* base, long long slot) {
    const long long* q = reinterpret_cast<const long long*>(base + slot * kSlotBytes);
    return Acc{q[0], (int)q[1], 0};
  }
};

// Integer carrier as one 64-bit key, for plans in which every ARG level sees 32-bit
// child values (the input, MIN / MAX of them, or an ARG level's index):
//   SUM        the int64 sum (wrapping);
//   MIN / MAX  the value;
//   ARGMIN     value << 32 | t;  ARGMAX  value << 32 | (2^32 - 1 - t).
// A signed 64-bit comparison of two ARG keys is the lexicographic order of (value,
// index) with ties to the smaller index, so every merge is a 64-bit add, min or max
// and butterfly steps move two words where the (value, index) pair moves three.
// Grid partials are written in IntT's (value, index) form, which the fold reads.
struct IntK {
  using Raw = int32_t;
  using Acc = long long;
  static constexpr bool kFloat = false;
  static constexpr bool kKey = true;
  __device__ static __forceinline__ bool minlike(int op) { return op == HP_OP_MIN || op == HP_OP_ARGMIN; }
  __device__ static __forceinline__ bool arg(int op) { return op == HP_OP_ARGMIN || op == HP_OP_ARGMAX; }
  __device__ static __forceinline__ Acc identity(int op) {
    if (op == HP_OP_MIN || op == HP_OP_ARGMIN) return 0x7FFFFFFFFFFFFFFFll;
    if (op == HP_OP_MAX || op == HP_OP_ARGMAX) return (long long)0x8000000000000000ull;
    return 0;
  }
  __device__ static __forceinline__ Acc key(long long x, long long t, int op) {
    const unsigned long long hi = (unsigned long long)(uint32_t)(int32_t)x << 32;
    if (op == HP_OP_ARGMIN) return (long long)(hi | (uint32_t)t);
    if (op == HP_OP_ARGMAX) return (long long)(hi | (0xFFFFFFFFu - (uint32_t)t));
    return x;
  }
  __device__ static __forceinline__ Acc merge(Acc a, Acc b, int op) {
    if (op == HP_OP_SUM) return (long long)((unsigned long long)a + (unsigned long long)b);
    if (op == HP_OP_NONE) return a;
    return minlike(op) ? (b < a ? b : a) : (b > a ? b : a);
  }
  __device__ static __forceinline__ void add(Acc& a, long long x, long long t, int op) { a = merge(a, key(x, t, op), op); }
  __device__ static __forceinline__ long long emit(Acc a, int op) {
    if (op == HP_OP_ARGMIN) return (long long)(uint32_t)a;
    if (op == HP_OP_ARGMAX) return (long long)(0xFFFFFFFFu - (uint32_t)a);
    return a;
  }
  // LDS slots hold the key itself
  __device__ static __forceinline__ void put(char* base, long long slot, Acc a) {
    *reinterpret_cast<long long*>(base + slot * kSlotBytes) = a;
  }
  __device__ static __forceinline__ Acc get(const char* base, long long slot) {
    return *reinterpret_cast<const long long*>(base + slot * kSlotBytes);
  }
  // grid partials in the (value, index) form of IntT
  __device__ static __forceinline__ void put_partial(char* base, long long slot, Acc a, int op) {
    long long* q = reinterpret_cast<long long*>(base + slot * kSlotBytes);
    q[0] = arg(op) ? (long long)(int32_t)(uint32_t)((unsigned long long)a >> 32) : a;
    q[1] = arg(op) ? emit(a, op) : 0;
  }
};

// ---------------------------------------------------------------------------
// chunk loads: C consecutive elements of the innermost level; 16 bytes for the
// vector chunk (aligned: the plan only picks it when the extent allows)

template <class Raw, int C>
struct Chunk;
template <>
struct Chunk<float, 4> { using V = f32x4; };
template <>
struct Chunk<float, 1> { using V = float; };
template <>
struct Chunk<int32_t, 4> { using V = i32x4; };
template <>
struct Chunk<int32_t, 1> { using V = int; };
template <>
struct Chunk<uint16_t, 8> { using V = u32x4; };
template <>
struct Chunk<uint16_t, 1> { using V = unsigned short; };

// Inputs always live in global memory: say so, so that pointers read from tables
// (batches) still give global loads rather than flat ones (flat loads also count
// on the LDS counter and would be waited for together with LDS reads).
// The data is read once: nontemporal loads (the cache policy must be a
// compile-time property of the load; a runtime choice between two load forms gets
// merged into a plain load).
template <class V>
__device__ __forceinline__ V load_chunk(const void* p) {
  typedef const __attribute__((address_space(1))) V GV;
  return __builtin_nontemporal_load((GV*)(p));
}

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// element that leaves a carrier unchanged (for lanes whose chunk is masked out);
// for ARG the masked chunk's index is beyond the extent, so real ties still win
template <class T, int OP>
__device__ __forceinline__ float masked_f(float x, bool ok) {
  return ok ? x : 0.0f;
}
template <int OP>
__device__ __forceinline__ int masked_i(int x, bool ok) {
  constexpr int id = (OP == HP_OP_MIN || OP == HP_OP_ARGMIN) ? 0x7FFFFFFF
                     : (OP == HP_OP_MAX || OP == HP_OP_ARGMAX) ? (int)0x80000000
                                                               : 0;
  return ok ? x : id;
}

template <class T, int C, int OP>
struct AddChunk;
template <int OP>
struct AddChunk<FloatT<float>, 4, OP> {
  __device__ static __forceinline__ void run(FAcc& a, f32x4 x, long long, bool ok) {
    FloatT<float>::add(a, masked_f<FloatT<float>, OP>(x.x, ok), 0, 0);
    FloatT<float>::add(a, masked_f<FloatT<float>, OP>(x.y, ok), 0, 0);
    FloatT<float>::add(a, masked_f<FloatT<float>, OP>(x.z, ok), 0, 0);
    FloatT<float>::add(a, masked_f<FloatT<float>, OP>(x.w, ok), 0, 0);
  }
};
template <int OP>
struct AddChunk<FloatT<float>, 1, OP> {
  __device__ static __forceinline__ void run(FAcc& a, float x, long long, bool ok) {
    FloatT<float>::add(a, masked_f<FloatT<float>, OP>(x, ok), 0, 0);
  }
};
template <int OP>
struct AddChunk<FloatT<uint16_t>, 8, OP> {
  __device__ static __forceinline__ void run(FAcc& a, u32x4 x, long long, bool ok) {
    const u32x4 m = ok ? x : u32x4{0u, 0u, 0u, 0u};
    FloatT<uint16_t>::add(a, bf16_lo(m.x), 0, 0);
    FloatT<uint16_t>::add(a, bf16_hi(m.x), 0, 0);
    FloatT<uint16_t>::add(a, bf16_lo(m.y), 0, 0);
    FloatT<uint16_t>::add(a, bf16_hi(m.y), 0, 0);
    FloatT<uint16_t>::add(a, bf16_lo(m.z), 0, 0);
    FloatT<uint16_t>::add(a, bf16_hi(m.z), 0, 0);
    FloatT<uint16_t>::add(a, bf16_lo(m.w), 0, 0);
    FloatT<uint16_t>::add(a, bf16_hi(m.w), 0, 0);
  }
};
template <int OP>
struct AddChunk<FloatT<uint16_t>, 1, OP> {
  __device__ static __forceinline__ void run(FAcc& a, unsigned short x, long long, bool ok) {
    FloatT<uint16_t>::add(a, bf16_lo(ok ? x : 0), 0, 0);
  }
};
template <int OP>
struct AddChunk<IntT, 4, OP> {
  __device__ static __forceinline__ void run(IAcc& a, i32x4 x, long long t, bool ok) {
    if constexpr (OP == HP_OP_MIN || OP == HP_OP_MAX || OP == HP_OP_ARGMIN || OP == HP_OP_ARGMAX) {
      // min/max are associative and commutative, and so is the lexicographic
      // (value, index) order of ARG: reduce the four elements in 32 bits first
      // (the smallest position among equal values), then merge once into the
      // 64-bit carrier
      constexpr bool mn = OP == HP_OP_MIN || OP == HP_OP_ARGMIN;
      const int x0 = masked_i<OP>(x.x, ok), x1 = masked_i<OP>(x.y, ok);
      const int x2 = masked_i<OP>(x.z, ok), x3 = masked_i<OP>(x.w, ok);
      const int m = mn ? min(min(x0, x1), min(x2, x3)) : max(max(x0, x1), max(x2, x3));
      int pos = 0;
      if constexpr (OP == HP_OP_ARGMIN || OP == HP_OP_ARGMAX) pos = x0 == m ? 0 : x1 == m ? 1 : x2 == m ? 2 : 3;
      IntT::add(a, m, t + pos, OP);
    } else {
      IntT::add(a, masked_i<OP>(x.x, ok), t, OP);
      IntT::add(a, masked_i<OP>(x.y, ok), t + 1, OP);
      IntT::add(a, masked_i<OP>(x.z, ok), t + 2, OP);
      IntT::add(a, masked_i<OP>(x.w, ok), t + 3, OP);
    }
  }
};
template <int OP>
struct AddChunk<IntT, 1, OP> {
  __device__ static __forceinline__ void run(IAcc& a, int x, long long t, bool ok) {
    IntT::add(a, masked_i<OP>(x, ok), t, OP);
  }
};
// Key carriers: the four elements are reduced in 32 bits (for ARG the first
// position of the extreme value), then merged into the key once.
template <int OP>
struct AddChunk<IntK, 4, OP> {
  __device__ static __forceinline__ void run(long long& a, i32x4 x, long long t, bool ok) {
    const int x0 = masked_i<OP>(x.x, ok), x1 = masked_i<OP>(x.y, ok);
    const int x2 = masked_i<OP>(x.z, ok), x3 = masked_i<OP>(x.w, ok);
    if constexpr (OP == HP_OP_SUM) {
      a = (long long)((unsigned long long)a + (unsigned long long)((long long)x0 + x1) +
                      (unsigned long long)((long long)x2 + x3));
    } else {
      constexpr bool mn = OP == HP_OP_MIN || OP == HP_OP_ARGMIN;
      const int m = mn ? min(min(x0, x1), min(x2, x3)) : max(max(x0, x1), max(x2, x3));
      int pos = 0;
      if constexpr (OP == HP_OP_ARGMIN || OP == HP_OP_ARGMAX) pos = x0 == m ? 0 : x1 == m ? 1 : x2 == m ? 2 : 3;
      IntK::add(a, m, t + pos, OP);
    }
  }
};
template <int OP>
struct AddChunk<IntK, 1, OP> {
  __device__ static __forceinline__ void run(long long& a, int x, long long t, bool ok) {
    IntK::add(a, masked_i<OP>(x, ok), t, OP);
  }
};

// ---------------------------------------------------------------------------
// per-thread view of one workgroup's share

template <int KD>
struct Thread {
  int w, lane;
  int tid;      // thread index inside the group that runs one task
  bool wave;    // the group is one wavefront (batched wave tasks): no workgroup barriers
  int lim[KD];   // strips on which this thread's unit of level m has t < e
  int targ[KD];  // first iteration of level m for this thread (used by ARG levels)
  int limc[KD];  // lim of inner dim k
};

// Walk the innermost segment for one setting of the outer levels: U chunk loads in
// flight, then folded in order.  ND is the number of the segment's levels that have
// more than one strip (1, 2, or any up to KD).  With CHECK, lanes whose chunk is
// masked out load element 0 instead (always in bounds) and fold the identity, so
// the loads are never predicated and stay in flight together.
__device__ __forceinline__ long long readfirstlane64(long long v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(unsigned long long)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

template <class T, int C, int OP, int U, int ND, int KD, bool CHECK, bool FAST = false>
__device__ __forceinline__ typename T::Acc stream(const DevPlan& P, const typename T::Raw* __restrict__ in,
                                                  long long base, bool valid, const Thread<KD>& th) {
  using Acc = typename T::Acc;
  using V = typename Chunk<typename T::Raw, C>::V;
  using Raw = typename T::Raw;
  constexpr bool kArg = (OP == HP_OP_ARGMIN || OP == HP_OP_ARGMAX);
  const int nid = P.nid;
  Acc a = T::identity(OP);
  long long t_first = 0, span_last = 0;
  if constexpr (kArg) {
    const int dl = P.depth - 1;
#pragma unroll
    for (int m = 0; m < KD; ++m)
      if (m == dl) {
        t_first = th.targ[m];
        span_last = P.last_dim_is_last_level ? P.lv[m].span : 0;
      }
  }
  const Raw* __restrict__ row = in + base;
  const long long F = P.inner_iters;
  if constexpr (ND == 1 && FAST && !CHECK) {
    // Lean streaming (no masking; the plan guarantees vlane32): the wave's lowest
    // address lane 0's is kept in scalar registers and each lane adds a 32-bit byte
    // offset, so a load costs one VGPR of address.  Loads are software-pipelined:
    // batch k+1 is issued before batch k is folded, so each wave keeps loads in
    // flight while it computes.
    const long long ss = nid > 0 ? P.id_sstride[0] : 0;
    const long long ub = readfirstlane64(base);
    const uint32_t lo = (uint32_t)((base - ub) * (long long)sizeof(Raw));
    const char* pu = reinterpret_cast<const char*>(in + ub);
    const long long ssb = ss * (long long)sizeof(Raw);
    auto ld = [&](long long f) -> V { return load_chunk<V>((pu + f * ssb) + lo); };
    const long long Ffull = F - F % U;
    long long f0 = 0;
    if (Ffull > 0) {
      V x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = ld(u);
      for (f0 = U; f0 < Ffull; f0 += U) {
        V y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) y[u] = ld(f0 + u);
#pragma unroll
        for (int u = 0; u < U; ++u) AddChunk<T, C, OP>::run(a, x[u], t_first + (f0 - U + u) * span_last, true);
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = y[u];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) AddChunk<T, C, OP>::run(a, x[u], t_first + (f0 - U + u) * span_last, true);
    }
    for (; f0 < F; ++f0) AddChunk<T, C, OP>::run(a, ld(f0), t_first + f0 * span_last, true);
  } else if constexpr (ND == 1) {
    // one strided dimension (or none): chunk f sits at f * sstride.  Full batches
    // are straight-line code (U loads, then U folds); the tail goes one by one.
    const long long ss = nid > 0 ? P.id_sstride[0] : 0;
    const bool rag = nid > 0 && P.id_ragged[0];
    const int lim = th.limc[0];
    const long long Ffull = F - F % U;
    long long f0 = 0;
    for (; f0 < Ffull; f0 += U) {
      V x[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long long f = f0 + u;
        ok[u] = true;
        if constexpr (CHECK) ok[u] = valid && (!rag || f < lim);
        x[u] = load_chunk<V>(ok[u] ? row + f * ss : in);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) AddChunk<T, C, OP>::run(a, x[u], t_first + (f0 + u) * span_last, ok[u]);
    }
    for (; f0 < F; ++f0) {
      bool ok = true;
      if constexpr (CHECK) ok = valid && (!rag || f0 < lim);
      const V x = load_chunk<V>(ok ? row + f0 * ss : in);
      AddChunk<T, C, OP>::run(a, x, t_first + f0 * span_last, ok);
    }
  } else if constexpr (ND == 2) {
    const long long S1 = P.id_strips[1];
    const long long ss0 = P.id_sstride[0], ss1 = P.id_sstride[1];
    const bool rag0 = P.id_ragged[0], rag1 = P.id_ragged[1];
    const int lim0 = th.limc[0], lim1 = th.limc[1];
    long long s0 = 0, s1 = 0, soff = 0;
    for (long long f0 = 0; f0 < F; f0 += U) {
      const int nu = (F - f0) < U ? (int)(F - f0) : U;
      V x[U];
      bool ok[U];
      long long sl[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ok[u] = true;
        if constexpr (CHECK) ok[u] = valid && (!rag0 || s0 < lim0) && (!rag1 || s1 < lim1);
        sl[u] = s1;
        if (u < nu) {
          x[u] = load_chunk<V>(ok[u] ? row + soff : in);
          soff += ss1;
          if (++s1 == S1) {
            s1 = 0;
            ++s0;
            soff += ss0 - S1 * ss1;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (u < nu) AddChunk<T, C, OP>::run(a, x[u], t_first + sl[u] * span_last, ok[u]);
    }
  } else {
    int s[KD];
#pragma unroll
    for (int k = 0; k < KD; ++k) s[k] = 0;
    long long soff = 0;
    for (long long f0 = 0; f0 < F; f0 += U) {
      const int nu = (F - f0) < U ? (int)(F - f0) : U;
      V x[U];
      bool ok[U];
      int sl[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        bool v = valid;
#pragma unroll
        for (int k = 0; k < KD; ++k)
          if (k < nid && P.id_ragged[k]) v = v && (s[k] < th.limc[k]);
        ok[u] = v;
        sl[u] = 0;
#pragma unroll
        for (int k = 0; k < KD; ++k)
          if (k == nid - 1) sl[u] = s[k];
        if (u < nu) {
          x[u] = load_chunk<V>(ok[u] ? row + soff : in);
          bool carry = true;
#pragma unroll
          for (int k = KD - 1; k >= 0; --k) {
            if (carry && k < nid) {
              ++s[k];
              soff += P.id_sstride[k];
              if (s[k] == P.id_strips[k]) {
                s[k] = 0;
                soff -= P.id_strips[k] * P.id_sstride[k];
              } else {
                carry = false;
              }
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (u < nu) AddChunk<T, C, OP>::run(a, x[u], t_first + (long long)sl[u] * span_last, ok[u]);
    }
  }
  return a;
}

template <class T, int C, int OP, int U, int KD, bool LEAN>
__device__ __forceinline__ typename T::Acc stream_any(const DevPlan& P, const typename T::Raw* __restrict__ in,
                                                      long long base, bool valid, const Thread<KD>& th) {
  // every lane of the wave valid and no ragged level: no masking needed
  bool rag = false;
#pragma unroll
  for (int k = 0; k < KD; ++k)
    if (k < P.nid && P.id_ragged[k]) rag = true;
  const bool check = rag || __builtin_amdgcn_ballot_w64(!valid) != 0;
  if (LEAN || P.nid <= 1) {  // lean kernels are only launched for plans with nid <= 1 and vlane32
    if (check || !(LEAN || P.vlane32)) return stream<T, C, OP, U, 1, KD, true>(P, in, base, valid, th);
    return stream<T, C, OP, (U < 4 ? U : 4), 1, KD, false, true>(P, in, base, valid, th);
  }
  if (P.nid == 2) {
    if (check) return stream<T, C, OP, U, 2, KD, true>(P, in, base, valid, th);
    return stream<T, C, OP, U, 2, KD, false>(P, in, base, valid, th);
  }
  return stream<T, C, OP, U, KD, KD, true>(P, in, base, valid, th);
}

template <class T, int C, int U, int KD, bool LEAN>
struct InnerStream;
template <class R, int C, int U, int KD, bool LEAN>
struct InnerStream<FloatT<R>, C, U, KD, LEAN> {
  __device__ static __forceinline__ FAcc run(const DevPlan& P, const R* __restrict__ in, long long base, bool valid,
                                             const Thread<KD>& th) {
    return stream_any<FloatT<R>, C, HP_OP_SUM, U, KD, LEAN>(P, in, base, valid, th);
  }
};
template <class I, int C, int U, int KD, bool LEAN>
struct IntInnerStream {
  __device__ static __forceinline__ typename I::Acc run(const DevPlan& P, const int32_t* __restrict__ in,
                                                        long long base, bool valid, const Thread<KD>& th) {
    switch (P.seg[P.nseg - 1].op) {
      case HP_OP_MIN: return stream_any<I, C, HP_OP_MIN, U, KD, LEAN>(P, in, base, valid, th);
      case HP_OP_MAX: return stream_any<I, C, HP_OP_MAX, U, KD, LEAN>(P, in, base, valid, th);
      case HP_OP_ARGMIN: return stream_any<I, C, HP_OP_ARGMIN, U, KD, LEAN>(P, in, base, valid, th);
      case HP_OP_ARGMAX: return stream_any<I, C, HP_OP_ARGMAX, U, KD, LEAN>(P, in, base, valid, th);
      default: return stream_any<I, C, HP_OP_SUM, U, KD, LEAN>(P, in, base, valid, th);
    }
  }
};
template <int C, int U, int KD, bool LEAN>
struct InnerStream<IntT, C, U, KD, LEAN> : IntInnerStream<IntT, C, U, KD, LEAN> {};
template <int C, int U, int KD, bool LEAN>
struct InnerStream<IntK, C, U, KD, LEAN> : IntInnerStream<IntK, C, U, KD, LEAN> {};

// Synchronise the threads that run one task: the whole workgroup, or (for wave
// tasks) one wavefront, which runs in lockstep and only needs its LDS accesses
// ordered.
__device__ __forceinline__ void group_sync(bool wave) {
  if (wave) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// One butterfly step on lane bit B for a carrier of float pairs or integer keys
// (moves from hp_lanes.h; `uni`: the step may take the mirror / permlane-swap form).
template <int B>
__device__ __forceinline__ FAcc lane_step(FAcc a, bool uni, int lane, int) {
  if constexpr (B >= 4) {
    if (uni) {
      int s0, s1, c0, c1;
      sides32<B>(__float_as_int(a.s), s0, s1);
      sides32<B>(__float_as_int(a.c), c0, c1);
      return FloatT<float>::merge(FAcc{__int_as_float(s0), __int_as_float(c0)},
                                  FAcc{__int_as_float(s1), __int_as_float(c1)}, 0);
    }
  }
  const FAcc o{__int_as_float(partner32<B>(__float_as_int(a.s), uni, lane)),
               __int_as_float(partner32<B>(__float_as_int(a.c), uni, lane))};
  return FloatT<float>::merge(a, o, 0);
}

// 64-bit integer sum step
template <int B>
__device__ __forceinline__ long long key_sum_step(long long a, bool uni, int lane) {
  const int lo = (int)(uint32_t)(unsigned long long)a, hi = (int)(uint32_t)((unsigned long long)a >> 32);
  if constexpr (B >= 4) {
    if (uni) {
      int l0, l1, h0, h1;
      sides32<B>(lo, l0, l1);
      sides32<B>(hi, h0, h1);
      const unsigned long long x = ((unsigned long long)(uint32_t)h0 << 32) | (uint32_t)l0;
      const unsigned long long y = ((unsigned long long)(uint32_t)h1 << 32) | (uint32_t)l1;
      return (long long)(x + y);
    }
  }
  const unsigned long long y = ((unsigned long long)(uint32_t)partner32<B>(hi, uni, lane) << 32) |
                               (uint32_t)partner32<B>(lo, uni, lane);
  return (long long)((unsigned long long)a + y);
}

// 32-bit min / max step (signed or unsigned)
template <int B, bool MN, class W>
__device__ __forceinline__ W word_step(W v, bool uni, int lane) {
  if constexpr (B >= 4) {
    if (uni) {
      int x0, x1;
      sides32<B>((int)v, x0, x1);
      return MN ? min((W)x0, (W)x1) : max((W)x0, (W)x1);
    }
  }
  const W o = (W)partner32<B>((int)v, uni, lane);
  return MN ? min(v, o) : max(v, o);
}

template <bool MN, class W>
__device__ __forceinline__ W word_allreduce(W v, uint32_t vmask, uint32_t ufast, int lane) {
  if (vmask & 1u) v = word_step<0, MN, W>(v, ufast & 1u, lane);
  if (vmask & 2u) v = word_step<1, MN, W>(v, ufast & 2u, lane);
  if (vmask & 4u) v = word_step<2, MN, W>(v, ufast & 4u, lane);
  if (vmask & 8u) v = word_step<3, MN, W>(v, ufast & 8u, lane);
  if (vmask & 16u) v = word_step<4, MN, W>(v, ufast & 16u, lane);
  if (vmask & 32u) v = word_step<5, MN, W>(v, ufast & 32u, lane);
  return v;
}

// Signed 64-bit min / max over a lane group in two 32-bit passes: the extreme high
// word, then the extreme low word (unsigned) among the lanes that hold it -- the
// same order as a 64-bit comparison, and each pass a single 32-bit op per step.
template <bool MN>
__device__ __forceinline__ long long key_minmax(long long a, uint32_t vmask, uint32_t ufast, int lane) {
  const int hi = (int)(uint32_t)((unsigned long long)a >> 32);
  const uint32_t lo = (uint32_t)(unsigned long long)a;
  const int m = word_allreduce<MN, int>(hi, vmask, ufast, lane);
  const uint32_t cand = hi == m ? lo : (MN ? 0xFFFFFFFFu : 0u);
  const uint32_t l = word_allreduce<MN, uint32_t>(cand, vmask, ufast, lane);
  return (long long)(((unsigned long long)(uint32_t)m << 32) | l);
}

template <class T>
__device__ __forceinline__ typename T::Acc lane_combine(typename T::Acc a, const DevSeg& S, int lane) {
  const uint32_t vm = S.vmask, uf = S.ufast;
  if constexpr (T::kFloat) {
    if (vm & 1u) a = lane_step<0>(a, uf & 1u, lane, 0);
    if (vm & 2u) a = lane_step<1>(a, uf & 2u, lane, 0);
    if (vm & 4u) a = lane_step<2>(a, uf & 4u, lane, 0);
    if (vm & 8u) a = lane_step<3>(a, uf & 8u, lane, 0);
    if (vm & 16u) a = lane_step<4>(a, uf & 16u, lane, 0);
    if (vm & 32u) a = lane_step<5>(a, uf & 32u, lane, 0);
    return a;
  } else if constexpr (T::kKey) {
    const int op = S.op;
    if (op == HP_OP_SUM) {
      if (vm & 1u) a = key_sum_step<0>(a, uf & 1u, lane);
      if (vm & 2u) a = key_sum_step<1>(a, uf & 2u, lane);
      if (vm & 4u) a = key_sum_step<2>(a, uf & 4u, lane);
      if (vm & 8u) a = key_sum_step<3>(a, uf & 8u, lane);
      if (vm & 16u) a = key_sum_step<4>(a, uf & 16u, lane);
      if (vm & 32u) a = key_sum_step<5>(a, uf & 32u, lane);
      return a;
    }
    if (op == HP_OP_MIN || op == HP_OP_ARGMIN) return key_minmax<true>(a, vm, uf, lane);
    return key_minmax<false>(a, vm, uf, lane);
  } else {
#pragma unroll
    for (int b = 0; b < 6; ++b)
      if ((vm >> b) & 1u) a = T::merge(a, T::shfl(a, 1 << b, lane), S.op);
    return a;
  }
}

// Combine a segment's partials across its lanes (butterfly) and waves (LDS).
// Afterwards every lane of a group holds the group's value.
template <class T, int KD>
__device__ __forceinline__ typename T::Acc combine_seg(const DevPlan& P, const DevSeg& S, typename T::Acc a,
                                                       const Thread<KD>& th, char* lds) {
  if (S.vmask) a = lane_combine<T>(a, S, th.lane);
  if (S.wmask) {
    const int lanes = P.lds_slot_lanes;
    const int lidx = lanes == 1 ? 0 : (int)(th.lane & S.lds_lanes);
    group_sync(th.wave);  // earlier readers of the slots are done
    if ((th.lane & ~(int)S.lds_lanes & 63) == 0) T::put(lds, th.w * lanes + lidx, a);
    group_sync(th.wave);
    const int wbase = th.w & ~(int)S.wmask;
    typename T::Acc r = T::get(lds, wbase * lanes + lidx);
    for (int j = 1; j < S.nwu; ++j) r = T::merge(r, T::get(lds, (wbase | (j << S.wlo)) * lanes + lidx), S.op);
    a = r;
  }
  return a;
}

// Flat blocks (DevPlan::flat_b): add the elements of the output's block that lie
// outside its aligned interior -- the h = (-s) mod chunk before it and the tail
// after it -- spread over the flat_units threads that share the output.  The tail
// starts on a 16-byte boundary (the interior is whole vectors), so its whole vectors
// are 16-byte loads, vector j taken by the thread of rank j mod flat_units; the h
// head elements and the tail's last partial vector are single-element loads spread
// the same way.  Every element of the block is inside the array, so no load leaves it.
template <class T>
struct RestAdd;
template <>
struct RestAdd<FloatT<float>> {
  __device__ static __forceinline__ void run(FAcc& a, float x, int) { FloatT<float>::add(a, x, 0, 0); }
};
template <>
struct RestAdd<FloatT<uint16_t>> {
  __device__ static __forceinline__ void run(FAcc& a, uint16_t x, int) {
    FloatT<uint16_t>::add(a, bf16_lo((uint32_t)x), 0, 0);
  }
};
template <>
struct RestAdd<IntT> {
  __device__ static __forceinline__ void run(IAcc& a, int x, int op) { IntT::add(a, x, 0, op); }
};
template <>
struct RestAdd<IntK> {
  __device__ static __forceinline__ void run(long long& a, int x, int op) { IntK::add(a, x, 0, op); }
};

// one whole vector of the tail (float sums fold it like a stream chunk; integer
// flat blocks carry a runtime operator, so their four elements go one by one)
template <class T, int C>
struct RestVec {
  using V = typename Chunk<typename T::Raw, C>::V;
  __device__ static __forceinline__ void run(typename T::Acc& a, const typename T::Raw* p, int op) {
    if constexpr (T::kFloat) {
      AddChunk<T, C, HP_OP_SUM>::run(a, load_chunk<V>(p), 0, true);
    } else if constexpr (C == 4) {
      const V x = load_chunk<V>(p);
      RestAdd<T>::run(a, x.x, op);
      RestAdd<T>::run(a, x.y, op);
      RestAdd<T>::run(a, x.z, op);
      RestAdd<T>::run(a, x.w, op);
    } else {
      RestAdd<T>::run(a, load_chunk<V>(p), op);
    }
  }
};

template <class T, int C, int KD>
__device__ __forceinline__ typename T::Acc flat_rest(const DevPlan& P, const typename T::Raw* __restrict__ in, long long s,
                                                  typename T::Acc a, const Thread<KD>& th) {
  const long long h = (-s) & (long long)(P.chunk - 1);
  const long long tail = s + h + P.flat_e;      // first tail element (16-byte aligned)
  const long long tl = P.flat_b - h - P.flat_e;  // tail length
  const long long nv = tl / C;                   // whole vectors in the tail
  const long long ns = h + (tl - nv * C);        // single elements: the head, then the tail's end
  const long long tv = tail + nv * C;
  long long r = 0;
#pragma unroll
  for (int m = 0; m < KD; ++m)
    if (m >= P.p && m < P.depth) {
      const DevLevel& L = P.lv[m];
      r = r * ((long long)L.gf * L.wf * L.vf) + (th.targ[m] >> L.csh);
    }
  const int op = P.seg[0].op;
  const long long U = P.flat_units;
  for (long long j = r; j < nv; j += U) RestVec<T, C>::run(a, in + tail + j * C, op);
  for (long long k = r; k < ns; k += U) RestAdd<T>::run(a, in[k < h ? s + k : tv + (k - h)], op);
  return a;
}

// Reduce the current output's block; returns segment P.gq's value (the output, or
// this workgroup's partial of it when that segment spans workgroups).
// FL: flat-block plans may run this instantiation (the rest-element code is
// compiled in); kernels that never see them leave it out and keep fewer registers.
template <class T, int C, int NS, int U, int KD, bool LEAN, bool PF = true, bool FL = true>
__device__ __forceinline__ typename T::Acc reduce_block(const DevPlan& P, const typename T::Raw* __restrict__ in,
                                                        long long base, bool vnone, const Thread<KD>& th, char* lds,
                                                        long long flat_s = 0) {
  using Acc = typename T::Acc;
  constexpr int NO = NS > 1 ? NS - 1 : 1;
  const int inner = P.nseg - 1;
  const int stop = P.gq;
  const int p = P.p, a_lv = P.a;
  Acc outer[NO];
#pragma unroll
  for (int j = 0; j < NO; ++j) outer[j] = T::identity(j < P.nseg ? P.seg[j].op : 0);
  int s[KD];
#pragma unroll
  for (int k = 0; k < KD; ++k) s[k] = 0;
  long long soff = 0;
  Acc fin = T::identity(0);
  // inner-segment levels with a single strip: a unit beyond the extent never loads
  bool inner_ok = true;
#pragma unroll
  for (int m = 0; m < KD; ++m)
    if (m >= a_lv && m < P.depth && P.lv[m].strips == 1 && P.lv[m].ragged) inner_ok = inner_ok && th.lim[m] > 0;
  auto outer_valid = [&]() -> bool {
    bool vo = vnone && inner_ok;
#pragma unroll
    for (int m = 0; m < KD; ++m)
      if (m >= p && m < a_lv && P.lv[m].ragged) vo = vo && (s[m] < th.lim[m]);
    return vo;
  };
  // advance the outer odometer (levels p .. a-1, innermost fastest)
  auto advance = [&]() {
    bool carry = true;
#pragma unroll
    for (int m = KD - 1; m >= 0; --m) {
      if (carry && m >= p && m < a_lv) {
        ++s[m];
        soff += P.lv[m].sstride;
        if (s[m] == P.lv[m].strips) {
          s[m] = 0;
          soff -= P.lv[m].strips * P.lv[m].sstride;
        } else {
          carry = false;
        }
      }
    }
  };
  // combine the innermost segment's lane partials, feed its value to the parent
  // segment, then finish the outer segments whose strips all end here
  auto consume = [&](Acc ai) {
    // flat blocks have one segment walked in one outer iteration: the rest of the
    // block joins the lane partials before they are combined
    if constexpr (FL)
      if (P.flat_b && vnone) ai = flat_rest<T, C, KD>(P, in, flat_s, ai, th);
    ai = combine_seg<T, KD>(P, P.seg[inner], ai, th, lds);
    if (inner == stop) {
      fin = ai;
    } else if constexpr (NS > 1) {
#pragma unroll
      for (int j = NO - 1; j >= 0; --j) {
        if (j == inner - 1) {
          const DevSeg& Sp = P.seg[j];
          bool vj = true;
          long long t = 0;
#pragma unroll
          for (int m = 0; m < KD; ++m) {
            if (m >= Sp.first && m <= Sp.last && P.lv[m].ragged) vj = vj && (s[m] < th.lim[m]);
            if (m == Sp.last) t = th.targ[m] + (long long)s[m] * P.lv[m].span;
          }
          if (vj) T::add(outer[j], T::emit(ai, P.seg[inner].op), t, Sp.op);
        }
      }
      // common case: the innermost outer level has strips left, so no outer
      // segment ends here
      bool more = false;
#pragma unroll
      for (int m = 0; m < KD; ++m)
        if (m == a_lv - 1 && m >= p) more = s[m] < P.lv[m].strips - 1;
      if (more) return;
      int J = 0;
#pragma unroll
      for (int m = 0; m < KD; ++m)
        if (m >= p && m < a_lv && s[m] < P.lv[m].strips - 1) J = P.lv[m].seg + 1;
#pragma unroll
      for (int j = NO - 1; j >= 0; --j) {
        if (j < inner && j >= J && j >= stop) {
          const DevSeg& S = P.seg[j];
          Acc v = combine_seg<T, KD>(P, S, outer[j], th, lds);
          if (j > stop) {
            const DevSeg& Sp = P.seg[j > 0 ? j - 1 : 0];
            bool vj = true;
            long long t = 0;
#pragma unroll
            for (int m = 0; m < KD; ++m) {
              if (m >= Sp.first && m <= Sp.last && P.lv[m].ragged) vj = vj && (s[m] < th.lim[m]);
              if (m == Sp.last) t = th.targ[m] + (long long)s[m] * P.lv[m].span;
            }
            if (vj) T::add(outer[j > 0 ? j - 1 : 0], T::emit(v, S.op), t, Sp.op);
            outer[j] = T::identity(S.op);
          } else {
            outer[j] = v;
          }
        }
      }
    }
  };
  bool done = false;
  if constexpr (!LEAN && PF) {
    if (P.outer_iters > 1 && P.nid <= 1 && P.inner_iters <= 4) {
      // The innermost segment is at most 4 chunks per outer iteration: load the
      // chunks of UO outer iterations back to back, then fold and combine them in
      // order, so that a wave has more than one iteration's loads in flight.
      auto prefetch = [&](auto opc, auto fmc) {
        constexpr int OPI = decltype(opc)::value;
        constexpr int FM = decltype(fmc)::value;  // chunks per outer iteration, at most
        constexpr int UO = FM == 1 ? (U >= 8 ? U / 2 : U) : (U / FM > 1 ? U / FM : 2);
        using V = typename Chunk<typename T::Raw, C>::V;
        const int F = (int)P.inner_iters;
        const long long ss = P.nid > 0 ? P.id_sstride[0] : 0;
        const bool rag = P.nid > 0 && P.id_ragged[0];
        const int lim = th.limc[0];
        long long t_first = 0, span_last = 0;
#pragma unroll
        for (int m = 0; m < KD; ++m)
          if (m == P.depth - 1) {
            t_first = th.targ[m];
            span_last = P.last_dim_is_last_level ? P.lv[m].span : 0;
          }
        for (long long q0 = 0; q0 < P.outer_iters; q0 += UO) {
          const int nu = (P.outer_iters - q0) < UO ? (int)(P.outer_iters - q0) : UO;
          V x[UO][FM];
          bool ok[UO];
          int s_keep[KD];
#pragma unroll
          for (int m = 0; m < KD; ++m) s_keep[m] = s[m];
          const long long soff_keep = soff;
#pragma unroll
          for (int u = 0; u < UO; ++u) {
            ok[u] = false;
            if (u < nu) {
              ok[u] = outer_valid();
#pragma unroll
              for (int f = 0; f < FM; ++f)
                if (f < F) {
                  const bool okf = ok[u] && (!rag || f < lim);
                  x[u][f] = load_chunk<V>(okf ? in + base + soff + f * ss : in);
                }
              advance();
            }
          }
#pragma unroll
          for (int m = 0; m < KD; ++m) s[m] = s_keep[m];
          soff = soff_keep;
#pragma unroll
          for (int u = 0; u < UO; ++u) {
            if (u < nu) {
              Acc ai = T::identity(OPI);
#pragma unroll
              for (int f = 0; f < FM; ++f)
                if (f < F) AddChunk<T, C, OPI>::run(ai, x[u][f], t_first + f * span_last, ok[u] && (!rag || f < lim));
              consume(ai);
              advance();
            }
          }
        }
      };
      auto by_op = [&](auto fmc) {
        if constexpr (T::kFloat) {
          prefetch(std::integral_constant<int, HP_OP_SUM>{}, fmc);
        } else {
          switch (P.seg[inner].op) {
            case HP_OP_MIN: prefetch(std::integral_constant<int, HP_OP_MIN>{}, fmc); break;
            case HP_OP_MAX: prefetch(std::integral_constant<int, HP_OP_MAX>{}, fmc); break;
            case HP_OP_ARGMIN: prefetch(std::integral_constant<int, HP_OP_ARGMIN>{}, fmc); break;
            case HP_OP_ARGMAX: prefetch(std::integral_constant<int, HP_OP_ARGMAX>{}, fmc); break;
            default: prefetch(std::integral_constant<int, HP_OP_SUM>{}, fmc); break;
          }
        }
      };
      if (P.inner_iters == 1) by_op(std::integral_constant<int, 1>{});
      else by_op(std::integral_constant<int, 4>{});
      done = true;
    }
  }
  if (!done) {
    for (long long q = 0; q < P.outer_iters; ++q) {
      const bool vo = outer_valid();
      consume(InnerStream<T, C, U, KD, LEAN>::run(P, in, base + soff, vo, th));
      advance();
    }
  }
  Acc r = fin;
#pragma unroll
  for (int j = 0; j < NO; ++j)
    if (j == stop && j != inner) r = outer[j];
  return r;
}

// ---------------------------------------------------------------------------
// outputs and the grid combine

__device__ __forceinline__ void store_int(const DevPlan& P, void* out, long long o, long long v) {
  if (P.out_kind == OUT_I64) reinterpret_cast<long long*>(out)[o] = v;
  else reinterpret_cast<int*>(out)[o] = (int)v;
}
__device__ __forceinline__ void store_flt(const DevPlan& P, void* out, long long o, double v) {
  if (P.out_kind == OUT_F64) reinterpret_cast<double*>(out)[o] = v;
  else reinterpret_cast<float*>(out)[o] = (float)v;
}

struct DPair {
  double s, c;
};
__device__ __forceinline__ void dpair_add(DPair& a, double x) {
  double s, e;
  two_sum(a.s, x, s, e);
  a.s = s;
  a.c += e;
}
__device__ __forceinline__ DPair dpair_merge(DPair a, DPair b) {
  double s, e;
  two_sum(a.s, b.s, s, e);
  const double c = (a.c + b.c) + e;
  const double s2 = s + c;
  return DPair{s2, c - (s2 - s)};
}

// ---------------------------------------------------------------------------
// one workgroup

template <class T, int C, int NS, int U, int KD, bool LEAN = false, bool WAVE = false, bool PF = true,
          bool FL = true>
__device__ __forceinline__ void wg_run(const DevPlan& P, const typename T::Raw* __restrict__ in,
                                       void* __restrict__ out, unsigned char* __restrict__ ws, uint32_t g,
                                       char* lds) {
  Thread<KD> th;
  th.w = WAVE ? 0 : (int)(threadIdx.x >> 6);
  th.lane = (int)(threadIdx.x & 63);
  th.tid = WAVE ? th.lane : (int)threadIdx.x;
  th.wave = WAVE;
  long long base_none = 0, base_o = 0, base_red = 0;
#pragma unroll
  for (int m = 0; m < KD; ++m) {
    th.lim[m] = 1;
    th.targ[m] = 0;
    if (m < P.depth) {
      const DevLevel& L = P.lv[m];
      const uint32_t ug = g_digit(g, L);
      const uint32_t uw = ((uint32_t)th.w >> L.wsh) & (uint32_t)(L.wf - 1);
      const uint32_t uv = ((uint32_t)th.lane >> L.vsh) & (uint32_t)(L.vf - 1);
      const long long t0 = (long long)(((unsigned long long)ug * L.wf + uw) * L.vf + uv) * L.chunk;
      // a level without a ragged tail has every strip in range (t0 < span), and
      // lim is only read for ragged levels: skip the per-lane division there
      if (!L.ragged) th.lim[m] = (int)L.strips;
      else if (t0 >= L.e) th.lim[m] = 0;
      else if (L.fd_span.m) th.lim[m] = (int)fdiv((uint32_t)(L.e - t0 + L.span - 1), L.fd_span, (uint32_t)L.span);
      else th.lim[m] = (int)((L.e - t0 + L.span - 1) / L.span);
      th.targ[m] = (int)t0;
      if (m < P.p) {
        base_none += t0 * L.stride;
        base_o += t0 * L.ostride;
      } else {
        base_red += t0 * L.stride;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KD; ++k) {
    th.limc[k] = 1;
#pragma unroll
    for (int m = 0; m < KD; ++m)
      if (k < P.nid && m == P.id_level[k]) th.limc[k] = th.lim[m];
  }
  const bool red_writer = ((th.lane & (int)(P.red_vmask | P.idle_vmask)) == 0) &&
                          ((th.w & (int)(P.red_wmask | P.idle_wmask)) == 0);
  const uint32_t gred = (uint32_t)((unsigned long long)g % (unsigned long long)P.gsplit);

  int sn[KD];
#pragma unroll
  for (int m = 0; m < KD; ++m) sn[m] = 0;
  long long noff = 0, nout = 0;
  for (long long q = 0; q < P.none_iters; ++q) {
    bool vnone = true;
#pragma unroll
    for (int m = 0; m < KD; ++m)
      if (m < P.p && P.lv[m].ragged) vnone = vnone && (sn[m] < th.lim[m]);
    const long long off = base_none + noff;
    const long long o = base_o + nout;
    if (P.p == P.depth) {  // nothing reduces: a copy
      if (vnone && red_writer) {
        if constexpr (T::kFloat) {
          double v;
          if constexpr (sizeof(typename T::Raw) == 2) v = (double)bf16_lo(in[off]);
          else v = (double)in[off];
          store_flt(P, out, o, v);
        } else {
          store_int(P, out, o, (long long)in[off]);
        }
      }
    } else {
      // flat blocks: the aligned interior starts h elements into the block
      const long long h = (FL && P.flat_b) ? ((-off) & (long long)(P.chunk - 1)) : 0;
      const typename T::Acc a =
          reduce_block<T, C, NS, U, KD, LEAN, PF, FL>(P, in, off + h + base_red, vnone, th, lds, off);
      if (P.gmode == GCOMB_NONE) {
        if (vnone && red_writer) {
          if constexpr (T::kFloat) store_flt(P, out, o, (double)a.s + (double)a.c);
          else store_int(P, out, o, T::emit(a, P.seg[0].op));
        }
      } else if (vnone) {  // uniform here: with a grid combine every NONE level is on G only
        // grid combine: this workgroup's partial; the fold kernel combines them
        char* part = reinterpret_cast<char*>(ws) + o * P.gsplit * kSlotBytes;
        if (th.tid == 0) {
          if constexpr (T::kKey) T::put_partial(part, gred, a, P.seg[P.gq].op);
          else T::put(part, gred, a);
        }
      }
    }
    // advance the NONE odometer
    bool carry = true;
#pragma unroll
    for (int m = KD - 1; m >= 0; --m) {
      if (carry && m < P.p) {
        ++sn[m];
        noff += P.lv[m].sstride;
        nout += P.lv[m].span * P.lv[m].ostride;
        if (sn[m] == P.lv[m].strips) {
          sn[m] = 0;
          noff -= P.lv[m].strips * P.lv[m].sstride;
          nout -= P.lv[m].strips * P.lv[m].span * P.lv[m].ostride;
        } else {
          carry = false;
        }
      }
    }
  }
}

// XCD-aware numbering: the dispatcher deals workgroups round-robin to the 8 XCDs
// (measured with hp_xcd_ids: workgroup b runs on XCD (b + c) mod 8, c fixed within a
// launch), so physical workgroups with one residue b mod 8 share an XCD and its L2.
// They get one contiguous range of logical workgroups -- the outermost grid digit,
// which an X level of the map takes.
__device__ __forceinline__ uint32_t logical_group(const DevPlan& P, uint32_t b) {
  if (!P.xcd) return b;
  const uint32_t per = (uint32_t)P.grid >> 3;  // grid % 8 == 0 when xcd is set
  return (b & 7u) * per + (b >> 3);
}

// Launchers, one per input type (each in its own translation unit).  P is the host
// copy (launch geometry), dP the same plan in device memory (read by the kernel).
hp_status launch_nest_f32(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds,
                          hipStream_t st);
hp_status launch_nest_bf16(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds,
                           hipStream_t st);
// Ordered products (AFFINE64 / MAT2X2_64 elements): the chunk kernel and, for split
// blocks, the in-order fold of the chunk products.
hp_status launch_ordered(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, hipStream_t st);
hp_status launch_nest_i32(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds,
                          hipStream_t st);

}  // namespace hp
