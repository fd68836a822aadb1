// Ordered products: associative, non-commutative reductions of affine maps and
// 2x2 matrices modulo 2^64 (HP_OP_PROD).  The paper points out that OpenMP
// reductions must be commutative (section 2); here siblings are combined strictly
// in iteration order at every level of the hierarchy:
//   lane    one contiguous 64th of a chunk, read K elements (one 128-byte line) at
//           a time through LDS after coalesced loads, each K as a balanced tree
//           over adjacent pairs, appended to the lane's running product;
//   wave    a xor butterfly in which the lower-lane half always stands on the left,
//           so after log2(64) steps every lane holds the chunk's product in order;
//   grid    chunk products folded left to right by a second kernel.
// The reduced block of one output is contiguous (row-major input), so every level
// of a nested product collapses into one ordered product over the block.
#include <hip/hip_runtime.h>

#include "hp_internal.h"
#include "hp_nest.h"

namespace hp {

typedef unsigned long long u64;

template <int W>
struct Elem {
  u64 v[W];
};

// x * y, x first.  Affine (a, b): x -> a x + b; matrices row-major.
template <int W>
__device__ __forceinline__ Elem<W> mul(const Elem<W>& x, const Elem<W>& y) {
  Elem<W> r;
  if constexpr (W == 2) {
    r.v[0] = x.v[0] * y.v[0];
    r.v[1] = y.v[0] * x.v[1] + y.v[1];
  } else {
    r.v[0] = x.v[0] * y.v[0] + x.v[1] * y.v[2];
    r.v[1] = x.v[0] * y.v[1] + x.v[1] * y.v[3];
    r.v[2] = x.v[2] * y.v[0] + x.v[3] * y.v[2];
    r.v[3] = x.v[2] * y.v[1] + x.v[3] * y.v[3];
  }
  return r;
}

template <int W>
__device__ __forceinline__ Elem<W> unit() {
  Elem<W> r;
#pragma unroll
  for (int k = 0; k < W; ++k) r.v[k] = 0;
  r.v[0] = 1;
  if constexpr (W == 4) r.v[3] = 1;
  return r;
}

template <int W>
__device__ __forceinline__ Elem<W> pick(bool c, const Elem<W>& a, const Elem<W>& b) {
  Elem<W> r;
#pragma unroll
  for (int k = 0; k < W; ++k) r.v[k] = c ? a.v[k] : b.v[k];
  return r;
}

// one element from global memory (16-byte nontemporal loads)
template <int W>
__device__ __forceinline__ Elem<W> load_elem(const u64* p) {
  typedef u64 u64x2 __attribute__((ext_vector_type(2)));
  typedef const __attribute__((address_space(1))) u64x2 G2;
  Elem<W> r;
#pragma unroll
  for (int h = 0; h < W / 2; ++h) {
    const u64x2 q = __builtin_nontemporal_load((G2*)(p + 2 * h));
    r.v[2 * h] = q.x;
    r.v[2 * h + 1] = q.y;
  }
  return r;
}

template <int W>
__device__ __forceinline__ Elem<W> shfl(const Elem<W>& a, int mask, int lane) {
  Elem<W> r;
#pragma unroll
  for (int k = 0; k < W; ++k) r.v[k] = (u64)xor_move_l((long long)a.v[k], mask, lane);
  return r;
}

// LDS layout of one wave's tile: 64 lane runs of RW sixteen-byte words (K elements),
// rows padded by 16 bytes so that the 16 lanes served together hit distinct banks.
template <int RW>
struct Slice {
  static constexpr int kRowBytes = RW * 16 + 16;
  static constexpr int kBytes = 64 * kRowBytes;
  __device__ static __forceinline__ int word_slot(int wi) { return (wi / RW) * kRowBytes + (wi % RW) * 16; }
};

// Order-keeping butterfly step on lane bit b: the half with the lower lanes stays
// on the left, so after the steps on bits 0..5 every lane holds the product of the
// 64 lanes' values in lane order.
template <int W>
__device__ __forceinline__ Elem<W> ordered_step(const Elem<W>& run, int b, int lane) {
  const Elem<W> other = shfl<W>(run, 1 << b, lane);
  const bool low = ((lane >> b) & 1) == 0;
  return mul<W>(pick<W>(low, run, other), pick<W>(low, other, run));
}

// Every wave is a worker: unit u = (output u / C, chunk u % C), grid-stride.  The
// unit's range is cut into 64 contiguous parts, lane l taking part l, so a lane's
// product is a plain running product and the lanes meet only once, in the
// order-keeping butterfly after the last tile.  A tile is every lane's next K
// elements (one 128-byte line per lane): read from HBM with coalesced 16-byte loads
// (load row q, lane l: word l % R of lane 64/R q + l / R's line, R words per line),
// staged in the wave's LDS slice, and read back as each lane's own K elements; the
// next tile's loads are issued before the current tile is multiplied.  The K
// elements are multiplied as a balanced tree and appended to the lane's product:
// K multiplies per K elements.
template <int W, int K>
__global__ void __launch_bounds__(256) k_ordered(const DevPlan* __restrict__ Pd, const u64* __restrict__ in,
                                                 u64* __restrict__ out, u64* __restrict__ ws) {
  constexpr int kRunWords = K * W / 2;  // sixteen-byte words per lane run
  static_assert(kRunWords * 16 == 128, "a lane run is one 128-byte line");
  constexpr int kJ = 64 / kRunWords;  // lane runs per load row
  using SL = Slice<kRunWords>;
  constexpr int kRowBytes = SL::kRowBytes;
  constexpr int kWaveSlice = SL::kBytes;
  typedef u64 u64x2 __attribute__((ext_vector_type(2)));
  typedef const __attribute__((address_space(1))) u64x2 G2;
  extern __shared__ __align__(16) char lds[];
  const DevPlan& P = *Pd;
  const int lane = (int)(threadIdx.x & 63);
  char* slice = lds + (threadIdx.x >> 6) * kWaveSlice;
  const long long C = P.gsplit, B = P.ord_block, S = P.ord_span;
  const long long units = P.n_out * C;
  const long long nwv = (long long)gridDim.x * (blockDim.x >> 6);
  constexpr int kEw = W / 2;  // sixteen-byte words per element
  // identity words: affine (1, 0); matrix rows (1, 0) and (0, 1)
  auto unit_word = [](int h) -> u64x2 { return h == 0 ? u64x2{1ull, 0ull} : u64x2{0ull, 1ull}; };
  // in load row q this lane fetches word lane % R of the line of lane kJ q + lane / R
  const int lw = lane % kRunWords, lh = lw % kEw;
  for (long long u = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); u < units; u += nwv) {
    const long long o = u / C, c = u - o * C;
    const u64* blk = in + (size_t)o * B * W;
    const long long lo = c * S, hi = (lo + S < B) ? lo + S : B;
    // elements per lane: whole tiles; the last lanes' parts may be short or empty
    const long long part = ((hi - lo + 63) / 64 + K - 1) / K * K;
    const long long le0 = lo + (long long)(lane / kRunWords) * part + lw / kEw;
    const u64* l0 = blk + (size_t)lo * W + lh * 2;  // an address inside the unit, for masked words
    auto fetch = [&](long long t, u64x2* g) {
      const long long lt = le0 + t;
      const u64* lp = blk + (size_t)lt * W + lh * 2;
#pragma unroll
      for (int q = 0; q < kRunWords; ++q) {
        const long long qo = (long long)(q * kJ) * part;  // lanes kJ q + ...: q kJ parts further
        const bool ok = lt < hi - qo;
        g[q] = __builtin_nontemporal_load((G2*)(ok ? lp + (size_t)qo * W : l0));
        if (!ok) g[q] = unit_word(lh);
      }
    };
    u64x2 g[kRunWords];
    fetch(0, g);
    Elem<W> acc = unit<W>();
#pragma unroll 1
    for (long long t = 0; t < part; t += K) {
#pragma unroll
      for (int q = 0; q < kRunWords; ++q) *reinterpret_cast<u64x2*>(slice + SL::word_slot(q * 64 + lane)) = g[q];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
      Elem<W> x[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int h = 0; h < kEw; ++h) {
          const u64x2 v = *reinterpret_cast<const u64x2*>(slice + lane * kRowBytes + (k * kEw + h) * 16);
          x[k].v[2 * h] = v.x;
          x[k].v[2 * h + 1] = v.y;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
      if (t + K < part) fetch(t + K, g);  // in flight while this tile is multiplied
      // the lane's K elements as a balanced tree (adjacent pairs, order kept), so
      // the multiplies of one level are independent of each other
#pragma unroll
      for (int h = 1; h < K; h *= 2) {
#pragma unroll
        for (int j = 0; j + h < K; j += 2 * h) x[j] = mul<W>(x[j], x[j + h]);
      }
      acc = mul<W>(acc, x[0]);
    }
#pragma unroll
    for (int b = 0; b < 6; ++b) acc = ordered_step<W>(acc, b, lane);
    if (lane == 0) {
      u64* dst = C > 1 ? ws + (size_t)u * W : out + (size_t)o * W;
#pragma unroll
      for (int k = 0; k < W; ++k) dst[k] = acc.v[k];
    }
  }
}

// The chunk products of every output, left to right (one lane per output).
template <int W>
__global__ void __launch_bounds__(256) k_ordered_fold(const DevPlan* __restrict__ Pd, const u64* __restrict__ ws,
                                                      u64* __restrict__ out) {
  const DevPlan& P = *Pd;
  const long long C = P.gsplit;
  for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < P.n_out;
       o += (long long)gridDim.x * blockDim.x) {
    Elem<W> acc = unit<W>();
    for (long long c = 0; c < C; ++c) {
      Elem<W> e;
#pragma unroll
      for (int k = 0; k < W; ++k) e.v[k] = ws[(size_t)(o * C + c) * W + k];
      acc = mul<W>(acc, e);
    }
#pragma unroll
    for (int k = 0; k < W; ++k) out[(size_t)o * W + k] = acc.v[k];
  }
}

// Many chunks per output: one wave per output, lane l folds chunks
// [l R, (l + 1) R) in order, then the order-keeping butterfly joins the lanes.
template <int W>
__global__ void __launch_bounds__(256) k_ordered_fold_wave(const DevPlan* __restrict__ Pd, const u64* __restrict__ ws,
                                                           u64* __restrict__ out) {
  const DevPlan& P = *Pd;
  const int lane = (int)(threadIdx.x & 63);
  const long long C = P.gsplit, R = (C + 63) / 64;
  const long long nwv = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long o = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); o < P.n_out; o += nwv) {
    Elem<W> acc = unit<W>();
    const long long c1 = (lane + 1) * R < C ? (lane + 1) * R : C;
    for (long long c = lane * R; c < c1; ++c) {
      Elem<W> e;
#pragma unroll
      for (int k = 0; k < W; ++k) e.v[k] = ws[(size_t)(o * C + c) * W + k];
      acc = mul<W>(acc, e);
    }
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      const Elem<W> other = shfl<W>(acc, 1 << b, lane);
      const bool low = ((lane >> b) & 1) == 0;
      acc = mul<W>(pick<W>(low, acc, other), pick<W>(low, other, acc));
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < W; ++k) out[(size_t)o * W + k] = acc.v[k];
    }
  }
}

// A nest without reducing levels: every element is its own output.
template <int W>
__global__ void __launch_bounds__(256) k_ordered_copy(const DevPlan* __restrict__ Pd, const u64* __restrict__ in,
                                                      u64* __restrict__ out) {
  const DevPlan& P = *Pd;
  const long long n = P.n_out * W;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = in[i];
}

hp_status launch_ordered(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, hipStream_t st) {
  const u64* x = reinterpret_cast<const u64*>(in);
  u64* y = reinterpret_cast<u64*>(out);
  u64* w = reinterpret_cast<u64*>(ws);
  const bool aff = P.dtype == HP_AFFINE64;
  if (P.p == P.depth) {
    const long long n = P.n_out * (aff ? 2 : 4);
    long long g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (aff) hipLaunchKernelGGL(k_ordered_copy<2>, dim3((unsigned)g), dim3(256), 0, st, dP, x, y);
    else hipLaunchKernelGGL(k_ordered_copy<4>, dim3((unsigned)g), dim3(256), 0, st, dP, x, y);
  } else {
    const dim3 grid((unsigned)P.grid), block((unsigned)(P.nw * kWave));
    // a lane run of K elements is one 128-byte line: 8 affine maps or 4 matrices
    const size_t lds = (size_t)P.nw * Slice<8>::kBytes;
    if (aff) hipLaunchKernelGGL((k_ordered<2, 8>), grid, block, lds, st, dP, x, y, w);
    else hipLaunchKernelGGL((k_ordered<4, 4>), grid, block, lds, st, dP, x, y, w);
    if (P.gsplit > 64) {  // long folds: a wave per output
      long long g = (P.n_out + 3) / 4;
      if (g > 4096) g = 4096;
      if (aff) hipLaunchKernelGGL(k_ordered_fold_wave<2>, dim3((unsigned)g), dim3(256), 0, st, dP, w, y);
      else hipLaunchKernelGGL(k_ordered_fold_wave<4>, dim3((unsigned)g), dim3(256), 0, st, dP, w, y);
    } else if (P.gsplit > 1) {
      long long g = (P.n_out + 255) / 256;
      if (g > 4096) g = 4096;
      if (aff) hipLaunchKernelGGL(k_ordered_fold<2>, dim3((unsigned)g), dim3(256), 0, st, dP, w, y);
      else hipLaunchKernelGGL(k_ordered_fold<4>, dim3((unsigned)g), dim3(256), 0, st, dP, w, y);
    }
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return HP_OK;
}

}  // namespace hp
