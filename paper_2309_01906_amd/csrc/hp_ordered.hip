// Ordered products: associative, non-commutative reductions of affine maps and
// 2x2 matrices modulo 2^64 (HP_OP_PROD).  The paper points out that OpenMP
// reductions must be commutative (section 2); here siblings are combined strictly
// in iteration order at every level of the hierarchy:
//   lane    K consecutive elements multiplied in registers (a balanced tree over
//           adjacent pairs, which keeps their order);
//   wave    a xor butterfly in which the lower-lane half always stands on the left,
//           so after log2(64) steps every lane holds the tile's product in order;
//   chunk   tile products appended left to right by the wave;
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

// Every wave is a worker: unit u = (output u / C, chunk u % C), grid-stride.
template <int W, int K>
__global__ void __launch_bounds__(256) k_ordered(const DevPlan* __restrict__ Pd, const u64* __restrict__ in,
                                                 u64* __restrict__ out, u64* __restrict__ ws) {
  const DevPlan& P = *Pd;
  const int lane = (int)(threadIdx.x & 63);
  const long long C = P.gsplit, B = P.ord_block, S = P.ord_span;
  const long long units = P.n_out * C;
  const long long nwv = (long long)gridDim.x * (blockDim.x >> 6);
  constexpr long long kTile = 64LL * K;
  for (long long u = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); u < units; u += nwv) {
    const long long o = u / C, c = u - o * C;
    const u64* blk = in + (size_t)o * B * W;
    const long long lo = c * S, hi = (lo + S < B) ? lo + S : B;
    Elem<W> acc = unit<W>();
    for (long long t = lo; t < hi; t += kTile) {
      // lane run: elements t + lane K + j; past the chunk end the unit element
      Elem<W> x[K];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const long long i = t + (long long)lane * K + j;
        x[j] = load_elem<W>(blk + (size_t)(i < hi ? i : lo) * W);
        if (!(i < hi)) x[j] = unit<W>();
      }
      // the lane's K elements as a balanced tree (adjacent pairs, order kept), so
      // the multiplies of one level are independent of each other
#pragma unroll
      for (int h = 1; h < K; h *= 2) {
#pragma unroll
        for (int j = 0; j + h < K; j += 2 * h) x[j] = mul<W>(x[j], x[j + h]);
      }
      Elem<W> run = x[0];
      // order-keeping butterfly: the half with the lower lanes stays on the left
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const Elem<W> other = shfl<W>(run, 1 << b, lane);
        const bool low = ((lane >> b) & 1) == 0;
        run = mul<W>(pick<W>(low, run, other), pick<W>(low, other, run));
      }
      acc = mul<W>(acc, run);
    }
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
    if (aff) hipLaunchKernelGGL((k_ordered<2, 16>), grid, block, 0, st, dP, x, y, w);
    else hipLaunchKernelGGL((k_ordered<4, 8>), grid, block, 0, st, dP, x, y, w);
    if (P.gsplit > 1) {
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
