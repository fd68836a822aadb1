// Stencils tiled through local memory (the paper's second class of multi-level
// algorithms, section 2, and its ghost surfaces, section 4): `steps` five-point
// Jacobi sweeps of a 2-D float array with fixed boundary cells,
//   B[i][j] = c0 A[i][j] + c1 ((A[i-1][j] + A[i+1][j]) + (A[i][j-1] + A[i][j+1])).
// Each workgroup owns a TH x TW output tile.  It reads the tile plus a ghost
// surface `steps` cells wide into LDS once, runs all sweeps there -- the valid
// region shrinks by one cell per sweep -- and writes the tile once: HBM sees one
// read and one write per cell for `steps` sweeps, plus the ghost cells.
#include <hip/hip_runtime.h>

#include <new>

#include "hp_internal.h"

namespace hp {

constexpr int kTH = 32;  // output rows per workgroup
constexpr int kTW = 64;  // output columns per workgroup
constexpr int kThreads = 256;

template <int T>
struct Tile {
  static constexpr int H = kTH + 2 * T;  // rows in LDS (with the ghost surface)
  static constexpr int W = kTW + 2 * T;  // columns in LDS
  static constexpr int P = W + 1;        // row pitch (odd: neighbouring rows in different banks)
  static constexpr int kFloats = H * P;
};

template <int T>
__global__ void __launch_bounds__(kThreads) k_stencil(const float* __restrict__ in, float* __restrict__ out,
                                                      long long R, long long C, float c0, float c1) {
  using G = Tile<T>;
  extern __shared__ float lds[];
  float* buf0 = lds;
  float* buf1 = lds + G::kFloats;
  const long long i0 = (long long)blockIdx.y * kTH - T;  // global row of LDS row 0
  const long long j0 = (long long)blockIdx.x * kTW - T;  // global column of LDS column 0
  const int tid = (int)threadIdx.x;
  // the tile and its ghost surface; cells outside the array are never read by an
  // updated cell (only interior cells change, and their neighbours are inside)
  // all of a thread's loads are issued before the first one is stored to LDS
  constexpr int kLoads = (G::H * G::W + kThreads - 1) / kThreads;
  float v[kLoads];
#pragma unroll
  for (int u = 0; u < kLoads; ++u) {
    const int k = tid + u * kThreads;
    const int r = k / G::W, c = k - (k / G::W) * G::W;
    const long long gi = i0 + r, gj = j0 + c;
    const bool ok = k < G::H * G::W && gi >= 0 && gi < R && gj >= 0 && gj < C;
    v[u] = ok ? in[ok ? gi * C + gj : 0] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < kLoads; ++u) {
    const int k = tid + u * kThreads;
    if (k < G::H * G::W) buf0[(k / G::W) * G::P + (k - (k / G::W) * G::W)] = v[u];
  }
  __syncthreads();
  // interior cells (global 1..R-2, 1..C-2) in tile-local coordinates, clamped to the
  // region, so that the per-cell test is four 32-bit compares
  auto local = [](long long lo_global, long long origin, int extent) -> int {
    const long long v = lo_global - origin;
    return (int)(v < -1 ? -1 : (v > extent ? extent : v));
  };
  const int ilo = local(1, i0, G::H), ihi = local(R - 2, i0, G::H);
  const int jlo = local(1, j0, G::W), jhi = local(C - 2, j0, G::W);
#pragma unroll
  for (int s = 1; s <= T; ++s) {
    const float* src = (s & 1) ? buf0 : buf1;
    float* dst = (s & 1) ? buf1 : buf0;
    // the region still valid after sweep s, in column strips of kRB cells: a thread
    // reads kRB + 2 cells of its column and kRB of each neighbouring column for kRB
    // updates, instead of 5 reads per update
    constexpr int kRB = 4;
    const int wr = G::W - 2 * s;
    const int hr = G::H - 2 * s;
    const int n = ((hr + kRB - 1) / kRB) * wr;
    for (int k = tid; k < n; k += kThreads) {
      const int rb = k / wr;
      const int c = s + (k - rb * wr);
      const int r0 = s + rb * kRB;
      const bool col_in = c >= jlo && c <= jhi;
      float up = src[(r0 - 1) * G::P + c];
      float mid = src[r0 * G::P + c];
#pragma unroll
      for (int d = 0; d < kRB; ++d) {
        const int r = r0 + d;
        if (r < s + hr) {
          const int q = r * G::P + c;
          const float dn = src[q + G::P];
          float v = mid;
          if (col_in && r >= ilo && r <= ihi) v = c0 * mid + c1 * ((up + dn) + (src[q - 1] + src[q + 1]));
          dst[q] = v;
          up = mid;
          mid = dn;
        }
      }
    }
    __syncthreads();
  }
  const float* fin = (T & 1) ? buf1 : buf0;
  for (int k = tid; k < kTH * kTW; k += kThreads) {
    const int r = T + k / kTW, c = T + (k - (k / kTW) * kTW);
    const long long gi = i0 + r, gj = j0 + c;
    if (gi < R && gj < C) out[gi * C + gj] = fin[r * G::P + c];
  }
}

template <int T>
hp_status launch_t(const float* in, float* out, long long R, long long C, float c0, float c1, hipStream_t st) {
  const dim3 grid((unsigned)((C + kTW - 1) / kTW), (unsigned)((R + kTH - 1) / kTH));
  hipLaunchKernelGGL(k_stencil<T>, grid, dim3(kThreads), 2 * Tile<T>::kFloats * sizeof(float), st, in, out, R, C, c0, c1);
  if (hipGetLastError() != hipSuccess) return hp::fail(HP_EDEVICE, "stencil launch failed");
  return HP_OK;
}

}  // namespace hp

using hp::kTH;
using hp::kTW;

struct hp_stencil_s {
  long long rows, cols;
  int steps;
  float c0, c1;
};

extern "C" hp_status hp_stencil_plan(int64_t rows, int64_t cols, int32_t steps, float c0, float c1, hp_stencil_t* out) {
  if (!out) return hp::fail(HP_EINVAL, "null output handle");
  *out = nullptr;
  if (rows < 1 || cols < 1) return hp::fail(HP_EINVAL, "array %lld x %lld is empty", (long long)rows, (long long)cols);
  if (steps < 1 || steps > 8) return hp::fail(HP_EUNSUPPORTED, "steps %d outside [1, 8]", steps);
  if ((rows + kTH - 1) / kTH > 65535 || (cols + kTW - 1) / kTW > 2147483647LL || rows > (int64_t(1) << 62) / cols)
    return hp::fail(HP_EUNSUPPORTED, "array too large for one launch");
  hp_stencil_s* s = new (std::nothrow) hp_stencil_s;
  if (!s) return hp::fail(HP_ENOMEM, "host allocation failed");
  s->rows = rows;
  s->cols = cols;
  s->steps = steps;
  s->c0 = c0;
  s->c1 = c1;
  *out = s;
  return HP_OK;
}

extern "C" hp_status hp_stencil_run(hp_stencil_t s, const float* d_in, float* d_out, void* stream) {
  if (!s || !d_in || !d_out) return hp::fail(HP_EINVAL, "null argument");
  const uintptr_t a = reinterpret_cast<uintptr_t>(d_in), b = reinterpret_cast<uintptr_t>(d_out);
  const uintptr_t bytes = (uintptr_t)(s->rows * s->cols) * sizeof(float);
  if (a < b + bytes && b < a + bytes) return hp::fail(HP_EINVAL, "input and output overlap");
  if ((a & 3u) || (b & 3u)) return hp::fail(HP_EINVAL, "arrays must be 4-byte aligned");
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const long long R = s->rows, C = s->cols;
  switch (s->steps) {
    case 1: return hp::launch_t<1>(d_in, d_out, R, C, s->c0, s->c1, st);
    case 2: return hp::launch_t<2>(d_in, d_out, R, C, s->c0, s->c1, st);
    case 3: return hp::launch_t<3>(d_in, d_out, R, C, s->c0, s->c1, st);
    case 4: return hp::launch_t<4>(d_in, d_out, R, C, s->c0, s->c1, st);
    case 5: return hp::launch_t<5>(d_in, d_out, R, C, s->c0, s->c1, st);
    case 6: return hp::launch_t<6>(d_in, d_out, R, C, s->c0, s->c1, st);
    case 7: return hp::launch_t<7>(d_in, d_out, R, C, s->c0, s->c1, st);
    default: return hp::launch_t<8>(d_in, d_out, R, C, s->c0, s->c1, st);
  }
}

extern "C" hp_status hp_stencil_destroy(hp_stencil_t s) {
  delete s;
  return HP_OK;
}
