// Stencils tiled through local memory (the paper's second class of multi-level
// algorithms, section 2, and its ghost surfaces, section 4): `steps` five-point
// Jacobi sweeps of a 2-D float array with fixed boundary cells,
//   B[i][j] = c0 A[i][j] + c1 ((A[i-1][j] + A[i+1][j]) + (A[i][j-1] + A[i][j+1])).
// The tiling is repeated on the levels that have local memory: each workgroup owns a
// TH x 64 output tile in LDS (the workgroup level), each lane a column strip of 4
// cells in registers (the lane level).  A launch reads the tile plus a ghost surface
// T cells wide into LDS once, runs T sweeps there -- the valid region shrinks by one
// cell per sweep -- and writes the tile once: HBM sees one read and one write per
// cell for T sweeps, plus the ghost cells.  The tiles are dealt to the XCDs in
// bands, so that the ghost cells neighbouring tiles share come from HBM once into
// the XCD's L2 (the X level's shared cache).  The plan checks the tile against the
// workgroup level's local memory in the level-property table; more sweeps than one
// launch holds run as several launches through a buffer the plan owns.
#include <hip/hip_runtime.h>

#include <new>
#include <type_traits>

#include "hp_internal.h"

namespace hp {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTW = 64;  // output columns per workgroup
// threads per workgroup: 8 per output row of the tile (256 for 32 rows, 512 for 64)
constexpr int threads_of(int th) { return 8 * th; }
constexpr int kMaxThreads = threads_of(64);
constexpr int kMaxSweeps = 8;  // sweeps one launch can hold (kernels are instantiated up to this)
// Cells of a column one thread updates per pass.  Strips of 8 and 16 were measured
// within 3 % of 4 at 1 to 8 sweeps (the arithmetic, not the neighbour reads, sets the
// pace), so the shortest is kept.
constexpr int kStrip = 4;

template <int T, int TH>
struct Tile {
  static constexpr int H = TH + 2 * T;   // rows in LDS (with the ghost surface)
  static constexpr int W = kTW + 2 * T;  // columns in LDS
  static constexpr int P = W + 1;        // row pitch (odd: neighbouring rows in different banks)
  static constexpr int kFloats = H * P;
};

// LDS bytes of a tile of th output rows and t sweeps (two ping-pong buffers)
static size_t tile_lds_bytes(int th, int t) {
  return 2u * (size_t)(th + 2 * t) * (size_t)(kTW + 2 * t + 1) * sizeof(float);
}

// One sweep over the region still valid after sweep S, in column strips of kRB
// cells: a thread reads kRB + 2 cells of its column and kRB of each neighbouring
// column for kRB updates, instead of 5 reads per update.  EDGE: the tile touches the
// array's boundary, so each cell is tested against the interior range; an interior
// tile (every workgroup but those on the array's rim) skips the tests.
template <int S, int H, int W, int PITCH, int kRB, int NT, bool EDGE>
__device__ __forceinline__ void sweep(const float* __restrict__ src, float* __restrict__ dst, int tid, float c0,
                                      float c1, int ilo, int ihi, int jlo, int jhi) {
  constexpr int wr = W - 2 * S;
  constexpr int hr = H - 2 * S;
  constexpr int nfull = hr / kRB;  // strips of kRB whole rows
  constexpr int rem = hr - nfull * kRB;
  constexpr int n = (nfull + (rem ? 1 : 0)) * wr;
  for (int k = tid; k < n; k += NT) {
    const int rb = k / wr;
    const int c = S + (k - rb * wr);
    const int r0 = S + rb * kRB;
    const int rows = (rem && rb == nfull) ? rem : kRB;
    const bool col_in = !EDGE || (c >= jlo && c <= jhi);
    const float* q0 = src + r0 * PITCH + c;
    float* d0 = dst + r0 * PITCH + c;
    float up = q0[-PITCH];
    float mid = q0[0];
#pragma unroll
    for (int d = 0; d < kRB; ++d) {
      if (d < rows) {
        const float dn = q0[(d + 1) * PITCH];
        float v = c0 * mid + c1 * ((up + dn) + (q0[d * PITCH - 1] + q0[d * PITCH + 1]));
        if (EDGE && !(col_in && r0 + d >= ilo && r0 + d <= ihi)) v = mid;
        d0[d * PITCH] = v;
        up = mid;
        mid = dn;
      }
    }
  }
}

// The tile a workgroup works on.  Workgroup b runs on the XCD b mod 8 selects (the
// dispatcher deals consecutive workgroups round-robin over the 8 XCDs, from a start
// that varies between launches, so the workgroups sharing b mod 8 share an XCD);
// those workgroups take one contiguous run of tiles in row-major tile order -- a band
// of the array -- so the ghost cells that neighbouring tiles both read are fetched
// from HBM once into that XCD's L2 (the shared cache of the X level).  Without XCD
// dealing, tile = b.
__device__ __forceinline__ uint32_t stencil_tile(uint32_t b, uint32_t nt, bool xcd) {
  if (!xcd) return b;
  const uint32_t x = b & 7u, k = b >> 3, q = nt >> 3, r = nt & 7u;
  return x * q + (x < r ? x : r) + k;
}

template <int T, int TH>
__global__ void __launch_bounds__(threads_of(TH)) k_stencil(const float* __restrict__ in, float* __restrict__ out,
                                                      long long R, long long C, uint32_t ntc, uint32_t nt, int xcd,
                                                      int off32, int vec4, float c0, float c1) {
  using G = Tile<T, TH>;
  constexpr int kThreads = threads_of(TH);
  extern __shared__ float lds[];
  float* buf0 = lds;
  float* buf1 = lds + G::kFloats;
  const uint32_t tile = stencil_tile(blockIdx.x, nt, xcd != 0);
  const uint32_t ty = tile / ntc, tx = tile - ty * ntc;
  const long long i0 = (long long)ty * TH - T;   // global row of LDS row 0
  const long long j0 = (long long)tx * kTW - T;  // global column of LDS column 0
  const int tid = (int)threadIdx.x;
  // the tile and its ghost surface; cells outside the array are never read by an
  // updated cell (only interior cells change, and their neighbours are inside)
  // all of a thread's loads are issued before the first one is stored to LDS
  // A tile whose ghost surface lies inside the array (all but the rim) needs no bounds
  // tests and addresses its cells with 32-bit offsets from the tile's first cell
  // (off32: the host found rows x columns of any tile within 32 bits).
  constexpr int kLoads = (G::H * G::W + kThreads - 1) / kThreads;
  float v[kLoads];
  const bool whole = off32 && i0 >= 0 && j0 >= 0 && i0 + G::H <= R && j0 + G::W <= C;
  if (whole && vec4) {
    // 16-byte loads: each row of the tile from its first 4-aligned column on (rows
    // are 4-aligned when C is a multiple of 4); the words left and right of the tile
    // are dropped, and the last vector of a row ends at most at column C - 1
    constexpr int kSh = (4 - T % 4) % 4;         // j0 mod 4 (j0 = 64 tx - T)
    constexpr int kN4 = (kSh + G::W + 3) / 4;    // vectors per row
    constexpr int kV = (G::H * kN4 + kThreads - 1) / kThreads;
    typedef const __attribute__((address_space(1))) f32x4 GV;
    const float* __restrict__ base = in + (i0 * C + (j0 - kSh));
    const uint32_t cu = (uint32_t)C;
    f32x4 q[kV];
#pragma unroll
    for (int u = 0; u < kV; ++u) {
      const int k = tid + u * kThreads;
      const int r = k / kN4, c4 = k - (k / kN4) * kN4;
      if (u + 1 < kV || k < G::H * kN4) q[u] = *(GV*)(base + (uint32_t)r * cu + 4u * (uint32_t)c4);
    }
#pragma unroll
    for (int u = 0; u < kV; ++u) {
      const int k = tid + u * kThreads;
      const int r = k / kN4, c4 = k - (k / kN4) * kN4;
      if (u + 1 < kV || k < G::H * kN4) {
        float* row = buf0 + r * G::P;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = 4 * c4 - kSh + e;
          if (c >= 0 && c < G::W) row[c] = q[u][e];
        }
      }
    }
  } else if (whole) {
    const float* __restrict__ base = in + (i0 * C + j0);
    const uint32_t cu = (uint32_t)C;
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int k = tid + u * kThreads;
      const int r = k / G::W, c = k - (k / G::W) * G::W;
      if (u + 1 < kLoads || k < G::H * G::W) v[u] = base[(uint32_t)r * cu + (uint32_t)c];
    }
  } else {
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int k = tid + u * kThreads;
      const int r = k / G::W, c = k - (k / G::W) * G::W;
      const long long gi = i0 + r, gj = j0 + c;
      const bool ok = k < G::H * G::W && gi >= 0 && gi < R && gj >= 0 && gj < C;
      v[u] = ok ? in[ok ? gi * C + gj : 0] : 0.f;
    }
  }
  if (!(whole && vec4)) {
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int k = tid + u * kThreads;
      if (k < G::H * G::W) buf0[(k / G::W) * G::P + (k - (k / G::W) * G::W)] = v[u];
    }
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
  // every cell any sweep updates is interior: rows 1..H-2 and columns 1..W-2 of the tile
  const bool edge = !(ilo <= 1 && ihi >= G::H - 2 && jlo <= 1 && jhi >= G::W - 2);
  auto run = [&](auto S_) {
    constexpr int S = decltype(S_)::value;
    const float* src = (S & 1) ? buf0 : buf1;
    float* dst = (S & 1) ? buf1 : buf0;
    if (edge) sweep<S, G::H, G::W, G::P, kStrip, kThreads, true>(src, dst, tid, c0, c1, ilo, ihi, jlo, jhi);
    else sweep<S, G::H, G::W, G::P, kStrip, kThreads, false>(src, dst, tid, c0, c1, ilo, ihi, jlo, jhi);
    __syncthreads();
  };
  static_assert(T >= 1 && T <= kMaxSweeps, "sweeps per launch");
  run(std::integral_constant<int, 1>{});
  if constexpr (T >= 2) run(std::integral_constant<int, 2>{});
  if constexpr (T >= 3) run(std::integral_constant<int, 3>{});
  if constexpr (T >= 4) run(std::integral_constant<int, 4>{});
  if constexpr (T >= 5) run(std::integral_constant<int, 5>{});
  if constexpr (T >= 6) run(std::integral_constant<int, 6>{});
  if constexpr (T >= 7) run(std::integral_constant<int, 7>{});
  if constexpr (T >= 8) run(std::integral_constant<int, 8>{});
  const float* fin = (T & 1) ? buf1 : buf0;
  if (off32 && vec4 && i0 + T + TH <= R && j0 + T + kTW <= C) {
    // 16-byte stores: the output tile's rows start at column 64 tx
    typedef __attribute__((address_space(1))) f32x4 GVW;
    float* __restrict__ base = out + ((i0 + T) * C + (j0 + T));
    const uint32_t cu = (uint32_t)C;
    static_assert((TH * kTW / 4) % kThreads == 0, "whole passes over the output tile");
#pragma unroll
    for (int u = 0; u < TH * kTW / 4 / kThreads; ++u) {
      const int k = tid + u * kThreads;
      const int r = k / (kTW / 4), c = 4 * (k - (k / (kTW / 4)) * (kTW / 4));
      const float* src = fin + (r + T) * G::P + c + T;
      *(GVW*)(base + (uint32_t)r * cu + (uint32_t)c) = f32x4{src[0], src[1], src[2], src[3]};
    }
  } else if (off32 && i0 + T + TH <= R && j0 + T + kTW <= C) {
    float* __restrict__ base = out + ((i0 + T) * C + (j0 + T));
    const uint32_t cu = (uint32_t)C;
    static_assert((TH * kTW) % kThreads == 0, "whole passes over the output tile");
#pragma unroll
    for (int u = 0; u < TH * kTW / kThreads; ++u) {
      const int k = tid + u * kThreads;
      const int r = k / kTW, c = k - (k / kTW) * kTW;
      base[(uint32_t)r * cu + (uint32_t)c] = fin[(r + T) * G::P + c + T];
    }
  } else {
    for (int k = tid; k < TH * kTW; k += kThreads) {
      const int r = T + k / kTW, c = T + (k - (k / kTW) * kTW);
      const long long gi = i0 + r, gj = j0 + c;
      if (gi < R && gj < C) out[gi * C + gj] = fin[r * G::P + c];
    }
  }
}

template <int T, int TH>
hp_status launch_t(const float* in, float* out, long long R, long long C, bool xcd, float c0, float c1,
                   hipStream_t st) {
  const uint32_t ntc = (uint32_t)((C + kTW - 1) / kTW), ntr = (uint32_t)((R + TH - 1) / TH);
  const uint32_t nt = ntc * ntr;
  constexpr size_t lds = 2 * Tile<T, TH>::kFloats * sizeof(float);
  // every offset within one tile (rows x columns with the widest ghost surface) fits 32 bits
  const int off32 = (unsigned long long)C * (TH + 2 * kMaxSweeps) + kTW + 2 * kMaxSweeps < (1ull << 32) ? 1 : 0;
  // 16-byte loads and stores when every row starts 16-byte aligned
  const int vec4 = (C % 4 == 0 && (reinterpret_cast<uintptr_t>(in) & 15u) == 0 &&
                    (reinterpret_cast<uintptr_t>(out) & 15u) == 0) ? 1 : 0;
  hipLaunchKernelGGL((k_stencil<T, TH>), dim3(nt), dim3(threads_of(TH)), lds, st, in, out, R, C, ntc, nt, xcd ? 1 : 0,
                     off32, vec4, c0, c1);
  if (hipGetLastError() != hipSuccess) return hp::fail(HP_EDEVICE, "stencil launch failed");
  return HP_OK;
}

template <int TH>
hp_status launch_th(int t, const float* in, float* out, long long R, long long C, bool xcd, float c0, float c1,
                    hipStream_t st) {
  switch (t) {
    case 1: return launch_t<1, TH>(in, out, R, C, xcd, c0, c1, st);
    case 2: return launch_t<2, TH>(in, out, R, C, xcd, c0, c1, st);
    case 3: return launch_t<3, TH>(in, out, R, C, xcd, c0, c1, st);
    case 4: return launch_t<4, TH>(in, out, R, C, xcd, c0, c1, st);
    case 5: return launch_t<5, TH>(in, out, R, C, xcd, c0, c1, st);
    case 6: return launch_t<6, TH>(in, out, R, C, xcd, c0, c1, st);
    case 7: return launch_t<7, TH>(in, out, R, C, xcd, c0, c1, st);
    default: return launch_t<8, TH>(in, out, R, C, xcd, c0, c1, st);
  }
}

}  // namespace hp

using hp::kTW;

struct hp_stencil_s {
  long long rows, cols;
  int steps;
  float c0, c1;
  int tile_rows;     // output rows per workgroup tile (32 or 64)
  bool xcd;          // tiles dealt to XCDs in bands
  int per_launch;    // sweeps per launch (1..8)
  int launches;      // ceil(steps / per_launch); the last launch takes the remainder
  float* tmp;        // rows x cols buffer for the intermediate launches (null for one launch)
  int device;
};

extern "C" hp_status hp_stencil_plan_ex(int64_t rows, int64_t cols, int32_t steps, float c0, float c1,
                                        int32_t tile_rows, int32_t sweeps_per_launch, uint32_t flags,
                                        hp_stencil_t* out) {
  if (!out) return hp::fail(HP_EINVAL, "null output handle");
  *out = nullptr;
  if (rows < 1 || cols < 1) return hp::fail(HP_EINVAL, "array %lld x %lld is empty", (long long)rows, (long long)cols);
  if (steps < 1) return hp::fail(HP_EINVAL, "steps %d < 1", steps);
  if (tile_rows != 0 && tile_rows != 32 && tile_rows != 64)
    return hp::fail(HP_EINVAL, "tile rows %d: 0 (choose), 32 or 64", tile_rows);
  if (flags & ~(uint32_t)HP_STENCIL_NO_XCD) return hp::fail(HP_EINVAL, "unknown stencil flags 0x%x", flags);
  if (sweeps_per_launch < 0 || sweeps_per_launch > hp::kMaxSweeps)
    return hp::fail(HP_EINVAL, "sweeps per launch %d outside [0, %d]", sweeps_per_launch, hp::kMaxSweeps);
  // the workgroup level's local memory, from the level-property table
  hp_level_props lv[8];
  int32_t nl = 0;
  int64_t fill = 0;
  if (hp_level_table(lv, 8, &nl, &fill) != HP_OK) return HP_EDEVICE;
  int64_t lds = 0;
  for (int i = 0; i < nl && i < 8; ++i)
    if (lv[i].scope == HP_SCOPE_W) lds = lv[i].shared_bytes;
  // Sweeps per launch: as many as a launch holds, spread evenly over the launches
  // (each launch is one HBM round trip; the wider ghost surface of more sweeps per
  // launch costs less than a round trip up to 8: 16 sweeps of an 8192 x 8192 array
  // run as 2 launches of 8 in 0.94x the time of 4 launches of 4).
  int t = sweeps_per_launch;
  if (t == 0) {
    const int k = (steps + hp::kMaxSweeps - 1) / hp::kMaxSweeps;
    t = (steps + k - 1) / k;
  }
  // Tile rows: a 64-row tile (512 threads) recomputes fewer ghost cells per output
  // cell -- 24 % extra updates at 8 sweeps instead of 36 % -- but holds 3 workgroups
  // per CU instead of 5.  On an 8192 x 8192 array it is 6-9 % faster from 6 sweeps
  // per launch on and slower below, so it is taken from 6 sweeps when it fits the
  // workgroup's local memory and the array still gives the chip its fill target of
  // workgroups (both from the level-property table).
  int th = tile_rows;
  if (th == 0) {
    const int64_t tiles64 = ((rows + 63) / 64) * ((cols + kTW - 1) / kTW);
    th = (t >= 6 && (int64_t)hp::tile_lds_bytes(64, t) <= lds && tiles64 >= fill) ? 64 : 32;
  }
  if ((int64_t)hp::tile_lds_bytes(th, t) > lds)
    return hp::fail(HP_EUNSUPPORTED, "a %d-row tile with %d sweeps needs %zu bytes of LDS", th, t,
                    hp::tile_lds_bytes(th, t));
  // one workgroup per tile, and a launch holds at most 2^32 - 1 work-items
  const int64_t max_tiles = (int64_t)(0xFFFFFFFFu / (uint32_t)hp::kMaxThreads);
  if (rows > (int64_t(1) << 62) / cols || (rows + th - 1) / th > max_tiles / ((cols + kTW - 1) / kTW))
    return hp::fail(HP_EUNSUPPORTED, "array of %lld x %lld cells needs more tiles than a launch holds",
                    (long long)rows, (long long)cols);
  hp_stencil_s* s = new (std::nothrow) hp_stencil_s;
  if (!s) return hp::fail(HP_ENOMEM, "host allocation failed");
  s->rows = rows;
  s->cols = cols;
  s->steps = steps;
  s->c0 = c0;
  s->c1 = c1;
  s->tile_rows = th;
  s->xcd = !(flags & HP_STENCIL_NO_XCD);
  s->per_launch = t;
  s->launches = (steps + t - 1) / t;
  s->tmp = nullptr;
  s->device = -1;
  if (s->launches > 1) {
    if (hipGetDevice(&s->device) != hipSuccess) {
      delete s;
      return hp::fail(HP_EDEVICE, "no HIP device");
    }
    if (hipMalloc(&s->tmp, (size_t)rows * (size_t)cols * sizeof(float)) != hipSuccess) {
      delete s;
      return hp::fail(HP_ENOMEM, "stencil buffer of %lld x %lld floats", (long long)rows, (long long)cols);
    }
  }
  *out = s;
  return HP_OK;
}

extern "C" hp_status hp_stencil_plan(int64_t rows, int64_t cols, int32_t steps, float c0, float c1, hp_stencil_t* out) {
  return hp_stencil_plan_ex(rows, cols, steps, c0, c1, 0, 0, 0, out);
}

extern "C" hp_status hp_stencil_info(hp_stencil_t s, int32_t* tile_rows, int32_t* tile_cols, int32_t* sweeps_per_launch,
                                     int32_t* launches) {
  if (!s || !tile_rows || !tile_cols || !sweeps_per_launch || !launches) return hp::fail(HP_EINVAL, "null argument");
  *tile_rows = s->tile_rows;
  *tile_cols = kTW;
  *sweeps_per_launch = s->per_launch;
  *launches = s->launches;
  return HP_OK;
}

extern "C" hp_status hp_stencil_run(hp_stencil_t s, const float* d_in, float* d_out, void* stream) {
  if (!s || !d_in || !d_out) return hp::fail(HP_EINVAL, "null argument");
  const uintptr_t a = reinterpret_cast<uintptr_t>(d_in), b = reinterpret_cast<uintptr_t>(d_out);
  const uintptr_t bytes = (uintptr_t)(s->rows * s->cols) * sizeof(float);
  if (a < b + bytes && b < a + bytes) return hp::fail(HP_EINVAL, "input and output overlap");
  if ((a & 3u) || (b & 3u)) return hp::fail(HP_EINVAL, "arrays must be 4-byte aligned");
  if (s->launches > 1) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != s->device)
      return hp::fail(HP_EINVAL, "stencil plan was made on device %d, current device is %d", s->device, dev);
  }
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const long long R = s->rows, C = s->cols;
  // launch j reads the previous launch's result; the last one writes d_out, and
  // counting back from it the launches alternate between d_out and the plan's buffer
  const float* src = d_in;
  int left = s->steps;
  for (int j = 0; j < s->launches; ++j) {
    const int t = left < s->per_launch ? left : s->per_launch;
    float* dst = ((s->launches - 1 - j) % 2 == 0) ? d_out : s->tmp;
    const hp_status r = s->tile_rows == 64 ? hp::launch_th<64>(t, src, dst, R, C, s->xcd, s->c0, s->c1, st)
                                           : hp::launch_th<32>(t, src, dst, R, C, s->xcd, s->c0, s->c1, st);
    if (r != HP_OK) return r;
    src = dst;
    left -= t;
  }
  return HP_OK;
}

extern "C" hp_status hp_stencil_destroy(hp_stencil_t s) {
  if (!s) return HP_OK;
  hp_status r = HP_OK;
  if (s->tmp && hipFree(s->tmp) != hipSuccess) r = hp::fail(HP_EDEVICE, "stencil buffer free failed");
  delete s;
  return r;
}
