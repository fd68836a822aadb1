// Nest kernels for int32 inputs on (value, index) pairs: any nest up to depth 8 and
// 8 segments (NS = KD = 8), and a copy bounded like the segmented kernel (depth <= 4,
// <= 3 segments: NS = 3, KD = 4) whose per-level state takes fewer registers.
#include "hp_nest.h"

namespace hp {

template <int C, int NS, int KD>
__global__ void __launch_bounds__(1024) k_nest_i32_deep(const DevPlan* __restrict__ Pd, const int32_t* __restrict__ in,
                                                   void* __restrict__ out, unsigned char* __restrict__ ws) {
  extern __shared__ __align__(16) char lds[];
  const DevPlan& P = *Pd;
  wg_run<IntT, C, NS, 4, KD, false, false, false>(P, in, out, ws, logical_group(P, blockIdx.x), lds);
}

hp_status launch_nest_i32_deep(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds, hipStream_t st) {
  const dim3 grid((unsigned int)P.grid), block((unsigned int)(P.nw * kWave));
  const int32_t* x = reinterpret_cast<const int32_t*>(in);
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  if (P.depth <= 4 && P.nseg <= 3) {
    if (P.chunk == 4) hipLaunchKernelGGL((k_nest_i32_deep<4, 3, 4>), grid, block, lds, st, dP, x, out, w);
    else hipLaunchKernelGGL((k_nest_i32_deep<1, 3, 4>), grid, block, lds, st, dP, x, out, w);
  } else {
    if (P.chunk == 4) hipLaunchKernelGGL((k_nest_i32_deep<4, kMaxDepth, kMaxDepth>), grid, block, lds, st, dP, x, out, w);
    else hipLaunchKernelGGL((k_nest_i32_deep<1, kMaxDepth, kMaxDepth>), grid, block, lds, st, dP, x, out, w);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return HP_OK;
}

}  // namespace hp
