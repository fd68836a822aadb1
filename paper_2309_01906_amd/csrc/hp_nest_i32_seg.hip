// Nest kernels for int32 inputs: two or three reducing segments, depth <= 4.
#include "hp_nest.h"

namespace hp {

template <int C>
__global__ void __launch_bounds__(1024) k_nest_i32_seg(const DevPlan* __restrict__ Pd, const int32_t* __restrict__ in,
                                                   void* __restrict__ out, unsigned char* __restrict__ ws) {
  extern __shared__ __align__(16) char lds[];
  const DevPlan& P = *Pd;
  wg_run<IntK, C, 3, 8, 4, false, false, true, false>(P, in, out, ws, logical_group(P, blockIdx.x), lds);
}

hp_status launch_nest_i32_seg(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds, hipStream_t st) {
  const dim3 grid((unsigned int)P.grid), block((unsigned int)(P.nw * kWave));
  const int32_t* x = reinterpret_cast<const int32_t*>(in);
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  if (P.chunk == 4) hipLaunchKernelGGL(k_nest_i32_seg<4>, grid, block, lds, st, dP, x, out, w);
  else hipLaunchKernelGGL(k_nest_i32_seg<1>, grid, block, lds, st, dP, x, out, w);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return HP_OK;
}

}  // namespace hp
