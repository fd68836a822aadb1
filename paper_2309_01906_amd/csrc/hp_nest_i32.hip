// Nest kernels for int32 inputs: one reducing segment, depth <= 4.
#include "hp_nest.h"

namespace hp {

template <int C>
__global__ void __launch_bounds__(1024) k_nest_i32_flat(const DevPlan* __restrict__ Pd, const int32_t* __restrict__ in,
                                                   void* __restrict__ out, unsigned char* __restrict__ ws) {
  extern __shared__ __align__(16) char lds[];
  const DevPlan& P = *Pd;
  wg_run<IntK, C, 1, 8, 4>(P, in, out, ws, logical_group(P, blockIdx.x), lds);
}

hp_status launch_nest_i32_flat(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds, hipStream_t st) {
  const dim3 grid((unsigned int)P.grid), block((unsigned int)(P.nw * kWave));
  const int32_t* x = reinterpret_cast<const int32_t*>(in);
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  if (P.chunk == 4) hipLaunchKernelGGL(k_nest_i32_flat<4>, grid, block, lds, st, dP, x, out, w);
  else hipLaunchKernelGGL(k_nest_i32_flat<1>, grid, block, lds, st, dP, x, out, w);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return HP_OK;
}

hp_status launch_nest_i32_seg(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds, hipStream_t st);
hp_status launch_nest_i32_deep(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds, hipStream_t st);
hp_status launch_nest_i32_chain(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds,
                                hipStream_t st);

// one segment and depth <= 4; a chain of two or three single-level segments; two or
// three segments and depth <= 4; anything else
hp_status launch_nest_i32(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds, hipStream_t st) {
  if (P.kernel == HP_KERNEL_INT_FLAT) return launch_nest_i32_flat(P, dP, in, out, ws, lds, st);
  if (P.kernel == HP_KERNEL_INT_SEG) return launch_nest_i32_seg(P, dP, in, out, ws, lds, st);
  if (P.kernel == HP_KERNEL_INT_CHAIN) return launch_nest_i32_chain(P, dP, in, out, ws, lds, st);
  return launch_nest_i32_deep(P, dP, in, out, ws, lds, st);
}

}  // namespace hp
