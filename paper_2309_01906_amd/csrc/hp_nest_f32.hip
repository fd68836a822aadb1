// Nest kernels for fp32 inputs (SUM levels, fp32 pair accumulation, fp64 output).
#include "hp_nest.h"

namespace hp {

template <int C, int KD>
__global__ void __launch_bounds__(1024) k_nest_f32(const DevPlan* __restrict__ Pd, const float* __restrict__ in,
                                                   void* __restrict__ out, unsigned char* __restrict__ ws) {
  extern __shared__ __align__(16) char lds[];
  const DevPlan& P = *Pd;
  wg_run<FloatT<float>, C, 1, (C == 1 ? 16 : 8), KD>(P, in, out, ws, logical_group(P, blockIdx.x), lds);
}

// Lean variant for the common streaming case: one strided inner dimension, at
// most 8 waves, depth <= 4.  Only the streaming paths it needs are compiled, so
// it keeps 8 chunk loads per lane in flight within fewer registers.
template <int C>
__global__ void __launch_bounds__(512)
k_nest_f32_lean(const DevPlan* __restrict__ Pd, const float* __restrict__ in, void* __restrict__ out,
               unsigned char* __restrict__ ws) {
  extern __shared__ __align__(16) char lds[];
  const DevPlan& P = *Pd;
  wg_run<FloatT<float>, C, 1, 4, 4, true, false, true, false>(P, in, out, ws, logical_group(P, blockIdx.x), lds);
}

// The same for flat-block plans (blocks that are not a multiple of the vector).
template <int C>
__global__ void __launch_bounds__(512)
k_nest_f32_lean_flat(const DevPlan* __restrict__ Pd, const float* __restrict__ in, void* __restrict__ out,
               unsigned char* __restrict__ ws) {
  extern __shared__ __align__(16) char lds[];
  const DevPlan& P = *Pd;
  wg_run<FloatT<float>, C, 1, 4, 4, true>(P, in, out, ws, logical_group(P, blockIdx.x), lds);
}

hp_status launch_nest_f32(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds, hipStream_t st) {
  const dim3 grid((unsigned int)P.grid), block((unsigned int)(P.nw * kWave));
  const float* x = reinterpret_cast<const float*>(in);
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  if (P.kernel == HP_KERNEL_LEAN) {
    if (P.flat_b) hipLaunchKernelGGL(k_nest_f32_lean_flat<4>, grid, block, lds, st, dP, x, out, w);
    else hipLaunchKernelGGL(k_nest_f32_lean<4>, grid, block, lds, st, dP, x, out, w);
  } else if (P.kernel == HP_KERNEL_GENERIC4) {
    if (P.chunk == 4) hipLaunchKernelGGL((k_nest_f32<4, 4>), grid, block, lds, st, dP, x, out, w);
    else hipLaunchKernelGGL((k_nest_f32<1, 4>), grid, block, lds, st, dP, x, out, w);
  } else {
    if (P.chunk == 4) hipLaunchKernelGGL((k_nest_f32<4, kMaxDepth>), grid, block, lds, st, dP, x, out, w);
    else hipLaunchKernelGGL((k_nest_f32<1, kMaxDepth>), grid, block, lds, st, dP, x, out, w);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return HP_OK;
}

}  // namespace hp
