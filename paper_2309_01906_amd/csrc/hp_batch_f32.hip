// Persistent batched kernels: fp32 nests.
#include "hp_batch_dev.h"

namespace hp {

__global__ void __launch_bounds__(256) k_batch_f32_0(const BatchArgs B) {
  extern __shared__ __align__(16) char lds[];
  batch_run_waves<FloatT<float>, 4, 1, 4, 4>(B, lds);
}

__global__ void __launch_bounds__(256) k_batch_f32_1(const BatchArgs B) {
  extern __shared__ __align__(16) char lds[];
  batch_run_waves<FloatT<float>, 1, 1, 4, 4>(B, lds);
}

__global__ void __launch_bounds__(256) k_batch_f32_2(const BatchArgs B) {
  extern __shared__ __align__(16) char lds[];
  batch_run_waves<FloatT<float>, 4, 1, 4, kMaxDepth>(B, lds);
}

__global__ void __launch_bounds__(256) k_batch_f32_3(const BatchArgs B) {
  extern __shared__ __align__(16) char lds[];
  batch_run_waves<FloatT<float>, 1, 1, 4, kMaxDepth>(B, lds);
}

static hp_status launch_check() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HP_EDEVICE, "batch kernel launch failed: %s", hipGetErrorString(e));
  return HP_OK;
}

hp_status batch_f32_launch(int family, int chunk, const BatchArgs& B, int grid, int nw, size_t lds, hipStream_t st) {
  if (family == FAM_F32_4 && chunk == 4) {
    hipLaunchKernelGGL(k_batch_f32_0, dim3((unsigned)grid), dim3((unsigned)(nw * kWave)), lds, st, B);
    return launch_check();
  }
  if (family == FAM_F32_4 && chunk == 1) {
    hipLaunchKernelGGL(k_batch_f32_1, dim3((unsigned)grid), dim3((unsigned)(nw * kWave)), lds, st, B);
    return launch_check();
  }
  if (family == FAM_F32_8 && chunk == 4) {
    hipLaunchKernelGGL(k_batch_f32_2, dim3((unsigned)grid), dim3((unsigned)(nw * kWave)), lds, st, B);
    return launch_check();
  }
  if (family == FAM_F32_8 && chunk == 1) {
    hipLaunchKernelGGL(k_batch_f32_3, dim3((unsigned)grid), dim3((unsigned)(nw * kWave)), lds, st, B);
    return launch_check();
  }
  return fail(HP_EUNSUPPORTED, "no batch kernel for family %d chunk %d", family, chunk);
}
int batch_f32_occupancy(int family, int chunk, int nw, size_t lds) {
  int nb = 0;
  if (family == FAM_F32_4 && chunk == 4) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_f32_0, nw * kWave, lds) != hipSuccess) return 0;
    return nb;
  }
  if (family == FAM_F32_4 && chunk == 1) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_f32_1, nw * kWave, lds) != hipSuccess) return 0;
    return nb;
  }
  if (family == FAM_F32_8 && chunk == 4) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_f32_2, nw * kWave, lds) != hipSuccess) return 0;
    return nb;
  }
  if (family == FAM_F32_8 && chunk == 1) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_f32_3, nw * kWave, lds) != hipSuccess) return 0;
    return nb;
  }
  return 0;
}

}  // namespace hp
