// Persistent batched kernels: int32 nests with up to three segments, depth <= 4.  One
// segment: one 64-bit key per lane (as the single-nest kernels; an ARG level then sees
// 32-bit input values).  Two or three: (value, index) pairs, so that an ARG level over
// int64 sums runs in the same launch as the other served nests of its depth.
#include "hp_batch_dev.h"

namespace hp {

__global__ void __launch_bounds__(256) k_batch_i32_0(const BatchArgs B) {
  extern __shared__ __align__(16) char lds[];
  batch_run_waves<IntK, 4, 1, 4, 4>(B, lds);
}

__global__ void __launch_bounds__(256) k_batch_i32_1(const BatchArgs B) {
  extern __shared__ __align__(16) char lds[];
  batch_run_waves<IntK, 1, 1, 4, 4>(B, lds);
}

__global__ void __launch_bounds__(256) k_batch_i32_2(const BatchArgs B) {
  extern __shared__ __align__(16) char lds[];
  batch_run_waves<IntT, 4, 3, 4, 4>(B, lds);
}

__global__ void __launch_bounds__(256) k_batch_i32_3(const BatchArgs B) {
  extern __shared__ __align__(16) char lds[];
  batch_run_waves<IntT, 1, 3, 4, 4>(B, lds);
}

static hp_status launch_check() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HP_EDEVICE, "batch kernel launch failed: %s", hipGetErrorString(e));
  return HP_OK;
}

hp_status batch_i32_launch(int family, int chunk, const BatchArgs& B, int grid, int nw, size_t lds, hipStream_t st) {
  if (family == FAM_I32_FLAT && chunk == 4) {
    hipLaunchKernelGGL(k_batch_i32_0, dim3((unsigned)grid), dim3((unsigned)(nw * kWave)), lds, st, B);
    return launch_check();
  }
  if (family == FAM_I32_FLAT && chunk == 1) {
    hipLaunchKernelGGL(k_batch_i32_1, dim3((unsigned)grid), dim3((unsigned)(nw * kWave)), lds, st, B);
    return launch_check();
  }
  if (family == FAM_I32_SEG && chunk == 4) {
    hipLaunchKernelGGL(k_batch_i32_2, dim3((unsigned)grid), dim3((unsigned)(nw * kWave)), lds, st, B);
    return launch_check();
  }
  if (family == FAM_I32_SEG && chunk == 1) {
    hipLaunchKernelGGL(k_batch_i32_3, dim3((unsigned)grid), dim3((unsigned)(nw * kWave)), lds, st, B);
    return launch_check();
  }
  return fail(HP_EUNSUPPORTED, "no batch kernel for family %d chunk %d", family, chunk);
}
int batch_i32_occupancy(int family, int chunk, int nw, size_t lds) {
  int nb = 0;
  if (family == FAM_I32_FLAT && chunk == 4) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_i32_0, nw * kWave, lds) != hipSuccess) return 0;
    return nb;
  }
  if (family == FAM_I32_FLAT && chunk == 1) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_i32_1, nw * kWave, lds) != hipSuccess) return 0;
    return nb;
  }
  if (family == FAM_I32_SEG && chunk == 4) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_i32_2, nw * kWave, lds) != hipSuccess) return 0;
    return nb;
  }
  if (family == FAM_I32_SEG && chunk == 1) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_i32_3, nw * kWave, lds) != hipSuccess) return 0;
    return nb;
  }
  return 0;
}

}  // namespace hp
