// Calibration: a plain streaming read of a buffer (no nesting, no compensation), the
// ceiling the reduction kernels are compared with on this device.
#include <hip/hip_runtime.h>

#include "hp_internal.h"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) f32x4 GF4;

// The buffer is cut into blocks of U*256 sixteen-byte words (16 KiB for U = 4);
// workgroup b reads blocks b, b + grid, ..., thread t the words u*256 + t of a block
// (U nontemporal loads in flight, each one 4 KiB contiguous per workgroup), adds
// them, and writes one float per workgroup so that the loads are not removed.
template <int U>
__global__ void __launch_bounds__(256) k_stream_read(const f32x4* __restrict__ in, long long n4, float* __restrict__ out) {
  constexpr long long kBlock = 256LL * U;
  float acc = 0.f;
  for (long long b0 = (long long)blockIdx.x * kBlock; b0 < n4; b0 += (long long)gridDim.x * kBlock) {
    f32x4 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = b0 + u * 256LL + threadIdx.x;
      x[u] = __builtin_nontemporal_load((GF4*)(in + (i < n4 ? i : b0)));
      if (!(i < n4)) x[u] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += (x[u].x + x[u].y) + (x[u].z + x[u].w);
  }
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

}  // namespace

extern "C" hp_status hp_stream_read(const void* d_in, size_t bytes, float* d_out, int32_t grid, void* stream) {
  if (!d_in || !d_out) return hp::fail(HP_EINVAL, "null pointer");
  if ((reinterpret_cast<uintptr_t>(d_in) & 15u) || (bytes & 15u))
    return hp::fail(HP_EINVAL, "input and size must be multiples of 16 bytes");
  if (grid < 1 || grid > 65536) return hp::fail(HP_EINVAL, "grid %d outside [1, 65536]", grid);
  hipLaunchKernelGGL(k_stream_read<4>, dim3((unsigned)grid), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<const f32x4*>(d_in), (long long)(bytes / 16), d_out);
  if (hipGetLastError() != hipSuccess) return hp::fail(HP_EDEVICE, "launch failed");
  return HP_OK;
}

namespace {

// The XCD (accelerator complex die) each workgroup runs on, read from the
// hardware register XCC_ID (bits 3:0): thread 0 of workgroup b writes it to out[b].
__global__ void __launch_bounds__(1024) k_xcd_ids(int32_t* __restrict__ out) {
  const uint32_t id = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);  // hwreg(HW_REG_XCC_ID, 0, 4)
  if (threadIdx.x == 0) out[blockIdx.x] = (int32_t)(id & 0xFu);
}

}  // namespace

extern "C" hp_status hp_xcd_ids(int32_t* d_out, int32_t grid, int32_t threads, size_t lds_bytes, void* stream) {
  if (!d_out) return hp::fail(HP_EINVAL, "null output");
  if (grid < 1 || grid > (1 << 20)) return hp::fail(HP_EINVAL, "grid %d outside [1, 2^20]", grid);
  if (threads < 64 || threads > 1024 || threads % 64) return hp::fail(HP_EINVAL, "threads %d not 64..1024 in 64s", threads);
  if (lds_bytes > 65536) return hp::fail(HP_EINVAL, "lds_bytes %zu above 64 KiB", lds_bytes);
  hipLaunchKernelGGL(k_xcd_ids, dim3((unsigned)grid), dim3((unsigned)threads), lds_bytes,
                     reinterpret_cast<hipStream_t>(stream), d_out);
  if (hipGetLastError() != hipSuccess) return hp::fail(HP_EDEVICE, "launch failed");
  return HP_OK;
}
