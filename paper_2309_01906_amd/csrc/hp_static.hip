// Single-nest reduction that allocates nothing: the plan, the fold tasks and the
// grid-combine partials live in one file-scope device array per GPU.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hp_internal.h"

#include "hp_fold.h"

namespace hp {

// Layout of the array: the device copy of the plan, then the fold tasks, then the
// workgroup partials of a grid-split nest.
constexpr size_t kStaticPlanBytes = 4096;
constexpr size_t kStaticFoldBytes = 1u << 20;
constexpr size_t kStaticBytes = HP_STATIC_SCRATCH_BYTES;
constexpr size_t kStaticWsOffset = kStaticPlanBytes + kStaticFoldBytes;
constexpr size_t kStaticWsBytes = kStaticBytes - kStaticWsOffset;
constexpr long long kStaticMaxFold = (long long)(kStaticFoldBytes / sizeof(FoldTask));
static_assert(sizeof(DevPlan) <= kStaticPlanBytes, "plan does not fit its slot");
static_assert(kStaticBytes > kStaticWsOffset, "scratch too small for its layout");

// Host code must not pass `scratch` itself to a kernel: its device address comes
// from hipGetSymbolAddress, once per device (static_base).
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kStaticMaxDevices = 64;
static void* g_base[kStaticMaxDevices];
static std::mutex g_base_mu;

// The array's address on the current device (looked up on the first call there).
static hp_status static_base(int dev, unsigned char** base) {
  if (dev < 0 || dev >= kStaticMaxDevices) return fail(HP_EUNSUPPORTED, "device %d beyond %d", dev, kStaticMaxDevices);
  std::lock_guard<std::mutex> lock(g_base_mu);
  if (!g_base[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(HP_EDEVICE, "scratch address lookup failed: %s", hipGetErrorString(e));
    g_base[dev] = p;
  }
  *base = reinterpret_cast<unsigned char*>(g_base[dev]);
  return HP_OK;
}

// Copy the plan (a kernel argument, so the launch captures it by value) into the
// array and write the fold tasks that fold_tasks_of would make for it.
__global__ void __launch_bounds__(256) k_static_install(DevPlan P, DevPlan* plan_dst, FoldTask* fold_dst,
                                                         int n_fold) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  constexpr int words = (int)(sizeof(DevPlan) / 4);
  static_assert(sizeof(DevPlan) % 4 == 0, "plan is not a whole number of words");
  if (i < words) reinterpret_cast<uint32_t*>(plan_dst)[i] = reinterpret_cast<const uint32_t*>(&P)[i];
  if (i < n_fold) {
    FoldTask t;
    t.nest = 0;
    if (fold_on_lane(P)) {
      const long long o0 = (long long)i * kWave;
      t.o0 = (int)o0;
      t.n = (int)(P.n_out - o0 < kWave ? P.n_out - o0 : kWave);
      t.wave = 0;
    } else {
      t.o0 = i;
      t.n = 1;
      t.wave = 1;
    }
    fold_dst[i] = t;
  }
}

}  // namespace hp

extern "C" hp_status hp_reduce_static(const hp_nest* nest, const hp_level_map* map, uint32_t flags, const void* d_in,
                                      void* d_out, void* stream) {
  using namespace hp;
  if (!d_in || !d_out) return fail(HP_EINVAL, "null input or output pointer");
  if (reinterpret_cast<uintptr_t>(d_in) & 15u) return fail(HP_EINVAL, "input not 16-byte aligned");
  Lowered L;
  hp_status s = lower(nest, map, flags, &L);
  if (s != HP_OK) return s;
  const DevPlan& P = L.dp;
  const int od = L.info.out_dtype;
  const uintptr_t oal = (od == HP_AFFINE64 || od == HP_MAT2X2_64) ? 15u : (od == HP_I64 || od == HP_F64) ? 7u : 3u;
  if (reinterpret_cast<uintptr_t>(d_out) & oal) return fail(HP_EINVAL, "output misaligned for its type");
  if (L.info.workspace_bytes > kStaticWsBytes)
    return fail(HP_ETOOBIG, "nest needs %zu bytes of workspace; the static scratch holds %zu", L.info.workspace_bytes,
                kStaticWsBytes);
  const long long n_fold = P.kernel == HP_KERNEL_ORDERED ? 0 : fold_task_count(P);
  if (n_fold > kStaticMaxFold)
    return fail(HP_ETOOBIG, "nest needs %lld fold tasks; the static scratch holds %lld", n_fold, kStaticMaxFold);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HP_EDEVICE, "no HIP device");
  unsigned char* base = nullptr;
  s = static_base(dev, &base);
  if (s != HP_OK) return s;
  DevPlan* dP = reinterpret_cast<DevPlan*>(base);
  FoldTask* dF = reinterpret_cast<FoldTask*>(base + kStaticPlanBytes);
  void* ws = L.info.workspace_bytes ? base + kStaticWsOffset : nullptr;
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const long long words = (long long)(sizeof(DevPlan) / 4);
  const long long n_inst = n_fold > words ? n_fold : words;
  hipLaunchKernelGGL(k_static_install, dim3((unsigned)((n_inst + 255) / 256)), dim3(256), 0, st, P, dP, dF,
                     (int)n_fold);
  if (hipGetLastError() != hipSuccess) return fail(HP_EDEVICE, "plan install launch failed");
  if (P.kernel == HP_KERNEL_ORDERED) return launch_ordered(P, dP, d_in, d_out, ws, st);
  switch (P.dtype) {
    case HP_F32: s = launch_nest_f32(P, dP, d_in, d_out, ws, L.info.lds_bytes, st); break;
    case HP_BF16: s = launch_nest_bf16(P, dP, d_in, d_out, ws, L.info.lds_bytes, st); break;
    default: s = launch_nest_i32(P, dP, d_in, d_out, ws, L.info.lds_bytes, st); break;
  }
  if (s == HP_OK && n_fold)
    s = launch_fold_one(dP, dF, (int)n_fold, d_out, reinterpret_cast<const unsigned char*>(ws), st);
  return s;
}
