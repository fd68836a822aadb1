// Plan objects and the single-nest entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "hp_internal.h"

#include "hp_fold.h"

struct hp_plan_s {
  hp::DevPlan dp;        // host copy: launch geometry
  hp::DevPlan* d_dp;     // device copy: read by the kernels, followed by the fold tasks
  hp::FoldTask* d_fold;  // grid combine: the fold kernel's tasks (n_fold of them)
  int n_fold;
  hp_plan_info info;
  void* ws;
  int device;
};

extern "C" hp_status hp_plan(const hp_nest* nest, const hp_level_map* map, uint32_t flags, hp_plan_t* out) {
  if (!out) return hp::fail(HP_EINVAL, "null output handle");
  *out = nullptr;
  hp::Lowered L;
  hp_status s = hp::lower(nest, map, flags, &L);
  if (s != HP_OK) return s;
  hp_plan_s* p = new (std::nothrow) hp_plan_s;
  if (!p) return hp::fail(HP_ENOMEM, "host allocation of the plan failed");
  p->dp = L.dp;
  p->info = L.info;
  p->ws = nullptr;
  p->d_dp = nullptr;
  p->d_fold = nullptr;
  std::vector<hp::FoldTask> folds;
  if (p->dp.kernel != HP_KERNEL_ORDERED) hp::fold_tasks_of(p->dp, 0, folds);  // ordered products fold themselves
  p->n_fold = (int)folds.size();
  const size_t plan_bytes = (sizeof(hp::DevPlan) + 255) / 256 * 256;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return hp::fail(HP_EDEVICE, "no HIP device");
  }
  if (hipMalloc(&p->d_dp, plan_bytes + folds.size() * sizeof(hp::FoldTask)) != hipSuccess) {
    delete p;
    return hp::fail(HP_ENOMEM, "device plan allocation failed");
  }
  p->d_fold = reinterpret_cast<hp::FoldTask*>(reinterpret_cast<unsigned char*>(p->d_dp) + plan_bytes);
  if (hipMemcpy(p->d_dp, &p->dp, sizeof(hp::DevPlan), hipMemcpyHostToDevice) != hipSuccess ||
      (!folds.empty() &&
       hipMemcpy(p->d_fold, folds.data(), folds.size() * sizeof(hp::FoldTask), hipMemcpyHostToDevice) != hipSuccess)) {
    (void)hipFree(p->d_dp);
    delete p;
    return hp::fail(HP_EDEVICE, "device plan upload failed");
  }
  if (p->info.workspace_bytes) {
    if (hipMalloc(&p->ws, p->info.workspace_bytes) != hipSuccess) {
      (void)hipFree(p->d_dp);
      delete p;
      return hp::fail(HP_ENOMEM, "workspace allocation of %zu bytes failed", L.info.workspace_bytes);
    }
    // every run writes all partials before the fold reads them; cleared for tidiness
    if (hipMemset(p->ws, 0, p->info.workspace_bytes) != hipSuccess) {
      (void)hipFree(p->ws);
      (void)hipFree(p->d_dp);
      delete p;
      return hp::fail(HP_EDEVICE, "workspace clear failed");
    }
  }
  *out = p;
  return HP_OK;
}

extern "C" hp_status hp_plan_info_get(hp_plan_t plan, hp_plan_info* info) {
  if (!plan || !info) return hp::fail(HP_EINVAL, "null argument");
  *info = plan->info;
  return HP_OK;
}

extern "C" hp_status hp_run(hp_plan_t plan, const void* d_in, void* d_out, void* stream) {
  if (!plan) return hp::fail(HP_EINVAL, "null plan");
  if (!d_in || !d_out) return hp::fail(HP_EINVAL, "null input or output pointer");
  if (reinterpret_cast<uintptr_t>(d_in) & 15u) return hp::fail(HP_EINVAL, "input not 16-byte aligned");
  const int od = plan->info.out_dtype;
  const uintptr_t oal = (od == HP_AFFINE64 || od == HP_MAT2X2_64) ? 15u : (od == HP_I64 || od == HP_F64) ? 7u : 3u;
  if (reinterpret_cast<uintptr_t>(d_out) & oal) return hp::fail(HP_EINVAL, "output misaligned for its type");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != plan->device)
    return hp::fail(HP_EINVAL, "plan was made on device %d, current device is %d", plan->device, dev);
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hp_status s;
  if (plan->dp.kernel == HP_KERNEL_ORDERED) return hp::launch_ordered(plan->dp, plan->d_dp, d_in, d_out, plan->ws, st);
  switch (plan->dp.dtype) {
    case HP_F32: s = hp::launch_nest_f32(plan->dp, plan->d_dp, d_in, d_out, plan->ws, plan->info.lds_bytes, st); break;
    case HP_BF16: s = hp::launch_nest_bf16(plan->dp, plan->d_dp, d_in, d_out, plan->ws, plan->info.lds_bytes, st); break;
    default: s = hp::launch_nest_i32(plan->dp, plan->d_dp, d_in, d_out, plan->ws, plan->info.lds_bytes, st); break;
  }
  if (s == HP_OK && plan->n_fold)
    s = hp::launch_fold_one(plan->d_dp, plan->d_fold, plan->n_fold, d_out,
                            reinterpret_cast<const unsigned char*>(plan->ws), st);
  return s;
}

extern "C" hp_status hp_destroy(hp_plan_t plan) {
  if (!plan) return HP_OK;
  hp_status s = HP_OK;
  if (plan->ws && hipFree(plan->ws) != hipSuccess) s = hp::fail(HP_EDEVICE, "workspace free failed");
  if (plan->d_dp && hipFree(plan->d_dp) != hipSuccess) s = hp::fail(HP_EDEVICE, "device plan free failed");
  delete plan;
  return s;
}
