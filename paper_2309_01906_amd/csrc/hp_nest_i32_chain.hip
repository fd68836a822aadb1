// Int32 nests whose reducing levels are a chain of single-level segments (two or
// three), each with its own operator -- e.g. sum over j of max over k of argmin over
// l: the recursive reduction of section 2 with a different operator on each level.
//
// The general kernels walk any plan through a runtime odometer; this one is built
// for the chain's fixed shape, so the per-strip work is a few instructions:
//   innermost level L (lanes x 16-byte chunks x F <= 4 strips, operator fixed at
//     compile time): F chunk loads per lane, reduced in 32 bits per chunk and into
//     one 64-bit key (IntK), then a butterfly over L's lanes;
//   middle level M (lanes x strips): each strip's L result is merged into M's key
//     (its operator a uniform branch), and the loads of the next strip are issued
//     before the current strip is combined;
//   outer level Q (three-level chains; workgroup, wave and lane units): M's results
//     merged the same way.
// The last level's lanes, waves (LDS) and workgroups (partials and the fold kernel)
// are combined as in the general kernels.  The planner picks this kernel only when
// every level divides evenly by its units (no masking), the NONE levels are on the
// grid alone and L and M (in three-level chains) use lanes only.
#include "hp_nest.h"

namespace hp {

template <int OP>
struct OpClass {
  static constexpr bool kSum = OP == HP_OP_SUM;
  static constexpr bool kMin = OP == HP_OP_MIN || OP == HP_OP_ARGMIN;
};

// All-reduce of a key over the lanes of one segment, operator fixed at compile time.
template <int OP>
__device__ __forceinline__ long long chain_lanes(long long a, const DevSeg& S, int lane) {
  const uint32_t vm = S.vmask, uf = S.ufast;
  if (!vm) return a;
  if constexpr (OpClass<OP>::kSum) {
    if (vm & 1u) a = key_sum_step<0>(a, uf & 1u, lane);
    if (vm & 2u) a = key_sum_step<1>(a, uf & 2u, lane);
    if (vm & 4u) a = key_sum_step<2>(a, uf & 4u, lane);
    if (vm & 8u) a = key_sum_step<3>(a, uf & 8u, lane);
    if (vm & 16u) a = key_sum_step<4>(a, uf & 16u, lane);
    if (vm & 32u) a = key_sum_step<5>(a, uf & 32u, lane);
    return a;
  } else {
    return key_minmax<OpClass<OP>::kMin>(a, vm, uf, lane);
  }
}

template <int OPL, int NS>
__global__ void __launch_bounds__(1024) k_nest_i32_chain(const DevPlan* __restrict__ Pd, const int32_t* __restrict__ in,
                                                         void* __restrict__ out, unsigned char* __restrict__ ws) {
  extern __shared__ __align__(16) char lds[];
  const DevPlan& P = *Pd;
  const uint32_t g = logical_group(P, blockIdx.x);
  Thread<4> th;
  th.w = (int)(threadIdx.x >> 6);
  th.lane = (int)(threadIdx.x & 63);
  th.tid = (int)threadIdx.x;
  th.wave = false;
  const int d = P.depth, p = P.p;
  const int iL = d - 1, iM = d - 2, iQ = NS == 3 ? d - 3 : d - 2;
  // this thread's first iteration on every level, and its element / output offsets
  long long base_none = 0, base_o = 0, base_red = 0;
  long long tM0 = 0, tQ0 = 0, tL0 = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if (m < d) {
      const DevLevel& L = P.lv[m];
      const uint32_t ug = g_digit(g, L);
      const uint32_t uw = ((uint32_t)th.w >> L.wsh) & (uint32_t)(L.wf - 1);
      const uint32_t uv = ((uint32_t)th.lane >> L.vsh) & (uint32_t)(L.vf - 1);
      const long long t0 = (long long)(((unsigned long long)ug * L.wf + uw) * L.vf + uv) * L.chunk;
      if (m < p) {
        base_none += t0 * L.stride;
        base_o += t0 * L.ostride;
      } else {
        base_red += t0 * L.stride;
      }
      if (m == iL) tL0 = t0;
      if (m == iM) tM0 = t0;
      if (m == iQ) tQ0 = t0;
    }
  }
  const DevLevel& LL = P.lv[iL];
  const DevLevel& LM = P.lv[iM];
  const DevLevel& LQ = P.lv[iQ];
  const DevSeg& SL = P.seg[P.nseg - 1];
  const DevSeg& SM = P.seg[P.nseg - 2];
  const DevSeg& SQ = P.seg[0];
  const int F = (int)LL.strips;  // 1..4
  const long long ssL = LL.sstride, ssM = LM.sstride, ssQ = LQ.sstride;
  const long long spanL = LL.span, spanM = LM.span, spanQ = LQ.span;
  const long long nM = LM.strips, nQ = NS == 3 ? LQ.strips : 1;
  const bool red_writer = ((th.lane & (int)(P.red_vmask | P.idle_vmask)) == 0) &&
                          ((th.w & (int)(P.red_wmask | P.idle_wmask)) == 0);
  const uint32_t gred = (uint32_t)((unsigned long long)g % (unsigned long long)P.gsplit);
  const int opM = SM.op, opQ = SQ.op;

  int sn[4] = {0, 0, 0, 0};
  long long noff = 0, nout = 0;
  for (long long q = 0; q < P.none_iters; ++q) {
    const int32_t* __restrict__ row = in + base_none + noff + base_red;
    long long accQ = IntK::identity(opQ);
    for (long long sq = 0; sq < nQ; ++sq) {
      const int32_t* __restrict__ rq = row + sq * ssQ;
      long long accM = IntK::identity(opM);
      // loads of strip sm of M, issued one strip ahead of the combine
      i32x4 cur[4], nxt[4] = {};
#pragma unroll
      for (int f = 0; f < 4; ++f)
        if (f < F) cur[f] = load_chunk<i32x4>(rq + f * ssL);
      for (long long sm = 0; sm < nM; ++sm) {
        if (sm + 1 < nM) {
#pragma unroll
          for (int f = 0; f < 4; ++f)
            if (f < F) nxt[f] = load_chunk<i32x4>(rq + (sm + 1) * ssM + f * ssL);
        }
        long long accL = IntK::identity(OPL);
#pragma unroll
        for (int f = 0; f < 4; ++f)
          if (f < F) AddChunk<IntK, 4, OPL>::run(accL, cur[f], tL0 + f * spanL, true);
        accL = chain_lanes<OPL>(accL, SL, th.lane);
        IntK::add(accM, IntK::emit(accL, OPL), tM0 + sm * spanM, opM);
#pragma unroll
        for (int f = 0; f < 4; ++f) cur[f] = nxt[f];
      }
      if constexpr (NS == 3) {
        accM = combine_seg<IntK, 4>(P, SM, accM, th, lds);
        IntK::add(accQ, IntK::emit(accM, opM), tQ0 + sq * spanQ, opQ);
      } else {
        accQ = accM;
      }
    }
    accQ = combine_seg<IntK, 4>(P, SQ, accQ, th, lds);
    const long long o = base_o + nout;
    if (P.gmode == GCOMB_NONE) {
      if (red_writer) store_int(P, out, o, IntK::emit(accQ, opQ));
    } else {
      char* part = reinterpret_cast<char*>(ws) + o * P.gsplit * kSlotBytes;
      if (th.tid == 0) IntK::put_partial(part, gred, accQ, opQ);
    }
    // advance the NONE odometer
    bool carry = true;
#pragma unroll
    for (int m = 3; m >= 0; --m) {
      if (carry && m < p) {
        ++sn[m];
        noff += P.lv[m].sstride;
        nout += P.lv[m].span * P.lv[m].ostride;
        if (sn[m] == P.lv[m].strips) {
          sn[m] = 0;
          noff -= P.lv[m].strips * P.lv[m].sstride;
          nout -= P.lv[m].strips * P.lv[m].span * P.lv[m].ostride;
        } else {
          carry = false;
        }
      }
    }
  }
}

template <int NS>
static void launch_chain(const DevPlan& P, const DevPlan* dP, const int32_t* x, void* out, unsigned char* w,
                         size_t lds, hipStream_t st) {
  const dim3 grid((unsigned int)P.grid), block((unsigned int)(P.nw * kWave));
  switch (P.seg[P.nseg - 1].op) {
    case HP_OP_MIN: hipLaunchKernelGGL((k_nest_i32_chain<HP_OP_MIN, NS>), grid, block, lds, st, dP, x, out, w); break;
    case HP_OP_MAX: hipLaunchKernelGGL((k_nest_i32_chain<HP_OP_MAX, NS>), grid, block, lds, st, dP, x, out, w); break;
    case HP_OP_ARGMIN:
      hipLaunchKernelGGL((k_nest_i32_chain<HP_OP_ARGMIN, NS>), grid, block, lds, st, dP, x, out, w);
      break;
    case HP_OP_ARGMAX:
      hipLaunchKernelGGL((k_nest_i32_chain<HP_OP_ARGMAX, NS>), grid, block, lds, st, dP, x, out, w);
      break;
    default: hipLaunchKernelGGL((k_nest_i32_chain<HP_OP_SUM, NS>), grid, block, lds, st, dP, x, out, w); break;
  }
}

hp_status launch_nest_i32_chain(const DevPlan& P, const DevPlan* dP, const void* in, void* out, void* ws, size_t lds,
                                hipStream_t st) {
  const int32_t* x = reinterpret_cast<const int32_t*>(in);
  unsigned char* w = reinterpret_cast<unsigned char*>(ws);
  if (P.nseg == 3) launch_chain<3>(P, dP, x, out, w, lds, st);
  else launch_chain<2>(P, dP, x, out, w, lds, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HP_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return HP_OK;
}

}  // namespace hp
