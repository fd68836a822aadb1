// Butterfly steps across the lanes of a wave64 (gfx950), one lane-index bit at a
// time: after the step on bit b every lane holds op(own value, value of lane ^ 2^b).
//
// Moves by bit:
//   b = 0, 1  DPP quad_perm [1,0,3,2] / [2,3,0,1]: the exact xor partner;
//   b = 2, 3  row_half_mirror / row_mirror (lane i <- lane 7 - i within 8 lanes,
//             15 - i within 16) when the value is already the same on every lane
//             that differs from this one only in bits below b: the mirror lane then
//             holds the xor partner's value.  Otherwise row_shr / row_shl and a
//             select give the exact partner;
//   b = 4, 5  v_permlane16_swap / v_permlane32_swap of the value with itself: the
//             first result holds, on the upper row (half), the lower row's (half's)
//             values and the second the upper's on the lower one.  When the value is
//             uniform within rows (halves) the two results are the two sides of the
//             step, and op(first, second) needs no select.
// Every op used with these steps is symmetric in its operands (integer sum, min,
// max, and the float pair merge), so both partners of a step compute the same bits
// and the choice of move never changes a result.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hp {

// DPP controls
constexpr int kDppQuad1032 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kDppQuad2301 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
constexpr int kDppRowShr4 = 0x114, kDppRowShl4 = 0x104;
constexpr int kDppRowShr8 = 0x118, kDppRowShl8 = 0x108;

template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

// The partner's value for one 32-bit word.  B is the lane bit; uni: the word is the
// same on lanes that differ only in bits below B.
template <int B>
__device__ __forceinline__ int partner32(int v, bool uni, int lane) {
  if constexpr (B == 0) {
    return dpp<kDppQuad1032>(v);
  } else if constexpr (B == 1) {
    return dpp<kDppQuad2301>(v);
  } else if constexpr (B == 2) {
    if (uni) return dpp<kDppHalfMirror>(v);
    const int dn = dpp<kDppRowShr4>(v), up = dpp<kDppRowShl4>(v);
    return (lane & 4) ? dn : up;
  } else if constexpr (B == 3) {
    if (uni) return dpp<kDppMirror>(v);
    const int dn = dpp<kDppRowShr8>(v), up = dpp<kDppRowShl8>(v);
    return (lane & 8) ? dn : up;
  } else if constexpr (B == 4) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16) ? (int)r[0] : (int)r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32) ? (int)r[0] : (int)r[1];
  }
}

// Both sides of a step on bit 4 or 5 for a word that is uniform below that bit:
// (lower row's value, upper row's value) on every lane.
template <int B>
__device__ __forceinline__ void sides32(int v, int& lo_side, int& hi_side) {
  static_assert(B == 4 || B == 5, "sides32 is for the permlane steps");
  if constexpr (B == 4) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    lo_side = (int)r[0];
    hi_side = (int)r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    lo_side = (int)r[0];
    hi_side = (int)r[1];
  }
}

}  // namespace hp
