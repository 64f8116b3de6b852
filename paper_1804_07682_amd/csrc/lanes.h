// Cross-lane sums of a 64-lane wavefront without the LDS crossbar.  A
// shuffle (ds_bpermute) is an LDS round trip per 32-bit word; DPP moves
// within a row of 16 lanes and gfx950's row swaps take a few VALU cycles.
#pragma once

#include <hip/hip_runtime.h>

namespace gna {

// Word of lane l ^ O, O = 16 or 32: the row swaps exchange rows 1, 3 of one
// operand with rows 0, 2 of the other (O = 16), or the upper half with the
// lower half (O = 32); with the same word in both operands the first result
// holds the partner's word on lanes with bit O set, the second on the rest.
template <int O>
__device__ __forceinline__ unsigned xor_word_rows(unsigned w) {
  const bool upper = (threadIdx.x & O) != 0;
  if constexpr (O == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(w, w, false, false);
    return upper ? r[0] : r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(w, w, false, false);
    return upper ? r[0] : r[1];
  }
}

// Word of a partner lane within a row of 16, by DPP: O = 1, 2 are the
// exchanges l ^ 1, l ^ 2 in each quad; O = 4, 8 are the mirrors within 8
// and 16 lanes, which pair lane l with a lane of the other half, and so give
// the same sum as l ^ O inside a butterfly taken in the order 1, 2, 4, 8
// (after the lower steps every lane of a quad, an octet, holds the same
// partial sum, bit for bit: IEEE addition commutes).
template <int O>
__device__ __forceinline__ unsigned xor_word_dpp(unsigned w) {
  constexpr int ctrl = O == 1 ? 0xB1 : O == 2 ? 0x4E : O == 4 ? 0x141 : 0x140;
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)w, ctrl, 0xf, 0xf, false);
}

template <int O>
__device__ __forceinline__ unsigned xor_word(unsigned w) {
  static_assert(O == 1 || O == 2 || O == 4 || O == 8 || O == 16 || O == 32, "lane offset");
  if constexpr (O >= 16)
    return xor_word_rows<O>(w);
  else
    return xor_word_dpp<O>(w);
}

// The butterfly partner's value (see xor_word_dpp for O = 4, 8: only inside
// an ascending butterfly).
template <int O>
__device__ __forceinline__ double partner(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = xor_word<O>((unsigned)b), hi = xor_word<O>((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int O>
__device__ __forceinline__ float partner(float v) {
  return __uint_as_float(xor_word<O>(__float_as_uint(v)));
}

// x[k] summed over aligned groups of G lanes (G a power of two <= 64), the
// total on every lane of the group: butterfly steps 1, 2, 4, ... in that
// order.  Every lane of the wavefront takes part.
template <class T, int N>
__device__ __forceinline__ void group_sums(T (&x)[N], int G) {
  if (G > 1) {
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] += partner<1>(x[k]);
  }
  if (G > 2) {
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] += partner<2>(x[k]);
  }
  if (G > 4) {
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] += partner<4>(x[k]);
  }
  if (G > 8) {
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] += partner<8>(x[k]);
  }
  if (G > 16) {
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] += partner<16>(x[k]);
  }
  if (G > 32) {
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] += partner<32>(x[k]);
  }
}

// v of the lane that DPP control CTRL selects (0 where the row / bank masks
// disable the lane or the source lane does not exist), both halves moved.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ double dpp_take(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, BANK_MASK, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK,
                                             BANK_MASK, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}

// Sum of v over the wavefront's 64 lanes, complete in lane 63: a prefix sum
// within each row of 16 lanes (shifts by 1, 2, 3, then 4 and 8 on the upper
// banks), then row 0's total broadcast into rows 1 and 3 and lane 31's into
// rows 2 and 3.  Called with every lane of the wavefront active (lanes with
// nothing to add pass 0).
__device__ __forceinline__ double wave_total(double v) {
  double s = v + dpp_take<0x111, 0xf, 0xf>(v);  // row_shr:1
  s += dpp_take<0x112, 0xf, 0xf>(v);            // row_shr:2
  s += dpp_take<0x113, 0xf, 0xf>(v);            // row_shr:3
  s += dpp_take<0x114, 0xf, 0xe>(s);            // row_shr:4, banks 1-3
  s += dpp_take<0x118, 0xf, 0xc>(s);            // row_shr:8, banks 2-3
  s += dpp_take<0x142, 0xa, 0xf>(s);            // row_bcast:15 into rows 1, 3
  s += dpp_take<0x143, 0xc, 0xf>(s);            // row_bcast:31 into rows 2, 3
  return s;
}

}  // namespace gna
