// Cross-lane sums inside a 64-wide wavefront built from DPP lane swizzles.
//
// __shfl_xor lowers to ds_bpermute on gfx950: a round trip through the LDS
// crossbar with a full wait per step.  The data-parallel-primitive (DPP) modifiers
// instead read a neighbour lane's register inside the VALU instruction, so an
// 8-lane butterfly costs three DPP moves.  The patterns used here stay inside one
// 16-lane row:
//   quad_perm [1,0,3,2]  lane ^ 1
//   quad_perm [2,3,0,1]  lane ^ 2
//   row_half_mirror      lane i <-> 7 - i inside each 8-lane half (after the first
//                        two steps every lane of a quad holds the quad total, so
//                        this adds the other quad's total exactly like lane ^ 4)
//   row_mirror           lane i <-> 15 - i inside the row (the same argument for 16)
// All lanes of a group end with bit-identical totals, in the same summation order
// as the xor butterfly.  Every lane of the wavefront must be active.
#pragma once

#include <hip/hip_runtime.h>

namespace fem {

enum : int { kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140 };

template <int CTRL>
__device__ __forceinline__ float dpp_read(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_read(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffu), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(unsigned(hi)) << 32) | unsigned(lo));
}

// Sum over the aligned group of 8 lanes (all 8 lanes receive it).
template <typename T>
__device__ __forceinline__ T lane_sum8(T v) {
    v += dpp_read<kDppXor1>(v);
    v += dpp_read<kDppXor2>(v);
    v += dpp_read<kDppHalfMirror>(v);
    return v;
}

// Sum over the aligned group of 16 lanes (all 16 lanes receive it).
template <typename T>
__device__ __forceinline__ T lane_sum16(T v) {
    v = lane_sum8(v);
    v += dpp_read<kDppMirror>(v);
    return v;
}

// Exchange between the two 16-lane rows of a 32-lane group (v_permlane16_swap): a
// lane of the lower row receives its partner's `a`, a lane of the upper row its
// partner's `b` (the partner is the lane 16 positions away).
__device__ __forceinline__ unsigned swap_rows_u32(unsigned a, unsigned b, bool upper) {
    const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    return upper ? r[0] : r[1];
}

__device__ __forceinline__ float swap_rows(float a, float b, bool upper) {
    return __builtin_bit_cast(float, swap_rows_u32(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b), upper));
}

__device__ __forceinline__ double swap_rows(double a, double b, bool upper) {
    const unsigned long long ua = __builtin_bit_cast(unsigned long long, a), ub = __builtin_bit_cast(unsigned long long, b);
    const unsigned lo = swap_rows_u32(unsigned(ua & 0xffffffffu), unsigned(ub & 0xffffffffu), upper);
    const unsigned hi = swap_rows_u32(unsigned(ua >> 32), unsigned(ub >> 32), upper);
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// Sum over a 32-lane group; lane 0 of the group holds the total.
template <typename T>
__device__ __forceinline__ T group32_sum(T a, int lane32) {
    T s = a + swap_rows(a, a, lane32 >= 16);
    s += dpp_read<kDppMirror>(s);
    s += dpp_read<kDppHalfMirror>(s);
    s += dpp_read<kDppXor2>(s);
    s += dpp_read<kDppXor1>(s);
    return s;
}

// Reduce-scatter of three sums over a 32-lane group: lane 0 gets sum a0, lane 8 sum
// a1, lane 16 sum a2 (six exchanges instead of three full butterflies).  Step 1
// moves a0/a1 to the lower row and a2 to the upper row, step 2 splits each row
// into halves, and three in-half steps finish the sums.
template <typename T>
__device__ __forceinline__ T group32_sum3(T a0, T a1, T a2, int lane32) {
    const bool upper = lane32 >= 16;
    const T b0 = (upper ? a2 : a0) + swap_rows(a0, a2, upper);
    const T b1 = (upper ? T(0) : a1) + swap_rows(a1, T(0), upper);
    const bool low = (lane32 & 15) < 8;
    T c = (low ? b0 : b1) + dpp_read<kDppMirror>(low ? b1 : b0);
    c += dpp_read<kDppHalfMirror>(c);
    c += dpp_read<kDppXor2>(c);
    c += dpp_read<kDppXor1>(c);
    return c;
}

}  // namespace fem
