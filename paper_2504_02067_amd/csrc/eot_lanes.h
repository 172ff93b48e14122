// Cross-lane sums of a wave64 in registers (gfx950): no LDS, no barrier; and
// the global -> LDS copy used to stage tiles.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace eot {

// Lane exchanges without LDS. permlane32_swap exchanges lanes 32..63 of its
// first operand with lanes 0..31 of its second; permlane16_swap does the same
// for the odd and even 16-lane rows. So for a = v[k], b = v[k + half] the sum
// of the two swapped registers is, on every lane, a summed over the lane pair
// (l, l ^ 32) (resp. l ^ 16) where that bit of l is clear and b summed where it
// is set: one stage of the transpose-reduction with no select.
__device__ __forceinline__ double pair_sum32(double a, double b)
{
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a),
                                                     (unsigned)__double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a),
                                                     (unsigned)__double2hiint(b), false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

__device__ __forceinline__ double pair_sum16(double a, double b)
{
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a),
                                                     (unsigned)__double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a),
                                                     (unsigned)__double2hiint(b), false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// x from another lane of the same 16-lane row (a DPP move of both halves).
constexpr int kDppXor1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;   // lane i <-> 7 - i within each 8 lanes
constexpr int kDppMirror = 0x140;       // lane i <-> 15 - i within each 16 lanes
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// One select stage of the transpose-reduction inside a 16-lane row: the lanes
// paired by CTRL differ in bit OFF; each keeps the value its bit selects.
template <int CTRL, int OFF>
__device__ __forceinline__ double pair_sum_dpp(double a, double b, int lane)
{
    const bool upper = (lane & OFF) != 0;
    const double keep = upper ? b : a;
    const double give = upper ? a : b;
    return keep + dpp_f64<CTRL>(give);
}

// Sum over the 64 lanes of a wave of G per-lane values at once (a butterfly
// transpose-reduction in registers, no LDS, no barrier): after it, lane l holds
// the full sum of value g = (l >> (6 - log2 G)) & (G - 1).
template <int G>
__device__ __forceinline__ double wave_transpose_sum(const double (&v)[G], int lane)
{
    static_assert(G == 4 || G == 8 || G == 16, "G");
    double x;
    if constexpr (G == 4) {
        x = pair_sum16(pair_sum32(v[0], v[2]), pair_sum32(v[1], v[3]));
    } else if constexpr (G == 8) {
        const double t0 = pair_sum16(pair_sum32(v[0], v[4]), pair_sum32(v[2], v[6]));
        const double t1 = pair_sum16(pair_sum32(v[1], v[5]), pair_sum32(v[3], v[7]));
        x = pair_sum_dpp<kDppMirror, 8>(t0, t1, lane);
    } else {
        double t[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            t[k] = pair_sum16(pair_sum32(v[k], v[k + 8]), pair_sum32(v[k + 4], v[k + 12]));
        const double w0 = pair_sum_dpp<kDppMirror, 8>(t[0], t[2], lane);
        const double w1 = pair_sum_dpp<kDppMirror, 8>(t[1], t[3], lane);
        x = pair_sum_dpp<kDppHalfMirror, 4>(w0, w1, lane);
    }
    // the remaining 16 / 8 / 4 lanes of each group: every lane ends with the sum
    x += dpp_f64<kDppXor1>(x);
    x += dpp_f64<kDppXor2>(x);
    if constexpr (G <= 8) x += dpp_f64<kDppHalfMirror>(x);
    if constexpr (G == 4) x += dpp_f64<kDppMirror>(x);
    return x;
}

// Sum over the 32 lanes of each wave half of 16 per-lane values at once (the
// same transpose-reduction): after it, lane l holds the full sum of value
// (l & 31) >> 1 of its half.
__device__ __forceinline__ double half_transpose_sum16(const double (&v)[16], int lane)
{
    double w[8], z[4], q[2];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = pair_sum16(v[k], v[k + 8]);
#pragma unroll
    for (int k = 0; k < 4; ++k) z[k] = pair_sum_dpp<kDppMirror, 8>(w[k], w[k + 4], lane);
#pragma unroll
    for (int k = 0; k < 2; ++k) q[k] = pair_sum_dpp<kDppHalfMirror, 4>(z[k], z[k + 2], lane);
    double x = pair_sum_dpp<kDppXor2, 2>(q[0], q[1], lane);
    x += dpp_f64<kDppXor1>(x);
    return x;
}

// x summed over the lane pair (l, l ^ 32), on both lanes.
__device__ __forceinline__ float pair_total32(float x)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                    false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// x summed over the lane pair (l, l ^ 32), on both lanes (FP64).
__device__ __forceinline__ double pair_total32_f64(double x)
{
    return pair_sum32(x, x);
}

// x summed over the lanes l, l ^ 16, l ^ 32, l ^ 48, on all four (FP64).
__device__ __forceinline__ double quad_total_f64(double x)
{
    return pair_sum32(pair_sum16(x, x), pair_sum16(x, x));
}

// x summed over the lanes l, l ^ 16, l ^ 32, l ^ 48, on all four (FP32).
__device__ __forceinline__ float quad_total_f32(float x)
{
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                    false);
    const float y = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(y), __float_as_uint(y), false,
                                                    false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// LDS byte address of a __shared__ object.
template <typename T>
__device__ __forceinline__ uint32_t lds_addr(const T* p)
{
    return (uint32_t)(uintptr_t)((const __attribute__((address_space(3))) T*)p);
}

// Copies 16 bytes per lane from gptr (per lane) to LDS at lds_base + 16 * lane
// (global_load_lds_dwordx4; lds_base is the same on every lane). Written as
// inline assembly so that the compiler's wait-count pass does not make every
// later LDS read wait for it: the caller waits for its own copies (s_waitcnt
// vmcnt) before the barrier that publishes them. The base goes in through M0
// (an operand, so the compiler sets it and knows it is used); a scalar write
// of M0 needs one wait state before an LDS copy uses it.
__device__ __forceinline__ void lds_dma16(const void* gptr, uint32_t lds_base)
{
    asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(gptr), "{m0}"(__builtin_amdgcn_readfirstlane(lds_base))
                 : "memory");
}

}  // namespace eot
