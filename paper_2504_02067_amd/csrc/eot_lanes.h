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

// ---- FP64 exp for the streaming passes ---------------------------------------
// exp(x) by the table-driven method of P. T. P. Tang (ACM TOMS 15(2), 1989):
// x = (64 q + j) ln2 / 64 + r with |r| <= ln2 / 128, so exp(x) = 2^q 2^(j/64) e^r;
// 2^(j/64) is a table entry held as a pair T_hi + T_lo (T_hi rounded to double,
// T_lo the rounded remainder; copied to LDS by the kernel), e^r - 1 = s comes from
// its Taylor polynomial of degree 5 (truncation below 4e-17 relative), and
// 2^(j/64) e^r = T_hi + (T_hi s + T_lo) to within 2^-60 relative, leaving one
// final rounding: the result is within 0.82 ulp (largest error over 2e7 arguments
// against a long-double exp: the final rounding plus the polynomial's truncation,
// up to 0.3 ulp in the upper half of a binade). The reduction uses ln2 / 64
// split into a rounded part and its remainder. x is clamped to [-1100, 710] by
// fmin / fmax, so that -inf and very negative x give 0, x above 709.79 (also
// +inf) gives inf, and NaN (which fmin replaces by 710) gives inf: non-finite
// either way, as the passes' checks need. |k| = |rint(64 x / ln2)| stays below
// 2^17, and the table index k & 63 is in range for every input.
// {T_hi, T_lo} of 2^(j/64), j = 0..63 (from 60-digit decimal arithmetic).
static __constant__ double kExp2Tab64[128] = {
    1.0, 0.0, 1.0108892860517005, -1.5234778603368577e-17,
    1.0218971486541166, 5.109225028973444e-17, 1.0330248790212284, 7.600838874027088e-18,
    1.0442737824274138, 8.551889705537965e-17, 1.0556451783605572, 1.759325738772092e-18,
    1.0671404006768237, -7.899853966841582e-17, 1.0787607977571199, -6.656660436056593e-17,
    1.0905077326652577, -3.046782079812471e-17, 1.102382583307841, 5.2660368715706944e-17,
    1.1143867425958924, 1.0410278456845571e-16, 1.1265216186082418, 5.165856758795457e-17,
    1.1387886347566916, 8.912812676025408e-17, 1.1511892299529827, 3.250710218863827e-17,
    1.1637248587775775, 3.8292048369240935e-17, 1.1763969916502812, 5.554203254218079e-17,
    1.189207115002721, 3.982015231465646e-17, 1.202156731452703, 6.644981499252301e-17,
    1.215247359980469, -7.712630692681488e-17, 1.22848053610687, -1.89878163130253e-17,
    1.241857812073484, 4.658027591836937e-17, 1.255380757024691, -6.7113898212968784e-18,
    1.2690509571917332, 2.667932131342186e-18, 1.2828700160787783, 1.713594918243561e-17,
    1.2968395546510096, 2.5382502794888315e-17, 1.3109612115247644, -7.181536135519454e-17,
    1.3252366431597413, -2.8587312100388614e-17, 1.339667524053303, 8.927282594831732e-17,
    1.3542555469368927, 7.70094837980299e-17, 1.3690024229745905, 9.593797919118849e-17,
    1.383909881963832, -6.770511658794786e-17, 1.3989796725383112, -9.614213209051323e-17,
    1.4142135623730951, -9.667293313452913e-17, 1.42961333839197, -1.2031642489053655e-17,
    1.4451808069770467, -3.0237581349939873e-17, 1.460917794180647, -5.600377186075216e-17,
    1.4768261459394993, -3.483994556892796e-17, 1.4929077282912648, 1.4192920154284036e-17,
    1.5091644275934228, -1.016455327754295e-16, 1.5255981507445384, -1.1024941712342561e-16,
    1.5422108254079407, 7.949834809697621e-17, 1.559004400237837, 3.7812070533575275e-17,
    1.5759808451078865, -1.0136916471278304e-17, 1.593142151342267, -1.0094406542311964e-16,
    1.6104903319492543, 2.4707192569797888e-17, 1.6280274218573478, -6.712955084707084e-17,
    1.645755478153965, -1.0125679913674773e-16, 1.6636765803267364, 5.8909926967131e-17,
    1.681792830507429, 8.199010020581497e-17, 1.7001063537185235, -8.0237193703977e-18,
    1.718619298122478, -1.851380418263111e-17, 1.7373338352737062, 3.164389299292957e-17,
    1.7562521603732995, 2.960140695448873e-17, 1.7753764925265212, 6.429731796556572e-17,
    1.7947090750031072, 1.8227458427912087e-17, 1.8142521755003989, -9.969531538920349e-17,
    1.8340080864093424, 3.283107224245627e-17, 1.8539791250833855, 9.761887490727594e-17,
    1.8741676341103, -6.122763413004143e-17, 1.8945759815869656, 3.4034035352165297e-17,
    1.9152065613971474, -1.0619946056195963e-16, 1.9360617934922943, 1.0332385960676326e-16,
    1.9571441241754002, 8.960767791036668e-17, 1.978456026387951, 4.0388753109278167e-17,
};
constexpr double kInvLn2x64 = 92.33248261689366;        // 64 / ln 2
constexpr double kLn2d64Hi = 0.010830424696249145;       // ln 2 / 64, rounded
constexpr double kLn2d64Lo = 3.623510646634843e-19;       // ln 2 / 64 - kLn2d64Hi

// s_tab: 128 doubles of LDS, 16-byte aligned.
__device__ __forceinline__ void load_exp_table(double* s_tab)
{
    if (threadIdx.x < 128) s_tab[threadIdx.x] = kExp2Tab64[threadIdx.x];
}

__device__ __forceinline__ double exp_tab64(double x, const double* s_tab)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    x = fmax(fmin(x, 710.0), -1100.0);
    const double kf = __builtin_rint(x * kInvLn2x64);
    const int k = (int)kf;
    const double r = fma(-kf, kLn2d64Lo, fma(-kf, kLn2d64Hi, x));
    const double t = fma(fma(fma(1.0 / 120.0, r, 1.0 / 24.0), r, 1.0 / 6.0), r, 0.5);
    const double s = fma(r * r, t, r);          // e^r - 1
    const d2 T = reinterpret_cast<const d2*>(s_tab)[k & 63];
    return ldexp(T.x + fma(T.x, s, T.y), k >> 6);
}

}  // namespace eot
