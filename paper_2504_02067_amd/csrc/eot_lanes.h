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
// exp(x) by the table-driven method of P. T. P. Tang (ACM TOMS 15(2), 1989) with
// a 256-entry table: x = (256 q + j) ln2 / 256 + r with q, j integers,
// 0 <= j < 256 and |r| <= ln2 / 512, so exp(x) = 2^q 2^(j/256) e^r.
//  * Reduction: fma(x, 256 / ln2, 1.5 * 2^52) rounds x 256 / ln2 to the nearest
//    integer k in one step (the sum's last bit is worth 1); subtracting
//    1.5 * 2^52 again gives k exactly, and the low 32 bits of the sum hold k
//    (two's complement), so j = k & 255 and q = k >> 8 need no conversion.
//    r = x - k ln2 / 256 uses ln2 / 256 split into a rounded part and its
//    remainder (two fmas).
//  * 2^(j/256) is a table entry held as a pair T_hi + T_lo (T_hi the double
//    nearest to it, T_lo the rounded remainder), copied to LDS by the kernel.
//  * e^r - 1 = s from its Taylor polynomial of degree 4 (truncation below
//    4e-17 relative for |r| <= ln2 / 512).
//  * 2^(j/256) e^r = T_hi + (T_hi s + T_lo), scaled by 2^q with v_ldexp_f64.
// Largest error over 2e7 arguments against a long-double exp: 0.84 ulp (the
// final rounding plus the polynomial's truncation). The argument is the
// passes' own x, so the FP64 passes round their exponents as before any
// change of base. x is clamped to [-1100, 710] by fmin / fmax first: -inf and
// x below -745.2 give 0, x above 709.79 (also +inf) gives inf, and NaN (which
// fmin replaces by 710) gives inf: non-finite either way, as the passes'
// checks need. |k| < 2^19, so the integer read from the sum is exact and j is
// in range for every input.
// {T_hi, T_lo} of 2^(j/256), j = 0..255 (from 60-digit decimal arithmetic).
static __constant__ double kExp2Tab256[512] = {
    1.0, 0.0, 1.0027112750502025, -3.636615928692264e-17,
    1.0054299011128027, 9.499186535455032e-17, 1.0081558981184175, -3.252058756084308e-17,
    1.0108892860517005, -1.5234778603368577e-17, 1.0136300849514894, 9.283599768183568e-18,
    1.016378314910953, -5.77217007319966e-17, 1.019133996077738, 3.601904982259662e-17,
    1.0218971486541166, 5.109225028973444e-17, 1.0246677928971357, -7.56160786848778e-17,
    1.0274459491187637, -4.9560741746453704e-17, 1.030231637686041, 3.319830041080813e-17,
    1.0330248790212284, 7.600838874027088e-18, 1.0358256936019572, -7.806782391337636e-17,
    1.0386341019613787, 5.996273788852511e-17, 1.041450124688316, 3.784830480287576e-17,
    1.0442737824274138, 8.551889705537965e-17, 1.0471050958792898, 7.277077243104315e-17,
    1.0499440858006872, 5.592937848127003e-17, 1.0527907730046264, -9.629482899026936e-17,
    1.0556451783605572, 1.759325738772092e-18, 1.0585073227945128, -7.152651856637781e-17,
    1.061377227289262, -1.1973537085365658e-17, 1.0642549128844645, 5.0787541986112304e-17,
    1.0671404006768237, -7.899853966841582e-17, 1.0700337118202419, -9.937162711288919e-17,
    1.0729348675259756, -3.839668843358824e-18, 1.075843889062791, -1.0002716151144136e-17,
    1.0787607977571199, -6.656660436056593e-17, 1.0816856149932152, -4.782623902997086e-17,
    1.0846183622133092, 3.166152845816346e-17, 1.0875590609177697, 5.409349307820291e-18,
    1.0905077326652577, -3.046782079812471e-17, 1.0934643990728858, 1.441395814726921e-17,
    1.0964290818163769, -5.919933484449316e-17, 1.099401802630222, 7.170459599701923e-17,
    1.102382583307841, 5.2660368715706944e-17, 1.1053714457017412, 8.239288760500214e-17,
    1.1083684117236787, -8.786813845180527e-17, 1.1113735033448175, 5.563945026669698e-17,
    1.1143867425958924, 1.0410278456845571e-16, 1.1174081515673693, -7.97680590262822e-17,
    1.1204377524096067, -6.201085906554179e-17, 1.12347556733302, -9.699737588987043e-17,
    1.1265216186082418, 5.165856758795457e-17, 1.129575928566288, 6.712805858726257e-17,
    1.1326385195987192, 3.237356166738e-17, 1.1357094141578055, 5.066599926126156e-17,
    1.1387886347566916, 8.912812676025408e-17, 1.1418762039695616, 4.6510911775314124e-17,
    1.1449721444318042, 4.6412898921700107e-17, 1.148076478840179, 6.897740236627192e-17,
    1.1511892299529827, 3.250710218863827e-17, 1.154310420590216, 1.0417128946273266e-16,
    1.1574400736337511, -9.1238712311344e-17, 1.1605782120274988, -3.261040205417394e-17,
    1.1637248587775775, 3.8292048369240935e-17, 1.1668800369524817, -8.79187957999917e-17,
    1.1700437696832502, -1.8477442017900047e-18, 1.1732160801636373, -7.287562586584994e-17,
    1.1763969916502812, 5.554203254218079e-17, 1.1795865274628758, 1.009231277510039e-16,
    1.182784710984341, 1.542975430079076e-17, 1.1859915656609938, -9.209506835293106e-18,
    1.189207115002721, 3.982015231465646e-17, 1.1924313825831512, 4.3975514156097214e-17,
    1.1956643920398273, 4.6166036704814814e-17, 1.1989061670743806, -9.809193356008423e-17,
    1.202156731452703, 6.644981499252301e-17, 1.2054161090051239, -3.3572721932675296e-17,
    1.2086843236265816, -4.746725945228984e-17, 1.2119613992768012, -4.8906110775211184e-17,
    1.215247359980469, -7.712630692681488e-17, 1.2185422298274085, -9.006726958363838e-17,
    1.2218460329727576, -1.0611021211402691e-16, 1.2251587936371455, -8.903533814269983e-17,
    1.22848053610687, -1.89878163130253e-17, 1.2318112847340759, 7.38938247161005e-17,
    1.2351510639369334, -1.0755244344307841e-16, 1.2384998981998165, 2.7677020555739674e-17,
    1.241857812073484, 4.658027591836937e-17, 1.245224830175258, -4.6772404498467275e-17,
    1.2486009771892048, -8.261810999021964e-17, 1.2519862778663162, 4.8341671524698976e-17,
    1.255380757024691, -6.7113898212968784e-18, 1.2587844395497165, -8.421782587730599e-17,
    1.2621973503942507, -3.0844648874738465e-17, 1.2656195145788063, 4.2505770034508686e-17,
    1.2690509571917332, 2.667932131342186e-18, 1.2724917033894028, -1.0577916267212421e-17,
    1.275941778396392, 9.91543024421429e-17, 1.2794012075056693, -9.759095008356062e-17,
    1.2828700160787783, 1.713594918243561e-17, 1.2863482295460256, -3.416955706936182e-17,
    1.2898358734066657, 8.949257530897592e-17, 1.2933329732290895, -2.9745904431327516e-17,
    1.2968395546510096, 2.5382502794888315e-17, 1.3003556433796506, 5.678728102802217e-17,
    1.3038812651919358, 8.647675598267871e-17, 1.3074164459346773, -7.336645652878869e-17,
    1.3109612115247644, -7.181536135519454e-17, 1.3145155879493546, 2.2675433151045856e-17,
    1.318079601266064, -5.4579558271491535e-17, 1.3216532776031575, -2.4806382459130217e-17,
    1.3252366431597413, -2.8587312100388614e-17, 1.3288297242059544, 4.08908622391016e-17,
    1.3324325470831615, -5.101586630916744e-17, 1.3360451382041458, -5.891866356388801e-17,
    1.339667524053303, 8.927282594831732e-17, 1.3432997311868353, -5.802580890201438e-17,
    1.3469417862329458, 3.224065101254679e-17, 1.3505937158920345, -8.287110381462417e-17,
    1.3542555469368927, 7.70094837980299e-17, 1.3579273062129011, -9.529635744825189e-17,
    1.3616090206382248, 1.533787661270668e-18, 1.365300717204012, -1.0005363125974765e-16,
    1.3690024229745905, 9.593797919118849e-17, 1.3727141650876684, -4.495960595234841e-17,
    1.3764359707545302, -6.898588935871801e-17, 1.380167867260238, 1.0510314579969984e-16,
    1.383909881963832, -6.770511658794786e-17, 1.387662042298529, 8.422984274875415e-17,
    1.3914243757719262, -4.9061748652889893e-17, 1.3951969099662003, -9.329336224225497e-17,
    1.3989796725383112, -9.614213209051323e-17, 1.4027726912202048, -5.295783249407989e-17,
    1.4065759938190154, 7.034914812136422e-18, 1.4103896082172707, 4.166548728435062e-17,
    1.4142135623730951, -9.667293313452913e-17, 1.4180478843204152, 2.2744385421855295e-17,
    1.4218926021691656, -1.6077828915890244e-17, 1.4257477441054942, 9.880690758500607e-17,
    1.42961333839197, -1.2031642489053655e-17, 1.433489413367789, -5.802454243926826e-17,
    1.4373759974489824, -4.2040340164675566e-17, 1.4412731191286257, 5.602503650878986e-18,
    1.4451808069770467, -3.0237581349939873e-17, 1.449099089642035, -6.259405000819309e-17,
    1.4530279958490526, -5.779948609396106e-17, 1.4569675544014438, 5.648679453876998e-17,
    1.460917794180647, -5.600377186075216e-17, 1.4648787441464057, 9.530767543587157e-17,
    1.4688504333369818, 8.465882756533628e-17, 1.4728328908693675, 6.691774081940589e-17,
    1.4768261459394993, -3.483994556892796e-17, 1.4808302278224719, -9.686952102630619e-17,
    1.4848451658727524, 1.0780086764407481e-16, 1.488870989524397, 6.155367157742871e-17,
    1.4929077282912648, 1.4192920154284036e-17, 1.4969554117672355, -2.861663253899158e-17,
    1.5010140696264256, -6.413767275790235e-17, 1.5050837316234065, 7.074710613582846e-17,
    1.5091644275934228, -1.016455327754295e-16, 1.5132561874526098, 8.884497851338712e-17,
    1.5173590411982147, -4.308699472043341e-17, 1.5214730189088146, -5.9963876759456834e-18,
    1.5255981507445384, -1.1024941712342561e-16, 1.529734466947287, 3.7857921151572197e-17,
    1.533881997840956, 8.875226844438446e-17, 1.5380407738316568, 1.0174672351161359e-16,
    1.5422108254079407, 7.949834809697621e-17, 1.5463921831410214, 1.068396000565722e-16,
    1.550584877685, -1.4600706590689385e-17, 1.5547889397770887, -8.003161350116036e-17,
    1.559004400237837, 3.7812070533575275e-17, 1.5632312899713576, 7.484777645590734e-17,
    1.567469639965553, -1.0352061768849722e-16, 1.5717194812923414, -3.3429840046872e-17,
    1.5759808451078865, -1.0136916471278304e-17, 1.5802537626528246, -5.163402929554468e-17,
    1.5845382652524937, -1.9337717034585703e-17, 1.588834384317164, -5.9949501188244794e-18,
    1.593142151342267, -1.0094406542311964e-16, 1.597461597908627, 2.4868392796221e-17,
    1.6017927556826934, -6.054917453527784e-17, 1.606135656416771, -1.0354545288059995e-16,
    1.6104903319492543, 2.4707192569797888e-17, 1.6148568142048607, -7.316663399125123e-17,
    1.6192351351948637, 2.0941334154229092e-17, 1.6236253270173289, -3.584512851414475e-17,
    1.6280274218573478, -6.712955084707084e-17, 1.632441451987275, 9.852819230429993e-17,
    1.6368674497669644, 7.698325071319876e-17, 1.6413054476440063, -9.247568737640706e-17,
    1.645755478153965, -1.0125679913674773e-16, 1.6502175739206177, 9.133279588729904e-18,
    1.6546917676561943, 9.643294303196029e-17, 1.6591780921616162, -7.275545550823051e-17,
    1.6636765803267364, 5.8909926967131e-17, 1.6681872651305825, 4.269178019570615e-17,
    1.6727101796415966, -5.476715964599563e-17, 1.6772453570178785, 8.303949509950733e-17,
    1.681792830507429, 8.199010020581497e-17, 1.6863526334483934, -7.181463278358011e-17,
    1.6909247992693053, -9.66967147439488e-17, 1.6955093614893326, 7.238416872845167e-17,
    1.7001063537185235, -8.0237193703977e-18, 1.7047158096580513, -2.7288832847972816e-17,
    1.709337763100463, -9.868779456632931e-17, 1.713972247929926, 6.473975107753367e-17,
    1.718619298122478, -1.851380418263111e-17, 1.723278947746274, -9.5221238003938e-17,
    1.7279512309618377, -1.0750981861204642e-16, 1.732636182022311, -1.6980510743154155e-18,
    1.7373338352737062, 3.164389299292957e-17, 1.7420442251551564, -1.5259591189507888e-18,
    1.746767386199169, -1.0752290483507515e-16, 1.7515033530318782, -5.1244504205967247e-17,
    1.7562521603732995, 2.960140695448873e-17, 1.761013843037584, -7.943253125039228e-17,
    1.7657884359332727, 9.461315018083268e-17, 1.7705759740635547, 5.961794510040556e-17,
    1.7753764925265212, 6.429731796556572e-17, 1.7801900265154245, -5.2846272890916174e-17,
    1.785016611318935, 1.5330400121031314e-17, 1.789856282321401, -4.1543546606833504e-17,
    1.7947090750031072, 1.8227458427912087e-17, 1.7995750249405351, -2.526889233358898e-17,
    1.804454167806624, -5.177222408793318e-17, 1.809346539371032, -9.03264140245003e-17,
    1.8142521755003989, -9.969531538920349e-17, 1.8191711121586085, 7.402676901145839e-17,
    1.8241033854070534, -1.0159627862277083e-16, 1.8290490314048973, 6.889192908835696e-17,
    1.8340080864093424, 3.283107224245627e-17, 1.8389805867758937, 6.918969740272512e-18,
    1.843966568958626, -5.939742026949965e-17, 1.8489660695104508, 9.027580446261089e-17,
    1.8539791250833855, 9.761887490727594e-17, 1.8590057724288205, -9.528705461989941e-17,
    1.864046048397789, 6.540912680620572e-17, 1.8690999899412386, -9.938505214255067e-17,
    1.8741676341103, -6.122763413004143e-17, 1.8792490180565602, -1.6226315557835845e-17,
    1.8843441790323345, -8.226593125533711e-17, 1.8894531543909392, -9.005168285059127e-17,
    1.8945759815869656, 3.4034035352165297e-17, 1.8997126981765553, -3.8597397693785143e-17,
    1.9048633418176741, 6.533857514718279e-17, 1.9100279502703899, -5.90968800674406e-17,
    1.9152065613971474, -1.0619946056195963e-16, 1.9203992131630474, 7.116681540630314e-17,
    1.925605943636125, -9.914963769693741e-17, 1.930826790987627, 6.16714970616911e-17,
    1.9360617934922943, 1.0332385960676326e-16, 1.9413109895286405, -6.638029891621488e-17,
    1.9465744175792332, 6.811022349533877e-17, 1.9518521162309783, -2.199016969979351e-17,
    1.9571441241754002, 8.960767791036668e-17, 1.9624504802089273, 1.0976844000913547e-16,
    1.9677712232331759, -1.0314928011531132e-16, 1.9731063922552343, -7.451617863956037e-18,
    1.978456026387951, 4.0388753109278167e-17, 1.9838201648502194, -2.2034544123910627e-17,
    1.9891988469672663, 8.2051326383692e-18, 1.9945921121709402, 1.7909710352002645e-17,
};
constexpr int kExpTabDoubles = 512;
constexpr double kExpRound = 6755399441055744.0;         // 1.5 * 2^52
constexpr double kExpInvLn2x256 = 369.3299304675746;     // 256 / ln 2
constexpr double kExpLn2d256Hi = 0.0027076061740622863;  // ln 2 / 256, rounded
constexpr double kExpLn2d256Lo = 9.058776616587108e-20;  // ln 2 / 256 - kExpLn2d256Hi

// s_tab: kExpTabDoubles doubles of LDS, 16-byte aligned; every thread of the
// workgroup calls this, and a barrier must follow before the first read.
__device__ __forceinline__ void load_exp_table(double* s_tab)
{
    for (int i = threadIdx.x; i < kExpTabDoubles; i += blockDim.x) s_tab[i] = kExp2Tab256[i];
}

__device__ __forceinline__ double exp_tab256(double x, const double* s_tab)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    x = fmax(fmin(x, 710.0), -1100.0);
    const double kd = fma(x, kExpInvLn2x256, kExpRound);
    const double kf = kd - kExpRound;
    const int k = (int)(unsigned)__builtin_bit_cast(unsigned long long, kd);
    const double r = fma(-kf, kExpLn2d256Lo, fma(-kf, kExpLn2d256Hi, x));
    const double t = fma(fma(1.0 / 24.0, r, 1.0 / 6.0), r, 0.5);
    const double s = fma(r * r, t, r);          // e^r - 1
    const d2 T = reinterpret_cast<const d2*>(s_tab)[k & 255];
    return ldexp(T.x + fma(T.x, s, T.y), k >> 8);
}

}  // namespace eot
