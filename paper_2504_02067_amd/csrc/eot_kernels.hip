// Device kernels of the truncated-Newton entropic-OT library for gfx950.
//
// The hot path is the streaming pass over the implicit plan
//     P_ij = exp(u_i + v_j - beta C_ij)            (eq. lagrangian-closed-form)
// that serves every O(nm) primitive of the method: the LSE_r / LSE_c
// marginals (Sec. 2 Notation; used throughout Algs. 3 and 4), the two
// halves of the reduced Newton operator F_r(rho) p = r(P) p - rho P (P^T p / c)
// (eq. matrix-definitions) inside CG, the discounted Hessian-vector product
// (eq. discounted-hessian) and the preconditioner diagonal sum_j P_ij^2 / c_j
// (lemma "condo").
//
// Design (gfx950):
//  * A workgroup of 256 threads (4 wave64) owns a tile of rb x kTileCols
//    entries (rb = 8 .. kTileRows rows, chosen per problem by the host from a
//    measured table). Each thread owns 4 consecutive columns in each of 2
//    column chunks, so every row of the tile is read as 16-byte, fully
//    coalesced non-temporal loads; RS rows of one chunk load while the other
//    chunk computes (double buffer), and loads never sit behind a branch.
//  * One read of C feeds both directions: column sums accumulate in FP64
//    registers across the tile's rows (written once per tile), row sums
//    accumulate per thread over its 8 columns and are reduced per wave by a
//    butterfly transpose in registers (no LDS, no barrier in the loop).
//  * Per-tile partial sums are merged in a fixed order by small epilogue
//    kernels (bit-reproducible), except for problems whose partials would
//    exceed 512 MB, which accumulate with FP64 atomics.
//  * Point clouds: |x_i - y_j|^2 is recomputed per entry (difference form);
//    no cost bytes are read, so those passes are bound by VALU issue.
//  * Mixed precision: the exponent is assembled in FP32 without losing the
//    FP64 potentials. In base 2, U_i = log2(e)(u_i - a_i) and V_j = log2(e) v_j
//    are split per tile into a hi part on a grid 2^-g (g chosen from the
//    tile's largest |U|, |V|) and an FP32 lo part, and log2(e) beta into
//    Bh + Bl, so that Uh + Vh is exact in FP32 and
//        x = fma(-Bl, C, fma(-Bh, C, Uh + Vh))
//    carries two roundings of a number close to log2(P_ij / r(P)_i). 2^Ul and
//    exp(a_i) become an FP64 per-row factor, 2^Vl an FP64 per-column factor
//    (folded into the row weights and applied to the column totals). exp2 is
//    v_exp_f32; every sum is accumulated in FP64.
//  * FP64 mode evaluates x = fma(-beta, C, (u_i - a_i) + v_j) and exp in FP64.
// The row shift a_i (about log r(P)_i) only keeps exponentials in range.

#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>
#include <type_traits>
#include <vector>

#include "eot_internal.h"
#include "eot_lanes.h"

namespace eot {

namespace {

constexpr double kLog2e = 1.4426950408889634074;

__device__ __forceinline__ double wave_max(double x)
{
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}

__device__ __forceinline__ double wave_sum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Loads of 4 consecutive cost entries starting at column jb of one row. They
// never branch: addresses are clamped into the row's first m entries (vector
// loads are used only when m and ldc are multiples of 4, so a clamped
// 16-byte group never reaches the ldc padding), so the compiler keeps all
// loads of a sub-band in flight and whatever the padding holds (NaN, inf) is
// never read. Lanes past column m get a clamped finite entry whose plan weight
// the -inf column potential makes 0. Streaming data, so non-temporal (no
// reuse expected in the caches).
template <bool VEC>
__device__ __forceinline__ void load4(const float* __restrict__ row, int64_t jb, int64_t m,
                                      int64_t ldc, float (&out)[kVec])
{
    if constexpr (VEC) {   // m, ldc % 4 == 0 and 16-byte aligned base: row + jl is aligned
        const int64_t jl = jb < m - 3 ? jb : m - 4;
        const f32x4 x = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(row + jl));
        out[0] = x.x; out[1] = x.y; out[2] = x.z; out[3] = x.w;
    } else {
#pragma unroll
        for (int q = 0; q < kVec; ++q) {
            const int64_t jq = jb + q < m ? jb + q : m - 1;
            out[q] = __builtin_nontemporal_load(row + jq);
        }
    }
}

template <bool VEC>
__device__ __forceinline__ void load4(const float* __restrict__ row, int64_t jb, int64_t m,
                                      int64_t ldc, double (&out)[kVec])
{
    float t[kVec];
    load4<VEC>(row, jb, m, ldc, t);
#pragma unroll
    for (int q = 0; q < kVec; ++q) out[q] = (double)t[q];
}

template <bool VEC>
__device__ __forceinline__ void load4(const double* __restrict__ row, int64_t jb, int64_t m,
                                      int64_t ldc, double (&out)[kVec])
{
    if constexpr (VEC) {
        const int64_t jl = jb < m - 3 ? jb : m - 4;
        const f64x2 x0 = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(row + jl));
        const f64x2 x1 = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(row + jl + 2));
        out[0] = x0.x; out[1] = x0.y; out[2] = x1.x; out[3] = x1.y;
    } else {
#pragma unroll
        for (int q = 0; q < kVec; ++q) {
            const int64_t jq = jb + q < m ? jb + q : m - 1;
            out[q] = __builtin_nontemporal_load(row + jq);
        }
    }
}

// Writes one wave's row partials of a sub-band: row_part[k][tile * waves + wave][i].
template <int NR, int RS, int MODE2>
__device__ __forceinline__ void wave_rows_out(double (&racc)[NR][RS], const double* s_rf, int sb,
                                              int64_t i0, int64_t n, const PassArgs& A)
{
    constexpr int G = NR * RS;
    constexpr int LG = G == 4 ? 2 : (G == 8 ? 3 : 4);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[G];
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int rr = 0; rr < RS; ++rr) v[k * RS + rr] = racc[k][rr];
    const double tot = wave_transpose_sum<G>(v, lane);
    if ((lane & ((64 >> LG) - 1)) == 0) {
        const int g = (lane >> (6 - LG)) & (G - 1);
        const int k = g / RS, rr = g % RS;
        const int64_t i = i0 + sb + rr;
        if (i < n) {
            double fac = s_rf[sb + rr];
            if (k == 1 && MODE2 == R2_SQUARE) fac *= fac;
            if (A.atomic)
                atomicAdd(&A.row_part[(int64_t)k * n + i], tot * fac);
            else
                A.row_part[(((int64_t)k * A.tiles_m + blockIdx.x) * kWaves + wave) * n + i] = tot * fac;
        }
    }
}

template <typename TC, bool VEC, int RS>
__device__ __forceinline__ void load_rows(const TC* __restrict__ C, int64_t ldc, int64_t i0,
                                          int64_t n, int64_t jb, int64_t m,
                                          TC (&buf)[RS][kVec])
{
#pragma unroll
    for (int rr = 0; rr < RS; ++rr) {
        int64_t i = i0 + rr;
        i = i < n ? i : n - 1;
        if constexpr (sizeof(TC) == 4) {
            load4<VEC>(C + i * ldc, jb, m, ldc, buf[rr]);
        } else {
            load4<VEC>(C + i * ldc, jb, m, ldc, buf[rr]);
        }
    }
}

// ---------------------------------------------------------------- the pass
// Rows whose column sums a lane keeps in FP32 before adding them to its FP64
// totals (LANE32 passes; a multiple of the sub-band height).
constexpr int kLane32Rows = 16;

// PREC = EOT_PREC_MIXED (FP32 exponent / exp, FP64 sums; the point-cloud
// passes with one plain row and one column sum sum in FP32 within a lane, see
// LANE32) or EOT_PREC_FP64.
// DP = 0: dense cost streamed from memory. RS rows are in flight per chunk;
// the next chunk's loads are issued before the current chunk is computed
// (double buffer), and row partials are reduced per wave in registers, so the
// loop has no workgroup barrier.
// DP > 0: C_ij = |x_i - y_j|^2 recomputed per entry in the difference form
// (the O(n)-memory variant of Sec. 4.2): x rows in LDS, y columns in
// registers; the 1/scale of the cost is folded into beta by the host.
template <int PREC, typename TC, int NR, int NC, int MODE2, bool VEC, int RS, int DP>
__device__ __forceinline__ void pass_body(const PassArgs& A)
{
    if (A.skip && *A.skip) return;             // uniform: a finished CG chunk
    constexpr bool MIXED = PREC == EOT_PREC_MIXED;
    constexpr int RB = kTileRows, NCH = kChunks, V = kVec, T = kPassThreads;
    static_assert(NCH == 2, "the double buffer alternates the two column chunks");
    static_assert(RB <= T && RB % RS == 0, "tile rows");
    constexpr int NYW = MODE2 == R2_HVP ? 1 : (NR > 0 ? NR : 1);
    constexpr int NRA = NR > 0 ? NR : 1, NCA = NC > 0 ? NC : 1;
    __shared__ float s_uh[RB];          // mixed: hi part of log2e (u - a)
    __shared__ double s_A[RB];          // FP64: u - a
    __shared__ double s_rf[RB];         // per-row factor of the row partials (2^Ul or 1)
    __shared__ double s_xw[2][RB];      // column-sum weights
    __shared__ double s_rr[RB];         // R_i = exp(a_i) 2^Ul (HVP)
    __shared__ double s_wmax[kWaves];
    __shared__ float s_x[DP > 0 ? RB * DP : 1];   // point rows
    __shared__ __attribute__((aligned(16))) double s_exp[MIXED ? 2 : kExpTabDoubles];  // FP64: exp_tab256
    // Mixed point-cloud passes with one plain weighted row sum and one column
    // sum (the HVP with the marginals given, the marginal pass): the sums run in
    // FP32 within a lane and in FP64 from there on (lanes, waves, tiles), as in
    // the high-dimensional pass. (The column-sum pass keeps FP64 sums, FP32 ones
    // made it slower; mixed row-sum passes over points use k_rows_pts.)
    constexpr bool LANE32 = MIXED && DP > 0 && MODE2 != R2_HVP && NR == 1 && NC == 1;
    __shared__ float s_xwf[LANE32 ? RB : 1];      // FP32 copy of the column-sum weights

    const int tid = threadIdx.x;
    if constexpr (!MIXED) load_exp_table(s_exp);  // read after the prologue's barrier
    const int64_t n = A.n, m = A.m;
    const int rbt = A.rb;                      // rows of this launch's tiles (<= RB, % 8 == 0)
    const int64_t i0 = (int64_t)blockIdx.y * rbt;
    const int64_t j0 = (int64_t)blockIdx.x * kTileCols;
    const TC* __restrict__ C = static_cast<const TC*>(A.C);

    // ---- prologue: per-column values in registers, per-row values in LDS
    const int64_t irow = i0 + tid;
    const bool rvalid = tid < rbt && irow < n;
    float vh[NCH][V], vl[NCH][V];
    double vc[NCH][V];
    double arow = 0.0, ul = 0.0, uh = 0.0;
    if constexpr (MIXED) {
        double Vd[NCH][V];
        double mx = 0.0;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const int64_t j = j0 + (int64_t)ch * T * V + tid * V + q;
                Vd[ch][q] = (j < m) ? kLog2e * A.v[j] : 0.0;
                mx = fmax(mx, fabs(Vd[ch][q]));
            }
        double Ud = 0.0;
        if (rvalid) {
            arow = A.a[irow];
            Ud = kLog2e * (A.u[irow] - arow);
            mx = fmax(mx, fabs(Ud));
        }
        mx = wave_max(mx);
        if ((tid & 63) == 0) s_wmax[tid >> 6] = mx;
        __syncthreads();
        mx = s_wmax[0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) mx = fmax(mx, s_wmax[w]);
        if (!(mx < 4.0e6)) mx = 4.0e6;          // non-finite input: results flagged later
        int e2;
        frexp(2.0 * mx + 2.0, &e2);              // 2 mx + 2 < 2^e2
        const int g = 23 - e2;                   // |Uh + Vh| < 2^(23-g) on a 2^-g grid: exact
        const double sc = ldexp(1.0, g), isc = ldexp(1.0, -g);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const int64_t j = j0 + (int64_t)ch * T * V + tid * V + q;
                const double h = rint(Vd[ch][q] * sc) * isc;
                vh[ch][q] = (j < m) ? (float)h : -INFINITY;
                vl[ch][q] = (j < m) ? (float)(Vd[ch][q] - h) : 0.0f;
            }
        uh = rint(Ud * sc) * isc;
        ul = Ud - uh;
    } else {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const int64_t j = j0 + (int64_t)ch * T * V + tid * V + q;
                vc[ch][q] = (j < m) ? A.v[j] : -INFINITY;
            }
        if (rvalid) arow = A.a[irow];
    }
    if (tid < RB) {
        if (rvalid) {
            const double rf = MIXED ? exp2(ul) : 1.0;
            const double R = exp(arow) * rf;
            s_uh[tid] = (float)uh;
            s_A[tid] = MIXED ? 0.0 : A.u[irow] - arow;
            s_rf[tid] = rf;
            s_rr[tid] = R;
            if constexpr (MODE2 == R2_HVP) {   // xw0 = R sqrt(rho) x_i, xw1 = x_i
                s_xw[0][tid] = R * A.hvp_srho * A.xw1[irow];
                s_xw[1][tid] = A.xw1[irow];
            } else {
                s_xw[0][tid] = R * (A.xw0 ? A.xw0[irow] : 1.0);
                s_xw[1][tid] = R * (A.xw1 ? A.xw1[irow] : 1.0);
            }
        } else {
            s_uh[tid] = -INFINITY;
            s_A[tid] = -INFINITY;
            s_rf[tid] = 0.0;
            s_rr[tid] = 0.0;
            s_xw[0][tid] = 0.0;
            s_xw[1][tid] = 0.0;
        }
        if constexpr (LANE32) s_xwf[tid] = (float)s_xw[0][tid];
        if constexpr (DP > 0) {
#pragma unroll
            for (int k = 0; k < DP; ++k) s_x[tid * DP + k] = rvalid ? A.X[irow * DP + k] : 0.0f;
        }
    }
    float yr[DP > 0 ? NCH : 1][DP > 0 ? V : 1][DP > 0 ? DP : 1];
    if constexpr (DP > 0) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const int64_t j = j0 + (int64_t)ch * T * V + tid * V + q;
#pragma unroll
                for (int k = 0; k < DP; ++k) yr[ch][q][k] = (j < m) ? A.Y[j * DP + k] : 0.0f;
            }
    }
    const double Bd = kLog2e * A.beta;
    const float Bh = (float)Bd;
    const float Bl = (float)(Bd - (double)Bh);
    const double beta = A.beta;
    const double srho = A.hvp_srho;

    // Mixed: the column's lo exponent enters as the factor f_j = 2^Vl_j, folded
    // into the row weights here and applied to the column totals at the end,
    // so a plan entry costs exp2(fma(-Bl, C, fma(-Bh, C, Uh + Vh))) * f_j.
    double ywr[NYW][NCH][V];
    double fj[MODE2 == R2_HVP && MIXED ? NCH : 1][MODE2 == R2_HVP && MIXED ? V : 1];
    double ayw[MODE2 == R2_HVP && MIXED ? NCH : 1][MODE2 == R2_HVP && MIXED ? V : 1];
#pragma unroll
    for (int k = 0; k < NYW; ++k)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const int64_t j = j0 + (int64_t)ch * T * V + tid * V + q;
                const double* yw = MODE2 == R2_HVP ? A.yw1 : (k == 0 ? A.yw0 : A.yw1);
                double w = (j < m) ? (yw ? yw[j] : 1.0) : 0.0;
                if constexpr (MIXED) {
                    const double f = exp2((double)vl[ch][q]);
                    if constexpr (MODE2 == R2_HVP) {
                        fj[ch][q] = f;
                        ayw[ch][q] = srho * w * f;
                    } else {
                        w *= (k == NR - 1 && NR >= 2 && MODE2 == R2_SQUARE) ? f * f : f;
                    }
                }
                ywr[k][ch][q] = w;
            }
    double cacc[NCA][NCH][V];
#pragma unroll
    for (int k = 0; k < NCA; ++k)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int q = 0; q < V; ++q) cacc[k][ch][q] = 0.0;
    __syncthreads();

    // ---- main loop: one iteration = one sub-band of RS rows, both chunks
    const int64_t rows = n - i0 < rbt ? n - i0 : rbt;
    const int nsb = (int)((rows + RS - 1) / RS);
    const int64_t jb0 = j0 + tid * V, jb1 = j0 + (int64_t)T * V + tid * V;

    // getc(rr, q) -> cost entry (FP32 in mixed mode, FP64 otherwise)
    auto compute = [&](int sb, int ch, auto&& getc, double (&racc)[NRA][RS]) {
#pragma unroll
        for (int rr = 0; rr < RS; ++rr) {
            const double xw0 = s_xw[0][sb + rr];
            const double xw1 = s_xw[1][sb + rr];
#pragma unroll
            for (int q = 0; q < V; ++q) {
                double e64, cd;
                if constexpr (MIXED) {
                    const float c = getc(rr, q);
                    const float t = fmaf(-Bh, c, s_uh[sb + rr] + vh[ch][q]);
                    e64 = (double)__builtin_amdgcn_exp2f(fmaf(-Bl, c, t));
                    cd = (double)c;
                } else {
                    const double c = getc(rr, q);
                    e64 = exp_tab256(fma(-beta, c, s_A[sb + rr] + vc[ch][q]), s_exp);
                    cd = c;
                }
                if constexpr (MODE2 == R2_HVP) {
                    // rows: e (x_i + sqrt(rho) y_j); columns: R_i e (sqrt(rho) x_i + y_j)
                    if constexpr (MIXED)
                        racc[0][rr] = fma(e64, fma(xw1, fj[ch][q], ayw[ch][q]), racc[0][rr]);
                    else
                        racc[0][rr] = fma(e64, fma(srho, ywr[0][ch][q], xw1), racc[0][rr]);
                    cacc[0][ch][q] = fma(e64, fma(s_rr[sb + rr], ywr[0][ch][q], xw0), cacc[0][ch][q]);
                } else {
                    if constexpr (NR >= 1) racc[0][rr] = fma(e64, ywr[0][ch][q], racc[0][rr]);
                    if constexpr (NR >= 2) {
                        double term = e64;
                        if constexpr (MODE2 == R2_SQUARE) term = e64 * e64;
                        if constexpr (MODE2 == R2_COST) term = e64 * cd;
                        racc[NR - 1][rr] = fma(term, ywr[NR - 1][ch][q], racc[NR - 1][rr]);
                    }
                    if constexpr (NC >= 1) cacc[0][ch][q] = fma(e64, xw0, cacc[0][ch][q]);
                    if constexpr (NC >= 2) {
                        const double term = MODE2 == R2_COST ? e64 * cd : e64;
                        cacc[NC - 1][ch][q] = fma(term, xw1, cacc[NC - 1][ch][q]);
                    }
                }
                (void)cd;
            }
        }
    };

    if constexpr (DP == 0) {
        TC buf0[RS][V], buf1[RS][V];
        load_rows<TC, VEC, RS>(C, A.ldc, i0, n, jb0, m, buf0);
        // Columns past m load a clamped in-bounds (finite) entry; their
        // Vh = -inf (mixed) or v = -inf (FP64) makes the plan entry 0.
        auto dense = [&](TC (&buf)[RS][V]) {
            return [&buf](int rr, int q) {
                using E = typename std::conditional<MIXED, float, double>::type;
                return (E)buf[rr][q];
            };
        };
        for (int b = 0; b < nsb; ++b) {
            const int sb = b * RS;
            double racc[NRA][RS];
#pragma unroll
            for (int k = 0; k < NRA; ++k)
#pragma unroll
                for (int rr = 0; rr < RS; ++rr) racc[k][rr] = 0.0;
            load_rows<TC, VEC, RS>(C, A.ldc, i0 + sb, n, jb1, m, buf1);
            // keep each prefetch where it is issued: the scheduler would otherwise
            // sink it next to its use to save registers, emptying the pipeline
            __builtin_amdgcn_sched_barrier(0);
            compute(sb, 0, dense(buf0), racc);
            // the next sub-band; past the tile's last row the loads clamp to it
            // (cached), which keeps the loop free of a conditional buffer
            load_rows<TC, VEC, RS>(C, A.ldc, i0 + sb + RS, i0 + rows, jb0, m, buf0);
            __builtin_amdgcn_sched_barrier(0);
            compute(sb, 1, dense(buf1), racc);
            if constexpr (NR > 0) wave_rows_out<NR, RS, MODE2>(racc, s_rf, sb, i0, n, A);
        }
    } else {
        auto pts = [&](int sb, int ch) {
            return [&, sb, ch](int rr, int q) {
                if constexpr (MIXED) {
                    float d2 = 0.0f;
#pragma unroll
                    for (int k = 0; k < DP; ++k) {
                        const float df = s_x[(sb + rr) * DP + k] - yr[ch][q][k];
                        d2 = fmaf(df, df, d2);
                    }
                    return d2;
                } else {
                    double d2 = 0.0;
#pragma unroll
                    for (int k = 0; k < DP; ++k) {
                        const double df = (double)s_x[(sb + rr) * DP + k] - (double)yr[ch][q][k];
                        d2 = fma(df, df, d2);
                    }
                    return d2;
                }
            };
        };
        if constexpr (LANE32) {
            // Row sums: FP32 over the lane's NCH x V columns of a sub-band, then
            // the FP64 wave reduction. Column sums: FP32 over kLane32Rows rows,
            // then added to FP64.
            static_assert(kLane32Rows % RS == 0, "column runs of whole sub-bands");
            float ywf[NCH][V];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int q = 0; q < V; ++q) ywf[ch][q] = (float)ywr[0][ch][q];
            float cacc32[NCH][V];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int q = 0; q < V; ++q) cacc32[ch][q] = 0.0f;
            for (int b = 0; b < nsb; ++b) {
                const int sb = b * RS;
                // one row accumulator per chunk: shorter dependent chains
                float racc32s[NCH][RS];
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                    for (int rr = 0; rr < RS; ++rr) racc32s[ch][rr] = 0.0f;
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    float (&racc32)[RS] = racc32s[ch];
                    auto getc = pts(sb, ch);
#pragma unroll
                    for (int rr = 0; rr < RS; ++rr) {
                        const float uh_r = s_uh[sb + rr];
                        const float xw_r = s_xwf[sb + rr];
#pragma unroll
                        for (int q = 0; q < V; ++q) {
                            const float c = getc(rr, q);
                            const float t = fmaf(-Bh, c, uh_r + vh[ch][q]);
                            const float e = __builtin_amdgcn_exp2f(fmaf(-Bl, c, t));
                            if constexpr (NR > 0) racc32[rr] = fmaf(e, ywf[ch][q], racc32[rr]);
                            if constexpr (NC > 0) cacc32[ch][q] = fmaf(e, xw_r, cacc32[ch][q]);
                        }
                    }
                }
                if constexpr (NR > 0) {
                    double racc[NRA][RS];
#pragma unroll
                    for (int rr = 0; rr < RS; ++rr) {
                        float t = racc32s[0][rr];
#pragma unroll
                        for (int ch = 1; ch < NCH; ++ch) t += racc32s[ch][rr];
                        racc[0][rr] = (double)t;
                    }
                    wave_rows_out<NR, RS, MODE2>(racc, s_rf, sb, i0, n, A);
                }
                if constexpr (NC > 0) {
                    if (((b + 1) * RS) % kLane32Rows == 0 || b + 1 == nsb) {
#pragma unroll
                        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                            for (int q = 0; q < V; ++q) {
                                cacc[0][ch][q] += (double)cacc32[ch][q];
                                cacc32[ch][q] = 0.0f;
                            }
                    }
                }
            }
        } else {
            for (int b = 0; b < nsb; ++b) {
                const int sb = b * RS;
                double racc[NRA][RS];
#pragma unroll
                for (int k = 0; k < NRA; ++k)
#pragma unroll
                    for (int rr = 0; rr < RS; ++rr) racc[k][rr] = 0.0;
                compute(sb, 0, pts(sb, 0), racc);
                compute(sb, 1, pts(sb, 1), racc);
                if constexpr (NR > 0) wave_rows_out<NR, RS, MODE2>(racc, s_rf, sb, i0, n, A);
            }
        }
    }
    if constexpr (NC > 0) {
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const int64_t j = j0 + (int64_t)ch * T * V + tid * V + q;
                    if (j < m) {
                        double v = cacc[k][ch][q];
                        if constexpr (MIXED) v *= exp2((double)vl[ch][q]);
                        if (A.atomic)
                            atomicAdd(&A.col_part[(int64_t)k * m + j], v);
                        else
                            A.col_part[((int64_t)k * A.tiles_n + blockIdx.y) * m + j] = v;
                    }
                }
    }
}

template <int PREC, typename TC, int NR, int NC, int MODE2, bool VEC, int RS, int DP>
__global__ __launch_bounds__(kPassThreads) void k_pass(PassArgs A)
{
    pass_body<PREC, TC, NR, NC, MODE2, VEC, RS, DP>(A);
}

// The fused passes (row and column sums) hold the most registers; their
// occupancy request is a separate build-time tunable.
template <int PREC, typename TC, int NR, int NC, int MODE2, bool VEC, int RS, int DP>
__global__ __launch_bounds__(kPassThreads) EOT_FUSED_OCCUPANCY void k_pass_fused(PassArgs A)
{
    pass_body<PREC, TC, NR, NC, MODE2, VEC, RS, DP>(A);
}


// Mixed row-sum pass over point clouds (d = 2, 3) with the rows on the lanes:
// a workgroup takes 256 rows (one per thread) against the 2048 columns of a
// tile, whose coordinates, hi exponent parts and weights (times 2^Vl) sit in
// LDS and are read as broadcasts; every lane sums its own row, so no
// cross-lane reduction is needed (the general pass puts columns on the lanes
// and reduces each row over the wave). Each 512-column quarter of the tile
// gives one row partial, written to the slot the general pass gives its wave,
// so the outputs and their consumers are the same. The exponent is assembled
// from the same hi / lo parts on the tile's 2^-g grid. EXACT = false: sums in
// FP32 over runs of 16 columns, then FP64; EXACT = true: the FP64 weight and
// sum per entry (for CG solves to a tight residual).
constexpr int kRowsPtsRun = 16;
constexpr int64_t kRowsPtsMinGroups = 512;    // workgroups below which the general pass is used

template <int DP, bool EXACT>
__global__ __launch_bounds__(kPassThreads) void k_rows_pts(PassArgs A)
{
    static_assert(DP == 2 || DP == 3, "points in the plane or in space");
    if (A.skip && *A.skip) return;             // uniform: a finished CG chunk
    constexpr int T = kPassThreads, TC = kTileCols, Q = kTileCols / kWaves, NQ = TC / T;
    static_assert(Q % kRowsPtsRun == 0 && TC % T == 0, "tile split");
    __shared__ float4 s_c[TC];                 // y_j (zero-padded to 3) and Vh_j
    __shared__ float s_w[EXACT ? 1 : TC];      // w_j 2^Vl_j (FP32 sums)
    __shared__ double s_w64[EXACT ? TC : 1];   // w_j 2^Vl_j (FP64 sums)
    __shared__ double s_wmax[kWaves];
    const int tid = threadIdx.x;
    const int64_t n = A.n, m = A.m;
    const int64_t i = (int64_t)blockIdx.y * T + tid;
    const int64_t j0 = (int64_t)blockIdx.x * TC;
    const bool rvalid = i < n;

    // the tile's exponent grid: largest |U| of these rows, |V| of these columns
    double Ud = 0.0, mx = 0.0;
    if (rvalid) {
        Ud = kLog2e * (A.u[i] - A.a[i]);
        mx = fabs(Ud);
    }
    double Vd[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int64_t j = j0 + (int64_t)q * T + tid;
        Vd[q] = j < m ? kLog2e * A.v[j] : 0.0;
        mx = fmax(mx, fabs(Vd[q]));
    }
    mx = wave_max(mx);
    if ((tid & 63) == 0) s_wmax[tid >> 6] = mx;
    __syncthreads();
    mx = s_wmax[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) mx = fmax(mx, s_wmax[w]);
    if (!(mx < 4.0e6)) mx = 4.0e6;             // non-finite input: results flagged later
    int e2;
    frexp(2.0 * mx + 2.0, &e2);                // 2 mx + 2 < 2^e2
    const int g = 23 - e2;                     // |Uh + Vh| < 2^(23-g) on a 2^-g grid: exact
    const double sc = ldexp(1.0, g), isc = ldexp(1.0, -g);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int64_t j = j0 + (int64_t)q * T + tid;
        const double h = rint(Vd[q] * sc) * isc;
        float4 rec = make_float4(0.0f, 0.0f, 0.0f, -INFINITY);
        double w = 0.0;
        if (j < m) {
            rec.x = A.Y[j * DP];
            rec.y = A.Y[j * DP + 1];
            if constexpr (DP == 3) rec.z = A.Y[j * DP + 2];
            rec.w = (float)h;
            w = (A.yw0 ? A.yw0[j] : 1.0) * exp2((double)(float)(Vd[q] - h));
        }
        s_c[q * T + tid] = rec;
        if constexpr (EXACT) s_w64[q * T + tid] = w;
        else s_w[q * T + tid] = (float)w;
    }
    const double uhd = rint(Ud * sc) * isc;
    const float uh = rvalid ? (float)uhd : -INFINITY;
    const double rf = rvalid ? exp2(Ud - uhd) : 0.0;
    float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
    if (rvalid) {
        x0 = A.X[i * DP];
        x1 = A.X[i * DP + 1];
        if constexpr (DP == 3) x2 = A.X[i * DP + 2];
    }
    const double Bd = kLog2e * A.beta;
    const float Bh = (float)Bd;
    const float Bl = (float)(Bd - (double)Bh);
    __syncthreads();

    for (int s = 0; s < kWaves; ++s) {
        double acc = 0.0;
        for (int jb = s * Q; jb < (s + 1) * Q; jb += kRowsPtsRun) {
            float a32 = 0.0f;
#pragma unroll
            for (int k = 0; k < kRowsPtsRun; ++k) {
                const float4 rec = s_c[jb + k];
                const float d0 = x0 - rec.x, d1 = x1 - rec.y;
                float d2 = fmaf(d1, d1, d0 * d0);
                if constexpr (DP == 3) {
                    const float dz = x2 - rec.z;
                    d2 = fmaf(dz, dz, d2);
                }
                const float t = fmaf(-Bh, d2, uh + rec.w);
                const float e = __builtin_amdgcn_exp2f(fmaf(-Bl, d2, t));
                if constexpr (EXACT) acc = fma((double)e, s_w64[jb + k], acc);
                else a32 = fmaf(e, s_w[jb + k], a32);
            }
            if constexpr (!EXACT) acc += (double)a32;
        }
        if (rvalid) {
            const double out = acc * rf;
            if (A.atomic)
                atomicAdd(&A.row_part[i], out);
            else
                A.row_part[((int64_t)blockIdx.x * kWaves + s) * n + i] = out;
        }
    }
}

// Row shifts a_i ~ max_j (u_i + v_j - beta C_ij). They only keep the shifted
// row sums of the passes in range (every pass evaluates exp(x_ij - a_i) from the
// FP64 potentials, whatever a_i is), so they are computed in FP32: for |x| up
// to ~1e5 the error is ~1e-2, far inside the range guard. A block covers 256
// rows and `span` consecutive column tiles; each wave keeps per-row maxima in
// LDS; one output per (block, row): a partial [gridDim.x][n], or (A.atomic) an
// atomic max into out32[0..n) (float bits, pre-filled with -inf).
// DP > 0: C_ij = |x_i - y_j|^2 (beta already divided by the cost scale).
__device__ __forceinline__ float wave_max_f(float x)
{
    for (int off = 32; off > 0; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
    return x;
}

// atomic max of a float through the integer order of its bits
__device__ __forceinline__ void atomic_max_f32(float* addr, float val)
{
    if (val >= 0.0f)
        atomicMax(reinterpret_cast<int*>(addr), __float_as_int(val));
    else
        atomicMin(reinterpret_cast<unsigned int*>(addr), __float_as_uint(val));
}

template <typename TC, int DP, bool VEC>
__global__ __launch_bounds__(kPassThreads) void k_rowmax(PassArgs A, int span, double* part,
                                                         float* out32)
{
    constexpr int NCH = kChunks, V = kVec, T = kPassThreads, RB = kTileRows, RU = 4;
    __shared__ float s_u[RB];
    __shared__ float s_x[DP > 0 ? RB * DP : 1];
    __shared__ float s_wm[kWaves][RB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = A.n, m = A.m;
    const int rbt = A.rb;
    const int64_t i0 = (int64_t)blockIdx.y * rbt;
    const int rows = (int)(n - i0 < rbt ? n - i0 : rbt);
    if (tid < RB) {
        const int64_t i = i0 + tid;
        const bool ok = i < n;
        s_u[tid] = ok ? (float)A.u[i] : 0.0f;
        if constexpr (DP > 0) {
#pragma unroll
            for (int k = 0; k < DP; ++k) s_x[tid * DP + k] = ok ? A.X[i * DP + k] : 0.0f;
        }
        s_wm[0][tid] = s_wm[1][tid] = s_wm[2][tid] = s_wm[3][tid] = -INFINITY;
    }
    const float bf = (float)A.beta;
    const TC* __restrict__ C = static_cast<const TC*>(A.C);
    const int64_t tile_end = ((int64_t)blockIdx.x + 1) * span;
    const int64_t tiles_m = (m + kTileCols - 1) / kTileCols;
    const int64_t t_hi = tile_end < tiles_m ? tile_end : tiles_m;
    __syncthreads();
    for (int64_t t = (int64_t)blockIdx.x * span; t < t_hi; ++t) {
        const int64_t j0 = t * kTileCols;
        float vj[NCH][V];
        float yj[DP > 0 ? NCH : 1][DP > 0 ? V : 1][DP > 0 ? DP : 1];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const int64_t j = j0 + (int64_t)ch * T * V + tid * V + q;
                vj[ch][q] = j < m ? (float)A.v[j] : -INFINITY;
                if constexpr (DP > 0) {
#pragma unroll
                    for (int k = 0; k < DP; ++k) yj[ch][q][k] = j < m ? A.Y[j * DP + k] : 0.0f;
                }
            }
        for (int r0 = 0; r0 < rows; r0 += RU) {
            float mx[RU];
#pragma unroll
            for (int rr = 0; rr < RU; ++rr) {
                mx[rr] = -INFINITY;
                const int r = r0 + rr < rows ? r0 + rr : rows - 1;     // clamped, in bounds
                const float ur = s_u[r];
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int64_t jb = j0 + (int64_t)ch * T * V + tid * V;
                    float c[V];
                    if constexpr (DP == 0) {
                        if constexpr (sizeof(TC) == 4) {
                            load4<VEC>(reinterpret_cast<const float*>(C) + (i0 + r) * A.ldc, jb, m,
                                       A.ldc, c);
                        } else {
                            double cd[V];
                            load4<VEC>(reinterpret_cast<const double*>(C) + (i0 + r) * A.ldc, jb,
                                       m, A.ldc, cd);
#pragma unroll
                            for (int q = 0; q < V; ++q) c[q] = (float)cd[q];
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < V; ++q) {
                            float d2 = 0.0f;
#pragma unroll
                            for (int k = 0; k < DP; ++k) {
                                const float df = s_x[r * DP + k] - yj[ch][q][k];
                                d2 = fmaf(df, df, d2);
                            }
                            c[q] = d2;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < V; ++q)   // vj = -inf past m masks the clamped loads
                        mx[rr] = fmaxf(mx[rr], fmaf(-bf, c[q], ur + vj[ch][q]));
                }
            }
#pragma unroll
            for (int rr = 0; rr < RU; ++rr) {
                const float w = wave_max_f(mx[rr]);
                if (lane == 0 && r0 + rr < rows) s_wm[wave][r0 + rr] = fmaxf(s_wm[wave][r0 + rr], w);
            }
        }
    }
    __syncthreads();
    if (tid < rows) {
        float r = fmaxf(fmaxf(s_wm[0][tid], s_wm[1][tid]), fmaxf(s_wm[2][tid], s_wm[3][tid]));
        const int64_t i = i0 + tid;
        if (A.atomic)
            atomic_max_f32(&out32[i], r);
        else
            part[(int64_t)blockIdx.x * n + i] = (double)r;
    }
}

__global__ void k_f32_to_f64(const float* x, double* y, int64_t k)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

__global__ void k_fill_f32(float* x, float val, int64_t k)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = val;
}

__global__ void k_merge_max(const double* part, int tiles, int64_t n, double* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = part[i];
    for (int t = 1; t < tiles; ++t) r = fmax(r, part[(int64_t)t * n + i]);
    out[i] = r;
}

// ---------------------------------------------------------------- merges
__global__ void k_merge_rows(const double* part, int tiles, int64_t n, int nr, const double* a,
                             double* out0, double* out1, int sq1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ea = a ? exp(a[i]) : 1.0;
    const double ea1 = sq1 ? ea * ea : ea;
    double s0 = 0.0;
    for (int t = 0; t < tiles; ++t) s0 += part[(int64_t)t * n + i];
    if (out0) out0[i] = ea * s0;
    if (nr > 1 && out1) {
        double s1 = 0.0;
        for (int t = 0; t < tiles; ++t) s1 += part[((int64_t)tiles + t) * n + i];
        out1[i] = ea1 * s1;
    }
}

// Sum of `tiles` partials strided by m, in a fixed order: eight interleaved
// partial sums (independent loads in flight), then combined pairwise.
__device__ __forceinline__ double sum_tiles(const double* __restrict__ part, int tiles, int64_t m,
                                            int64_t j)
{
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int t = 0;
    for (; t + 8 <= tiles; t += 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] += part[(int64_t)(t + k) * m + j];
    }
    for (int k = 0; t < tiles; ++t, ++k) a[k] += part[(int64_t)t * m + j];
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Column merges: a workgroup of 256 threads sums the partials of 32
// consecutive columns, 8 threads per column, each over every 8th partial;
// the 8 group sums are added in a fixed order through LDS. Keeps many loads in
// flight when there are many row tiles (small tile heights).
constexpr int kColsPerBlock = 32, kColGroups = kVecThreads / kColsPerBlock;

__device__ __forceinline__ double col_sum_2d(const double* __restrict__ part, int tiles, int64_t m,
                                             int64_t j, double* s_p)
{
    const int c = threadIdx.x % kColsPerBlock, g = threadIdx.x / kColsPerBlock;
    double a = 0.0, b = 0.0;
    if (j < m) {
        int t = g;
        for (; t + kColGroups < tiles; t += 2 * kColGroups) {
            a += part[(int64_t)t * m + j];
            b += part[(int64_t)(t + kColGroups) * m + j];
        }
        if (t < tiles) a += part[(int64_t)t * m + j];
    }
    s_p[g * kColsPerBlock + c] = a + b;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < kColGroups; ++k) r += s_p[k * kColsPerBlock + c];
    __syncthreads();
    return r;                                   // the column total, on every group
}

__global__ void k_merge_cols(const double* part, int tiles, int64_t m, int nc, double* out0,
                             double* out1)
{
    __shared__ double s_p[kVecThreads];
    const int64_t j = (int64_t)blockIdx.x * kColsPerBlock + threadIdx.x % kColsPerBlock;
    const bool w = threadIdx.x < kColsPerBlock && j < m;
    const double s0 = col_sum_2d(part, tiles, m, j, s_p);
    if (w && out0) out0[j] = s0;
    if (nc > 1) {
        const double s1 = col_sum_2d(part + (int64_t)tiles * m, tiles, m, j, s_p);
        if (w && out1) out1[j] = s1;
    }
}

// log r(P)_i = a_i + log sum_t part[t][i]; flags[0] set when the shifted sum
// left the range where FP32 terms are exact (mixed) or is not finite.
__global__ void k_log_row(const double* part, int tiles, int64_t n, const double* a,
                          double* log_rP, int32_t* flags)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int t = 0; t < tiles; ++t) s += part[(int64_t)t * n + i];
    if (!(s > 5.421010862427522e-20 && s < 1.8446744073709552e19)) flags[0] = 1;   // 2^-64, 2^64
    log_rP[i] = a[i] + log(s);
}

// ---------------------------------------------------------------- reductions
template <int OP>
__device__ __forceinline__ double red_term(const double* x, const double* y, int64_t i)
{
    if (OP == RED_L1_DIFF_EXP) return fabs(x[i] - exp(y[i]));
    if (OP == RED_CHI2) { const double e = exp(y[i]); const double d = x[i] - e; return d * d / e; }
    if (OP == RED_DOT) return x[i] * y[i];
    if (OP == RED_SUM_EXP) return exp(y[i]);
    if (OP == RED_SUM) return x[i];
    if (OP == RED_ENTROPY) return x[i] > 0.0 ? -x[i] * log(x[i]) : 0.0;
    if (OP == RED_BAD) return (x[i] > 0.0 && x[i] < INFINITY) ? 0.0 : 1.0;
    if (OP == RED_MAXABS2) return fabs(x[i]) + fabs(y[i]);
    return fabs(x[i]);
}

__device__ __forceinline__ double block_sum(double v, double* s_w)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) s_w[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int k = 0; k < nw; ++k) r += s_w[k];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_max(double v, double* s_w)
{
    v = wave_max(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) s_w[w] = v;
    __syncthreads();
    double r = s_w[0];
    for (int k = 1; k < nw; ++k) r = fmax(r, s_w[k]);
    __syncthreads();
    return r;
}

template <int OP>
__global__ void k_reduce(const double* x, const double* y, int64_t k, double* red)
{
    __shared__ double s_w[kVecThreads / 64];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        if constexpr (OP == RED_MAXABS2) acc = fmax(acc, red_term<OP>(x, y, i));
        else acc += red_term<OP>(x, y, i);
    }
    acc = OP == RED_MAXABS2 ? block_max(acc, s_w) : block_sum(acc, s_w);
    if (threadIdx.x == 0) red[blockIdx.x] = acc;
}

__device__ __forceinline__ double sum_partials(const double* red, int nb, double* s_w)
{
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += red[b];
    return block_sum(acc, s_w);
}

__global__ void k_finish_sum(const double* red, int nb, double* dst)
{
    __shared__ double s_w[kVecThreads / 64];
    const double s = sum_partials(red, nb, s_w);
    if (threadIdx.x == 0) dst[0] = s;
}

__global__ void k_finish_max(const double* red, int nb, double* dst)
{
    __shared__ double s_w[kVecThreads / 64];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc = fmax(acc, red[b]);
    acc = block_max(acc, s_w);
    if (threadIdx.x == 0) dst[0] = acc;
}

// ---------------------------------------------------------------- elementwise
#define EW_LOOP(k) for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (k); \
                        i += (int64_t)gridDim.x * blockDim.x)

__global__ void k_scale(const double* x, double alpha, double* y, int64_t k) { EW_LOOP(k) y[i] = alpha * x[i]; }
__global__ void k_divs(const double* x, double d, double* y, int64_t k) { EW_LOOP(k) y[i] = x[i] / d; }
__global__ void k_log_ratio_fix(double* v, const double* va, const double* log_ct, const double* colsum,
                                int64_t m, int32_t* flags)
{
    EW_LOOP(m) {
        const double s = colsum[i];
        if (s > 0.0 && s < INFINITY) v[i] = va[i] + log_ct[i] - log(s);
        else { v[i] = va[i]; flags[1] = 1; }
    }
}
// Hx_i = sum_j P_ij (x_i + sqrt(rho) y_j) = r(P)_i x_i + sqrt(rho) (P y)_i
__global__ void k_hvp_rows(const double* part, int tiles, int64_t n, const double* a, double* Hx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s0 = 0.0;
    for (int t = 0; t < tiles; ++t) s0 += part[(int64_t)t * n + i];
    Hx[i] = exp(a[i]) * s0;
}
// Hy_j = sum_i P_ij (sqrt(rho) x_i + y_j) = sqrt(rho) (P^T x)_j + c(P)_j y_j
__global__ void k_hvp_cols(const double* part, int tiles, int64_t m, double* Hy)
{
    __shared__ double s_p[kVecThreads];
    const int64_t j = (int64_t)blockIdx.x * kColsPerBlock + threadIdx.x % kColsPerBlock;
    const double sj = col_sum_2d(part, tiles, m, j, s_p);
    if (threadIdx.x < kColsPerBlock && j < m) Hy[j] = sj;
}
// The Hessian-vector product with the marginals given (eqs. hessian and
// discounted-hessian): the pass summed P y over rows and P^T x over columns;
// Hx_i = r(P)_i x_i + sqrt(rho) (P y)_i, Hy_j = sqrt(rho) (P^T x)_j + c(P)_j y_j.
__global__ void k_hvp_rows_diag(const double* part, int tiles, int64_t n, const double* a,
                                double srho, const double* log_rP, const double* x, double* Hx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s0 = 0.0;
    for (int t = 0; t < tiles; ++t) s0 += part[(int64_t)t * n + i];
    Hx[i] = fma(exp(log_rP[i]), x[i], srho * (exp(a[i]) * s0));
}
__global__ void k_hvp_cols_diag(const double* part, int tiles, int64_t m, double srho,
                                const double* log_cP, const double* y, double* Hy)
{
    __shared__ double s_p[kVecThreads];
    const int64_t j = (int64_t)blockIdx.x * kColsPerBlock + threadIdx.x % kColsPerBlock;
    const double sj = col_sum_2d(part, tiles, m, j, s_p);
    if (threadIdx.x < kColsPerBlock && j < m) Hy[j] = fma(exp(log_cP[j]), y[j], srho * sj);
}
__global__ void k_axpy(double alpha, const double* x, double* y, int64_t k) { EW_LOOP(k) y[i] += alpha * x[i]; }
__global__ void k_log(const double* x, double* y, int64_t k) { EW_LOOP(k) y[i] = log(x[i]); }
__global__ void k_exp(const double* x, double* y, int64_t k) { EW_LOOP(k) y[i] = exp(x[i]); }
__global__ void k_recip(const double* x, double* y, int64_t k) { EW_LOOP(k) y[i] = 1.0 / x[i]; }
__global__ void k_copy(const double* x, double* y, int64_t k) { EW_LOOP(k) y[i] = x[i]; }
__global__ void k_fill(double* x, double val, int64_t k) { EW_LOOP(k) x[i] = val; }
__global__ void k_add_logdiff(double* x, const double* la, const double* lb, int64_t k)
{
    EW_LOOP(k) x[i] += la[i] - lb[i];
}
__global__ void k_fix_cols(double* v, const double* log_ct, const double* colsum, int64_t m,
                           int32_t* flags)
{
    EW_LOOP(m) {
        const double s = colsum[i];
        if (s > 0.0 && s < INFINITY) v[i] += log_ct[i] - log(s);
        else flags[1] = 1;
    }
}
__global__ void k_smooth(const double* x, double w, double k_inv, double* out, double* log_out,
                         int64_t k)
{
    EW_LOOP(k) {
        const double y = (1.0 - w) * x[i] + w * k_inv;
        out[i] = y;
        log_out[i] = log(y);
    }
}
__global__ void k_extrapolate(double* z, double* z_prev, double ratio, int64_t k)
{
    EW_LOOP(k) {
        const double zn = z[i] + ratio * (z[i] - z_prev[i]);
        z_prev[i] = z[i];
        z[i] = zn;
    }
}
__global__ void k_shifted(const double* base, double alpha, const double* d, double* out, int64_t k)
{
    EW_LOOP(k) out[i] = base[i] + alpha * d[i];
}
__global__ void k_newton_init(const double* log_rP, const double* r, double* rP, double* grad,
                              double* b, double* d, int64_t n)
{
    EW_LOOP(n) {
        const double e = exp(log_rP[i]);
        const double gr = e - r[i];
        rP[i] = e;
        grad[i] = gr;
        b[i] = -gr;
        d[i] = -gr / e;
    }
}
__global__ void k_forcing_resid(const double* rP, const double* d, const double* pcptd,
                                const double* grad, double* e, int64_t n)
{
    EW_LOOP(n) e[i] = rP[i] * d[i] - pcptd[i] + grad[i];
}
__global__ void k_div(const double* x, const double* y, double* out, double sign, int64_t k)
{
    EW_LOOP(k) out[i] = sign * x[i] / y[i];
}

// ---------------------------------------------------------------- CG
__global__ void k_cg_init(const double* b, const double* rP, const double* s, double rho,
                          double* d, double* res, double* z, double* p, double* M, double* ptd,
                          double* pcptd, int64_t n, int64_t m, double* red)
{
    __shared__ double s_w[kVecThreads / 64];
    double rz = 0.0, l1 = 0.0;
    const int64_t k = n > m ? n : m;
    EW_LOOP(k) {
        if (i < n) {
            // M_i >= (1 - rho) r(P)_i; at rho = 1 (the gradient's solve) a floor of
            // 2^-40 r(P)_i keeps the preconditioner finite
            const double lo = fmax(1.0 - rho, 9.094947017729282e-13) * rP[i];
            double mi = rP[i] - rho * s[i];
            mi = mi > lo ? mi : lo;
            const double bi = b[i];
            const double zi = bi / mi;
            M[i] = mi;
            d[i] = 0.0;
            res[i] = bi;
            z[i] = zi;
            p[i] = zi;
            pcptd[i] = 0.0;
            rz += bi * zi;
            l1 += fabs(bi);
        }
        if (i < m) ptd[i] = 0.0;
    }
    rz = block_sum(rz, s_w);
    l1 = block_sum(l1, s_w);
    if (threadIdx.x == 0) {
        red[blockIdx.x] = rz;
        red[gridDim.x + blockIdx.x] = l1;
    }
}

// The CG iteration kernels below all return at once when sc->done is set
// (converged, broke down or out of iterations), so the host can enqueue a
// chunk of iterations without waiting for each convergence test.

// Progress of the CG loop for a host that watches it without synchronising:
// mirror[0] = iterations done, mirror[1] = the done flag, stored into pinned
// coherent host memory (nullable). Relaxed: the host uses them only to pace
// its launches and reads the scalars back after the stream has finished, so
// no ordering is needed (a release at system scope would write back the whole
// L2 after every iteration).
__device__ __forceinline__ void cg_publish(int32_t* mirror, int32_t iters, int32_t done)
{
    if (!mirror) return;
    __hip_atomic_store(mirror, iters, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(mirror + 1, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__global__ void k_cg_init_finish(const double* red, int nb, CgScalars* sc, double tol,
                                 int32_t max_iter, int32_t* mirror)
{
    __shared__ double s_w[kVecThreads / 64];
    const double rz = sum_partials(red, nb, s_w);
    const double l1 = sum_partials(red + nb, nb, s_w);
    if (threadIdx.x == 0) {
        sc->rz = rz;
        sc->rz_new = rz;
        sc->res_l1 = l1;
        sc->alpha = 0.0;
        sc->beta = 0.0;
        sc->pq = 0.0;
        sc->tol = tol;
        sc->iters = 0;
        sc->broke = 0;
        sc->max_iter = max_iter;
        sc->done = (l1 <= tol || max_iter <= 0) ? 1 : 0;
        cg_publish(mirror, 0, sc->done);
    }
}

__global__ void k_cg_colstep(const double* part, int tiles, int64_t m, const double* c, double* w,
                             double* wc, const CgScalars* sc)
{
    if (sc && sc->done) return;                // uniform
    __shared__ double s_p[kVecThreads];
    const int64_t j = (int64_t)blockIdx.x * kColsPerBlock + threadIdx.x % kColsPerBlock;
    const double sj = col_sum_2d(part, tiles, m, j, s_p);
    if (threadIdx.x < kColsPerBlock && j < m) {
        w[j] = sj;
        wc[j] = sj / c[j];
    }
}

__global__ void k_cg_rowstep(const double* part, int tiles, int64_t n, const double* a,
                             const double* rP, const double* p, double rho, double* t, double* q,
                             double* red, const CgScalars* sc)
{
    if (sc->done) return;
    __shared__ double s_w[kVecThreads / 64];
    double pq = 0.0;
    EW_LOOP(n) {
        const double s = sum_tiles(part, tiles, n, i);
        const double ti = exp(a[i]) * s;
        const double qi = rP[i] * p[i] - rho * ti;
        t[i] = ti;
        q[i] = qi;
        pq += p[i] * qi;
    }
    pq = block_sum(pq, s_w);
    if (threadIdx.x == 0) red[blockIdx.x] = pq;
}

// alpha = rz / <p, q>; d += alpha p; res -= alpha q; z = res / M; recurrences
// for P D(c)^-1 P^T d (n) and P^T d (m); partials of <res, z> and ||res||_1.
__global__ void k_cg_update(const double* red_pq, int nb_pq, double* d, double* res, double* z,
                            const double* p, const double* q, const double* M, const double* t,
                            double* pcptd, const double* w, double* ptd, int64_t n, int64_t m,
                            double* red, CgScalars* sc)
{
    if (sc->done) return;
    __shared__ double s_w[kVecThreads / 64];
    const double pq = sum_partials(red_pq, nb_pq, s_w);
    const double alpha = sc->rz / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->pq = pq;
        sc->alpha = alpha;
    }
    double rz = 0.0, l1 = 0.0;
    const int64_t k = n > m ? n : m;
    EW_LOOP(k) {
        if (i < n) {
            d[i] += alpha * p[i];
            const double ri = res[i] - alpha * q[i];
            res[i] = ri;
            const double zi = ri / M[i];
            z[i] = zi;
            pcptd[i] += alpha * t[i];
            rz += ri * zi;
            l1 += fabs(ri);
        }
        if (i < m) ptd[i] += alpha * w[i];
    }
    rz = block_sum(rz, s_w);
    l1 = block_sum(l1, s_w);
    if (threadIdx.x == 0) {
        red[blockIdx.x] = rz;
        red[gridDim.x + blockIdx.x] = l1;
    }
}

// beta = rz_new / rz; p = z + beta p. rz itself is replaced by the single
// thread of the tail kernel below, after every block has read it.
__global__ void k_cg_direction(const double* red, int nb, const double* z, double* p, int64_t n,
                               CgScalars* sc)
{
    if (sc->done) return;
    __shared__ double s_w[kVecThreads / 64];
    const double rz_new = sum_partials(red, nb, s_w);
    const double beta = rz_new / sc->rz;
    EW_LOOP(n) p[i] = z[i] + beta * p[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->rz_new = rz_new;
        sc->beta = beta;
    }
}

// End of one CG iteration: ||res||_1, the iteration count and the stop test.
__global__ void k_cg_tail(const double* red, int nb, CgScalars* sc, int32_t* mirror)
{
    if (sc->done) return;
    __shared__ double s_w[kVecThreads / 64];
    const double l1 = sum_partials(red + nb, nb, s_w);
    if (threadIdx.x == 0) {
        sc->res_l1 = l1;
        sc->rz = sc->rz_new;
        sc->iters += 1;
        if (!(fabs(sc->alpha) < INFINITY) || !(sc->pq > 0.0)) {
            sc->broke = 1;
            sc->done = 1;
        } else if (l1 <= sc->tol || sc->iters >= sc->max_iter) {
            sc->done = 1;
        }
        cg_publish(mirror, sc->iters, sc->done);
    }
}

// The rest of one CG iteration for small problems, in one workgroup of 1024
// threads: the row step, the update, the new direction and the stop test of
// k_cg_rowstep / k_cg_update / k_cg_direction / k_cg_tail, with workgroup
// reductions in place of the grid-wide partial sums (a different but fixed
// summation order). Saves three launches per iteration.
constexpr int kCgSmallThreads = 1024;

__device__ __forceinline__ double block_sum_small(double v, double* s_w)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_w[wave] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < kCgSmallThreads / 64; ++k) r += s_w[k];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kCgSmallThreads) void k_cg_small(
    const double* part, int tiles, int64_t n, int64_t m, const double* a, const double* rP,
    double* p, double rho, double* t, double* q, double* d, double* res, double* z,
    const double* M, double* pcptd, const double* w, double* ptd, CgScalars* sc, int32_t* mirror)
{
    if (sc->done) return;
    __shared__ double s_w[kCgSmallThreads / 64];
    const int tid = threadIdx.x;
    double pq = 0.0;
    for (int64_t i = tid; i < n; i += kCgSmallThreads) {
        const double ti = exp(a[i]) * sum_tiles(part, tiles, n, i);
        const double qi = rP[i] * p[i] - rho * ti;
        t[i] = ti;
        q[i] = qi;
        pq += p[i] * qi;
    }
    pq = block_sum_small(pq, s_w);
    const double rz_old = sc->rz;
    const double alpha = rz_old / pq;
    double rz = 0.0, l1 = 0.0;
    const int64_t k = n > m ? n : m;
    for (int64_t i = tid; i < k; i += kCgSmallThreads) {
        if (i < n) {
            d[i] += alpha * p[i];
            const double ri = res[i] - alpha * q[i];
            res[i] = ri;
            const double zi = ri / M[i];
            z[i] = zi;
            pcptd[i] += alpha * t[i];
            rz += ri * zi;
            l1 += fabs(ri);
        }
        if (i < m) ptd[i] += alpha * w[i];
    }
    rz = block_sum_small(rz, s_w);
    l1 = block_sum_small(l1, s_w);
    const double beta = rz / rz_old;
    for (int64_t i = tid; i < n; i += kCgSmallThreads) p[i] = z[i] + beta * p[i];
    if (tid == 0) {
        sc->pq = pq;
        sc->alpha = alpha;
        sc->rz_new = rz;
        sc->beta = beta;
        sc->res_l1 = l1;
        sc->rz = rz;
        sc->iters += 1;
        if (!(fabs(alpha) < INFINITY) || !(pq > 0.0)) {
            sc->broke = 1;
            sc->done = 1;
        } else if (l1 <= sc->tol || sc->iters >= sc->max_iter) {
            sc->done = 1;
        }
        cg_publish(mirror, sc->iters, sc->done);
    }
}

inline int vec_blocks(int64_t k)
{
    int64_t b = (k + kVecThreads - 1) / kVecThreads;
    if (b < 1) b = 1;
    if (b > kMaxRedBlocks) b = kMaxRedBlocks;
    return (int)b;
}

inline int col_blocks(int64_t m)
{
    return (int)((m + kColsPerBlock - 1) / kColsPerBlock);
}

inline int map_blocks(int64_t k)
{
    int64_t b = (k + kVecThreads - 1) / kVecThreads;
    return (int)(b < 1 ? 1 : b);
}

template <typename TC, int NR, int NC, int MODE2, bool VEC, int DP>
hipError_t launch_pass_v(const PassArgs& a, int prec, hipStream_t s)
{
    constexpr bool FUSED = MODE2 == R2_HVP || (NR > 0 && NC > 0);
    constexpr int RS = FUSED ? kSubRowsFused : kSubRows;
    // mixed point-cloud passes: their own sub-band height
    constexpr int RSM = DP > 0 ? (FUSED ? kPtsSubRowsFused : kPtsSubRows) : RS;
    // mixed point-cloud row sums: the rows-on-lanes kernel
    constexpr bool ROWS_PTS = DP > 0 && NR == 1 && NC == 0 && MODE2 == R2_WEIGHT;
    dim3 grid((unsigned)a.tiles_m, (unsigned)a.tiles_n);
    if (prec == EOT_PREC_MIXED) {
        if constexpr (sizeof(TC) == 4) {
            if constexpr (ROWS_PTS) {
                // 256 rows per workgroup: only where that still gives a full grid
                const int64_t gy = (a.n + kPassThreads - 1) / kPassThreads;
                if ((int64_t)a.tiles_m * gy >= kRowsPtsMinGroups) {
                    const dim3 g2((unsigned)a.tiles_m, (unsigned)gy);
                    if (a.exact_sums)
                        hipLaunchKernelGGL((k_rows_pts<DP, true>), g2, dim3(kPassThreads), 0, s, a);
                    else
                        hipLaunchKernelGGL((k_rows_pts<DP, false>), g2, dim3(kPassThreads), 0, s, a);
                    return hipGetLastError();
                }
            }
            if constexpr (FUSED)
                hipLaunchKernelGGL((k_pass_fused<EOT_PREC_MIXED, TC, NR, NC, MODE2, VEC, RSM, DP>),
                                   grid, dim3(kPassThreads), 0, s, a);
            else
                hipLaunchKernelGGL((k_pass<EOT_PREC_MIXED, TC, NR, NC, MODE2, VEC, RSM, DP>), grid,
                                   dim3(kPassThreads), 0, s, a);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        if constexpr (FUSED)
            hipLaunchKernelGGL((k_pass_fused<EOT_PREC_FP64, TC, NR, NC, MODE2, VEC, RS, DP>), grid,
                               dim3(kPassThreads), 0, s, a);
        else
            hipLaunchKernelGGL((k_pass<EOT_PREC_FP64, TC, NR, NC, MODE2, VEC, RS, DP>), grid,
                               dim3(kPassThreads), 0, s, a);
    }
    return hipGetLastError();
}

template <typename TC, int NR, int NC, int MODE2>
hipError_t launch_pass_t(const PassArgs& a, int prec, hipStream_t s)
{
    if (a.kind == EOT_COST_SQEUCLID_POINTS) {
        if constexpr (sizeof(TC) == 4) {
            if (a.d == 2) return launch_pass_v<TC, NR, NC, MODE2, true, 2>(a, prec, s);
            if (a.d == 3) return launch_pass_v<TC, NR, NC, MODE2, true, 3>(a, prec, s);
        }
        return hipErrorInvalidValue;
    }
    return a.vec_ok ? launch_pass_v<TC, NR, NC, MODE2, true, 0>(a, prec, s)
                    : launch_pass_v<TC, NR, NC, MODE2, false, 0>(a, prec, s);
}

template <typename TC>
hipError_t dispatch_pass(const PassArgs& a, int prec, int nr, int nc, int mode2, hipStream_t s)
{
    // Instantiated combinations (nr, nc, mode2); the mode-specific ones first.
    if (nr == 1 && nc == 1 && mode2 == R2_HVP) return launch_pass_t<TC, 1, 1, R2_HVP>(a, prec, s);
    if (nr == 1 && nc == 1) return launch_pass_t<TC, 1, 1, R2_WEIGHT>(a, prec, s);
    if (nr == 2 && nc == 1 && mode2 == R2_SQUARE) return launch_pass_t<TC, 2, 1, R2_SQUARE>(a, prec, s);
    if (nr == 2 && nc == 2 && mode2 == R2_WEIGHT) return launch_pass_t<TC, 2, 2, R2_WEIGHT>(a, prec, s);
    if (nr == 2 && nc == 1 && mode2 == R2_COST) return launch_pass_t<TC, 2, 1, R2_COST>(a, prec, s);
    if (nr == 2 && nc == 2 && mode2 == R2_COST) return launch_pass_t<TC, 2, 2, R2_COST>(a, prec, s);
    if (nr == 2 && nc == 0 && mode2 == R2_SQUARE) return launch_pass_t<TC, 2, 0, R2_SQUARE>(a, prec, s);
    if (nr == 2 && nc == 0 && mode2 == R2_COST) return launch_pass_t<TC, 2, 0, R2_COST>(a, prec, s);
    if (nr == 1 && nc == 0) return launch_pass_t<TC, 1, 0, R2_WEIGHT>(a, prec, s);
    if (nr == 0 && nc == 1) return launch_pass_t<TC, 0, 1, R2_WEIGHT>(a, prec, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- gradients
// Cotangent of a dense cost: G_ij = P_ij (ra_i + cb_j + kappa C_ij), FP64,
// written row-major with leading dimension ldg. One thread: 4 consecutive
// columns of kGradRows rows.
constexpr int kGradRows = 16;

template <typename TC>
__global__ __launch_bounds__(256) void k_plan_grad(const TC* __restrict__ C, int64_t ldc, int64_t n,
                                                   int64_t m, const double* __restrict__ u,
                                                   const double* __restrict__ v, double beta,
                                                   const double* __restrict__ ra,
                                                   const double* __restrict__ cb, double kappa,
                                                   double* __restrict__ G, int64_t ldg)
{
    const int64_t j0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    const int64_t i0 = (int64_t)blockIdx.y * kGradRows;
    if (j0 >= m) return;
    double vj[4], bj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool ok = j0 + q < m;
        vj[q] = ok ? v[j0 + q] : 0.0;
        bj[q] = ok ? cb[j0 + q] : 0.0;
    }
    for (int r = 0; r < kGradRows; ++r) {
        const int64_t i = i0 + r;
        if (i >= n) break;
        const double ui = u[i], ai = ra[i];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t j = j0 + q;
            if (j < m) {
                const double c = (double)C[i * ldc + j];
                const double P = exp(fma(-beta, c, ui + vj[q]));
                G[i * ldg + j] = P * fma(kappa, c, ai + bj[q]);
            }
        }
    }
}

// Row sums of the point-cloud cotangent G_ij = P_ij (ra_i + cb_j + kappa D_ij)
// with D_ij = |x_i - y_j|^2 (the cost scale folded into beta and kappa):
// g0_i += sum_j G_ij and gy[k]_i += sum_j G_ij y_jk over this block's column
// slice, FP64, accumulated atomically. One thread per row; the column slice is
// staged through LDS 256 points at a time. Called once per side (rows = x with
// columns = y, then rows = y with columns = x).
template <int DP>
__global__ __launch_bounds__(256) void k_points_grad_rows(
    const float* __restrict__ Xr, const float* __restrict__ Yc, int64_t n, int64_t m,
    const double* __restrict__ u, const double* __restrict__ v, double beta,
    const double* __restrict__ ra, const double* __restrict__ cb, double kappa, int64_t slice,
    double* g0, double* gy0, double* gy1, double* gy2)
{
    __shared__ double s_y[256][DP];
    __shared__ double s_v[256], s_b[256];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    const bool ok = i < n;
    double xi[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) xi[k] = ok ? (double)Xr[i * DP + k] : 0.0;
    const double ui = ok ? u[i] : 0.0, ai = ok ? ra[i] : 0.0;
    double acc0 = 0.0, accy[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) accy[k] = 0.0;
    const int64_t jb = (int64_t)blockIdx.y * slice;
    const int64_t je = jb + slice < m ? jb + slice : m;
    for (int64_t j0 = jb; j0 < je; j0 += 256) {
        __syncthreads();
        const int64_t j = j0 + tid;
        const bool jok = j < je;
#pragma unroll
        for (int k = 0; k < DP; ++k) s_y[tid][k] = jok ? (double)Yc[j * DP + k] : 0.0;
        s_v[tid] = jok ? v[j] : -INFINITY;
        s_b[tid] = jok ? cb[j] : 0.0;
        __syncthreads();
        const int cnt = (int)(je - j0 < 256 ? je - j0 : 256);
        for (int t = 0; t < cnt; ++t) {
            double d2 = 0.0;
#pragma unroll
            for (int k = 0; k < DP; ++k) {
                const double df = xi[k] - s_y[t][k];
                d2 = fma(df, df, d2);
            }
            const double P = exp(fma(-beta, d2, ui + s_v[t]));
            const double Gv = P * fma(kappa, d2, ai + s_b[t]);
            acc0 += Gv;
#pragma unroll
            for (int k = 0; k < DP; ++k) accy[k] = fma(Gv, s_y[t][k], accy[k]);
        }
    }
    if (!ok) return;
    atomicAdd(&g0[i], acc0);
    atomicAdd(&gy0[i], accy[0]);
    if constexpr (DP > 1) atomicAdd(&gy1[i], accy[1]);
    if constexpr (DP > 2) atomicAdd(&gy2[i], accy[2]);
}

// grad_i,k = (2 / s) (x_ik g0_i - gy[k]_i), row-major n x d output.
__global__ void k_points_grad_finish(const float* X, int64_t n, int d, double two_over_s,
                                     const double* g0, const double* gy0, const double* gy1,
                                     const double* gy2, double* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* gy[3] = {gy0, gy1, gy2};
    for (int k = 0; k < d; ++k)
        out[i * d + k] = two_over_s * ((double)X[i * d + k] * g0[i] - gy[k][i]);
}

// out = alpha x + beta y + c0 (x, y nullable)
__global__ void k_lincomb(double* out, int64_t k, double alpha, const double* x, double beta,
                          const double* y, double c0)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        double t = c0;
        if (x) t = fma(alpha, x[i], t);
        if (y) t = fma(beta, y[i], t);
        out[i] = t;
    }
}

// Rounding onto U(r, c): out = t / s clipped to 1 (1 where s = 0), and the
// marginal deficits t - x s.
__global__ void k_round_scale(const double* t, const double* sum, double* out, int64_t k)
{
    EW_LOOP(k) out[i] = sum[i] > 0.0 ? fmin(1.0, t[i] / sum[i]) : 1.0;
}
__global__ void k_round_err(const double* t, const double* x, const double* sum, double* out,
                            int64_t k)
{
    EW_LOOP(k) out[i] = t[i] - (x ? x[i] : 1.0) * sum[i];
}

// Dense rounded plan: out_ij = x_i P_ij y_j + er_i ec_j / |er|_1, FP64.
template <typename TC>
__global__ __launch_bounds__(256) void k_plan_round(const TC* __restrict__ C, int64_t ldc,
                                                    int64_t n, int64_t m,
                                                    const double* __restrict__ u,
                                                    const double* __restrict__ v, double beta,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ er,
                                                    const double* __restrict__ ec, double inv_nr,
                                                    double* __restrict__ out, int64_t ldo)
{
    const int64_t j0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    const int64_t i0 = (int64_t)blockIdx.y * kGradRows;
    if (j0 >= m) return;
    double vj[4], yj[4], ej[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool ok = j0 + q < m;
        vj[q] = ok ? v[j0 + q] : 0.0;
        yj[q] = ok ? y[j0 + q] : 0.0;
        ej[q] = ok ? ec[j0 + q] * inv_nr : 0.0;
    }
    for (int r = 0; r < kGradRows; ++r) {
        const int64_t i = i0 + r;
        if (i >= n) break;
        const double ui = u[i], xi = x[i], ei = er[i];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t j = j0 + q;
            if (j < m) {
                const double P = exp(fma(-beta, (double)C[i * ldc + j], ui + vj[q]));
                out[i * ldo + j] = fma(xi * P, yj[q], ei * ej[q]);
            }
        }
    }
}

}  // namespace

hipError_t launch_plan_grad(const PassArgs& a, const double* ra, const double* cb, double kappa,
                            double* G, int64_t ldg, hipStream_t s)
{
    dim3 grid((unsigned)((a.m + 1023) / 1024), (unsigned)((a.n + kGradRows - 1) / kGradRows));
    if (a.kind == EOT_COST_DENSE_F32)
        hipLaunchKernelGGL((k_plan_grad<float>), grid, dim3(256), 0, s,
                           static_cast<const float*>(a.C), a.ldc, a.n, a.m, a.u, a.v, a.beta, ra,
                           cb, kappa, G, ldg);
    else if (a.kind == EOT_COST_DENSE_F64)
        hipLaunchKernelGGL((k_plan_grad<double>), grid, dim3(256), 0, s,
                           static_cast<const double*>(a.C), a.ldc, a.n, a.m, a.u, a.v, a.beta, ra,
                           cb, kappa, G, ldg);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_points_grad_rows(const float* Xr, const float* Yc, int d, int64_t n, int64_t m,
                                   const double* u, const double* v, double beta, const double* ra,
                                   const double* cb, double kappa, double* g0, double* gy0,
                                   double* gy1, double* gy2, hipStream_t s)
{
    const int64_t bx = (n + 255) / 256;
    const int64_t col_blocks = (m + 255) / 256;
    int64_t by = (4096 + bx - 1) / bx;                 // aim at >= 4096 workgroups
    by = by < 1 ? 1 : (by > col_blocks ? col_blocks : by);
    const int64_t slice = ((m + by - 1) / by + 255) / 256 * 256;
    by = (m + slice - 1) / slice;
    dim3 grid((unsigned)bx, (unsigned)by);
    if (d == 2)
        hipLaunchKernelGGL((k_points_grad_rows<2>), grid, dim3(256), 0, s, Xr, Yc, n, m, u, v,
                           beta, ra, cb, kappa, slice, g0, gy0, gy1, gy2);
    else if (d == 3)
        hipLaunchKernelGGL((k_points_grad_rows<3>), grid, dim3(256), 0, s, Xr, Yc, n, m, u, v,
                           beta, ra, cb, kappa, slice, g0, gy0, gy1, gy2);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_points_grad_finish(const float* X, int64_t n, int d, double two_over_s,
                                     const double* g0, const double* gy0, const double* gy1,
                                     const double* gy2, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_points_grad_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X,
                       n, d, two_over_s, g0, gy0, gy1, gy2, out);
    return hipGetLastError();
}

hipError_t launch_plan_round(const PassArgs& a, const double* x, const double* y, const double* er,
                             const double* ec, double inv_nr, double* out, int64_t ldo,
                             hipStream_t s)
{
    dim3 grid((unsigned)((a.m + 1023) / 1024), (unsigned)((a.n + kGradRows - 1) / kGradRows));
    if (a.kind == EOT_COST_DENSE_F32)
        hipLaunchKernelGGL((k_plan_round<float>), grid, dim3(256), 0, s,
                           static_cast<const float*>(a.C), a.ldc, a.n, a.m, a.u, a.v, a.beta, x, y,
                           er, ec, inv_nr, out, ldo);
    else if (a.kind == EOT_COST_DENSE_F64)
        hipLaunchKernelGGL((k_plan_round<double>), grid, dim3(256), 0, s,
                           static_cast<const double*>(a.C), a.ldc, a.n, a.m, a.u, a.v, a.beta, x, y,
                           er, ec, inv_nr, out, ldo);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_lincomb(double* out, int64_t k, double alpha, const double* x, double beta,
                          const double* y, double c0, hipStream_t s)
{
    const int64_t b = (k + 255) / 256;
    hipLaunchKernelGGL(k_lincomb, dim3((unsigned)(b < 1024 ? b : 1024)), dim3(256), 0, s, out, k,
                       alpha, x, beta, y, c0);
    return hipGetLastError();
}

// ---------------------------------------------------------------- pass timer
namespace {
struct PassTiming {
    hipEvent_t start, stop;
    int nr, nc, prec, hvp;
};
std::mutex g_timing_mu;
bool g_timing_on = false;
std::vector<PassTiming> g_timings;

void clear_timings_locked()
{
    for (auto& t : g_timings) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    g_timings.clear();
}
}  // namespace

bool pass_timing_on()
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    return g_timing_on;
}

hipError_t set_pass_timing(bool on)
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    clear_timings_locked();
    g_timing_on = on;
    return hipSuccess;
}

hipError_t read_pass_timing(int nr, int nc, int prec, int hvp, int64_t* launches, double* ms)
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    int64_t k = 0;
    double tot = 0.0;
    for (auto& t : g_timings) {
        if ((nr >= 0 && t.nr != nr) || (nc >= 0 && t.nc != nc) || (prec >= 0 && t.prec != prec) ||
            (hvp >= 0 && t.hvp != hvp))
            continue;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e != hipSuccess) return e;
        float x = 0.0f;
        e = hipEventElapsedTime(&x, t.start, t.stop);
        if (e != hipSuccess) return e;
        tot += x;
        ++k;
    }
    *launches = k;
    *ms = tot;
    return hipSuccess;
}

hipError_t launch_pass(const PassArgs& a, int prec, int nr, int nc, int mode2, hipStream_t s)
{
    auto go = [&]() -> hipError_t {
        if (is_high_d(a)) return launch_pass_hd(a, prec, nr, nc, mode2, s);
        if (a.kind == EOT_COST_DENSE_F32 || a.kind == EOT_COST_SQEUCLID_POINTS)
            return dispatch_pass<float>(a, prec, nr, nc, mode2, s);
        if (a.kind == EOT_COST_DENSE_F64) return dispatch_pass<double>(a, prec, nr, nc, mode2, s);
        return hipErrorInvalidValue;
    };
    bool timed;
    {
        std::lock_guard<std::mutex> lk(g_timing_mu);
        timed = g_timing_on;
    }
    if (!timed) return go();
    PassTiming t{nullptr, nullptr, nr, nc, prec, mode2 == R2_HVP ? 1 : 0};
    hipError_t e = hipEventCreate(&t.start);
    if (e == hipSuccess) e = hipEventCreate(&t.stop);
    if (e == hipSuccess) e = hipEventRecord(t.start, s);
    if (e != hipSuccess) return e;
    e = go();
    if (e != hipSuccess) return e;
    e = hipEventRecord(t.stop, s);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_timing_mu);
    g_timings.push_back(t);
    return hipSuccess;
}

hipError_t launch_rowmax(const PassArgs& a, double* part, double* out, hipStream_t s)
{
    if (is_high_d(a)) return launch_rowmax_hd(a, part, out, s);
    // a block spans `span` column tiles so that at most 64 partials (or atomics) per row remain
    const int span = (a.tiles_m + 63) / 64;
    const int gx = (a.tiles_m + span - 1) / span;
    dim3 grid((unsigned)gx, (unsigned)a.tiles_n);
    float* out32 = reinterpret_cast<float*>(part);     // atomic mode: n floats of scratch
    if (a.atomic)
        hipLaunchKernelGGL(k_fill_f32, dim3(vec_blocks(a.n)), dim3(kVecThreads), 0, s, out32,
                           -INFINITY, a.n);
    const bool vec = a.vec_ok != 0;
    if (a.kind == EOT_COST_DENSE_F32) {
        if (vec)
            hipLaunchKernelGGL((k_rowmax<float, 0, true>), grid, dim3(kPassThreads), 0, s, a, span, part, out32);
        else
            hipLaunchKernelGGL((k_rowmax<float, 0, false>), grid, dim3(kPassThreads), 0, s, a, span, part, out32);
    } else if (a.kind == EOT_COST_DENSE_F64) {
        if (vec)
            hipLaunchKernelGGL((k_rowmax<double, 0, true>), grid, dim3(kPassThreads), 0, s, a, span, part, out32);
        else
            hipLaunchKernelGGL((k_rowmax<double, 0, false>), grid, dim3(kPassThreads), 0, s, a, span, part, out32);
    } else if (a.kind == EOT_COST_SQEUCLID_POINTS && a.d == 2) {
        hipLaunchKernelGGL((k_rowmax<float, 2, false>), grid, dim3(kPassThreads), 0, s, a, span, part, out32);
    } else if (a.kind == EOT_COST_SQEUCLID_POINTS && a.d == 3) {
        hipLaunchKernelGGL((k_rowmax<float, 3, false>), grid, dim3(kPassThreads), 0, s, a, span, part, out32);
    } else {
        return hipErrorInvalidValue;
    }
    if (a.atomic)
        hipLaunchKernelGGL(k_f32_to_f64, dim3(vec_blocks(a.n)), dim3(kVecThreads), 0, s, out32,
                           out, a.n);
    else
        hipLaunchKernelGGL(k_merge_max, dim3(map_blocks(a.n)), dim3(kVecThreads), 0, s, part, gx,
                           a.n, out);
    return hipGetLastError();
}

hipError_t launch_merge_rows(const double* part, int tiles, int64_t n, int nr, const double* a,
                             double* out0, double* out1, int sq1, hipStream_t s)
{
    hipLaunchKernelGGL(k_merge_rows, dim3(map_blocks(n)), dim3(kVecThreads), 0, s, part, tiles, n,
                       nr, a, out0, out1, sq1);
    return hipGetLastError();
}

hipError_t launch_merge_cols(const double* part, int tiles, int64_t m, int nc, double* out0,
                             double* out1, hipStream_t s)
{
    hipLaunchKernelGGL(k_merge_cols, dim3(col_blocks(m)), dim3(kVecThreads), 0, s, part, tiles, m,
                       nc, out0, out1);
    return hipGetLastError();
}

hipError_t launch_log_row_from_sums(const double* part, int tiles, int64_t n, const double* a,
                                    double* log_rP, int32_t* flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_log_row, dim3(map_blocks(n)), dim3(kVecThreads), 0, s, part, tiles, n, a,
                       log_rP, flags);
    return hipGetLastError();
}

hipError_t launch_reduce(int op, const double* x, const double* y, int64_t k, double* red,
                         int* nb_out, hipStream_t s)
{
    const int nb = vec_blocks(k);
    *nb_out = nb;
    dim3 g(nb), b(kVecThreads);
    switch (op) {
        case RED_L1_DIFF_EXP: hipLaunchKernelGGL(k_reduce<RED_L1_DIFF_EXP>, g, b, 0, s, x, y, k, red); break;
        case RED_CHI2: hipLaunchKernelGGL(k_reduce<RED_CHI2>, g, b, 0, s, x, y, k, red); break;
        case RED_DOT: hipLaunchKernelGGL(k_reduce<RED_DOT>, g, b, 0, s, x, y, k, red); break;
        case RED_SUM_EXP: hipLaunchKernelGGL(k_reduce<RED_SUM_EXP>, g, b, 0, s, x, y, k, red); break;
        case RED_SUM: hipLaunchKernelGGL(k_reduce<RED_SUM>, g, b, 0, s, x, y, k, red); break;
        case RED_ENTROPY: hipLaunchKernelGGL(k_reduce<RED_ENTROPY>, g, b, 0, s, x, y, k, red); break;
        case RED_L1: hipLaunchKernelGGL(k_reduce<RED_L1>, g, b, 0, s, x, y, k, red); break;
        case RED_BAD: hipLaunchKernelGGL(k_reduce<RED_BAD>, g, b, 0, s, x, y, k, red); break;
        case RED_MAXABS2: hipLaunchKernelGGL(k_reduce<RED_MAXABS2>, g, b, 0, s, x, y, k, red); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finish_sum(const double* red, int nb, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_sum, dim3(1), dim3(kVecThreads), 0, s, red, nb, dst);
    return hipGetLastError();
}

hipError_t launch_finish_max(const double* red, int nb, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_max, dim3(1), dim3(kVecThreads), 0, s, red, nb, dst);
    return hipGetLastError();
}

#define EW_LAUNCH(kern, k, ...)                                                                  \
    do {                                                                                         \
        hipLaunchKernelGGL(kern, dim3(vec_blocks(k)), dim3(kVecThreads), 0, s, __VA_ARGS__);   \
        return hipGetLastError();                                                                \
    } while (0)

hipError_t launch_scale(const double* x, double alpha, double* y, int64_t k, hipStream_t s) { EW_LAUNCH(k_scale, k, x, alpha, y, k); }
hipError_t launch_divs(const double* x, double d, double* y, int64_t k, hipStream_t s) { EW_LAUNCH(k_divs, k, x, d, y, k); }
hipError_t launch_log_ratio_fix(double* v, const double* va, const double* log_ct, const double* colsum, int64_t m, int32_t* flags, hipStream_t s) { EW_LAUNCH(k_log_ratio_fix, m, v, va, log_ct, colsum, m, flags); }
hipError_t launch_hvp_finish(const double* row_part, int tiles_m, const double* col_part, int tiles_n,
                             int64_t n, int64_t m, const double* a, double* Hx, double* Hy, hipStream_t s)
{
    hipLaunchKernelGGL(k_hvp_rows, dim3(map_blocks(n)), dim3(kVecThreads), 0, s, row_part, tiles_m, n, a, Hx);
    hipLaunchKernelGGL(k_hvp_cols, dim3(col_blocks(m)), dim3(kVecThreads), 0, s, col_part, tiles_n, m, Hy);
    return hipGetLastError();
}
hipError_t launch_hvp_finish_diag(const double* row_part, int tiles_m, const double* col_part,
                                  int tiles_n, int64_t n, int64_t m, const double* a, double srho,
                                  const double* log_rP, const double* log_cP, const double* x,
                                  const double* y, double* Hx, double* Hy, hipStream_t s)
{
    hipLaunchKernelGGL(k_hvp_rows_diag, dim3(map_blocks(n)), dim3(kVecThreads), 0, s, row_part,
                       tiles_m, n, a, srho, log_rP, x, Hx);
    hipLaunchKernelGGL(k_hvp_cols_diag, dim3(col_blocks(m)), dim3(kVecThreads), 0, s, col_part,
                       tiles_n, m, srho, log_cP, y, Hy);
    return hipGetLastError();
}
hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t k, hipStream_t s) { EW_LAUNCH(k_axpy, k, alpha, x, y, k); }
hipError_t launch_log(const double* x, double* y, int64_t k, hipStream_t s) { EW_LAUNCH(k_log, k, x, y, k); }
hipError_t launch_exp(const double* x, double* y, int64_t k, hipStream_t s) { EW_LAUNCH(k_exp, k, x, y, k); }
hipError_t launch_recip(const double* x, double* y, int64_t k, hipStream_t s) { EW_LAUNCH(k_recip, k, x, y, k); }
hipError_t launch_copy(const double* x, double* y, int64_t k, hipStream_t s) { EW_LAUNCH(k_copy, k, x, y, k); }
hipError_t launch_fill(double* x, double val, int64_t k, hipStream_t s) { EW_LAUNCH(k_fill, k, x, val, k); }
hipError_t launch_add_logdiff(double* x, const double* la, const double* lb, int64_t k, hipStream_t s) { EW_LAUNCH(k_add_logdiff, k, x, la, lb, k); }
hipError_t launch_fix_cols(double* v, const double* log_ct, const double* colsum, int64_t m, int32_t* flags, hipStream_t s) { EW_LAUNCH(k_fix_cols, m, v, log_ct, colsum, m, flags); }
hipError_t launch_smooth(const double* x, double w, double k_inv, double* out, double* log_out, int64_t k, hipStream_t s) { EW_LAUNCH(k_smooth, k, x, w, k_inv, out, log_out, k); }
hipError_t launch_extrapolate(double* z, double* z_prev, double ratio, int64_t k, hipStream_t s) { EW_LAUNCH(k_extrapolate, k, z, z_prev, ratio, k); }
hipError_t launch_shifted(const double* base, double alpha, const double* d, double* out, int64_t k, hipStream_t s) { EW_LAUNCH(k_shifted, k, base, alpha, d, out, k); }
hipError_t launch_newton_init(const double* log_rP, const double* r, double* rP, double* grad, double* b, double* d, int64_t n, hipStream_t s) { EW_LAUNCH(k_newton_init, n, log_rP, r, rP, grad, b, d, n); }
hipError_t launch_forcing_resid(const double* rP, const double* d, const double* pcptd, const double* grad, double* e, int64_t n, hipStream_t s) { EW_LAUNCH(k_forcing_resid, n, rP, d, pcptd, grad, e, n); }
hipError_t launch_div(const double* x, const double* y, double* out, double sign, int64_t k, hipStream_t s) { EW_LAUNCH(k_div, k, x, y, out, sign, k); }

hipError_t launch_cg_init(const double* b, const double* rP, const double* s_, double rho, double* d,
                          double* res, double* z, double* p, double* M, double* ptd, double* pcptd,
                          int64_t n, int64_t m, double* red, CgScalars* sc, double tol,
                          int32_t max_iter, int32_t* mirror, hipStream_t s)
{
    const int nb = vec_blocks(n > m ? n : m);
    hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(kVecThreads), 0, s, b, rP, s_, rho, d, res, z, p,
                       M, ptd, pcptd, n, m, red);
    hipLaunchKernelGGL(k_cg_init_finish, dim3(1), dim3(kVecThreads), 0, s, red, nb, sc, tol,
                       max_iter, mirror);
    return hipGetLastError();
}

hipError_t launch_cg_colstep(const double* part, int tiles, int64_t m, const double* c, double* w,
                             double* wc, const CgScalars* sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_colstep, dim3(col_blocks(m)), dim3(kVecThreads), 0, s, part, tiles, m,
                       c, w, wc, sc);
    return hipGetLastError();
}

hipError_t launch_cg_rowstep(const double* part, int tiles, int64_t n, const double* a,
                             const double* rP, const double* p, double rho, double* t, double* q,
                             double* red, int* nb, const CgScalars* sc, hipStream_t s)
{
    *nb = vec_blocks(n);
    hipLaunchKernelGGL(k_cg_rowstep, dim3(*nb), dim3(kVecThreads), 0, s, part, tiles, n, a, rP, p,
                       rho, t, q, red, sc);
    return hipGetLastError();
}

hipError_t launch_cg_update(const double* red_pq, int nb_pq, double* d, double* res, double* z,
                            const double* p, const double* q, const double* M, const double* t,
                            double* pcptd, const double* w, double* ptd, int64_t n, int64_t m,
                            double* red, int* nb, CgScalars* sc, hipStream_t s)
{
    *nb = vec_blocks(n > m ? n : m);
    hipLaunchKernelGGL(k_cg_update, dim3(*nb), dim3(kVecThreads), 0, s, red_pq, nb_pq, d, res, z,
                       p, q, M, t, pcptd, w, ptd, n, m, red, sc);
    return hipGetLastError();
}

hipError_t launch_cg_direction(const double* red, int nb, const double* z, double* p, int64_t n,
                               CgScalars* sc, int32_t* mirror, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_direction, dim3(vec_blocks(n)), dim3(kVecThreads), 0, s, red, nb, z, p,
                       n, sc);
    hipLaunchKernelGGL(k_cg_tail, dim3(1), dim3(kVecThreads), 0, s, red, nb, sc, mirror);
    return hipGetLastError();
}

hipError_t launch_cg_small(const double* part, int tiles, int64_t n, int64_t m, const double* a,
                           const double* rP, double* p, double rho, double* t, double* q,
                           double* d, double* res, double* z, const double* M, double* pcptd,
                           const double* w, double* ptd, CgScalars* sc, int32_t* mirror,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_small, dim3(1), dim3(kCgSmallThreads), 0, s, part, tiles, n, m, a, rP,
                       p, rho, t, q, d, res, z, M, pcptd, w, ptd, sc, mirror);
    return hipGetLastError();
}

hipError_t launch_round_scale(const double* t, const double* sum, double* out, int64_t k,
                              hipStream_t s)
{
    EW_LAUNCH(k_round_scale, k, t, sum, out, k);
}

hipError_t launch_round_err(const double* t, const double* x, const double* sum, double* out,
                            int64_t k, hipStream_t s)
{
    EW_LAUNCH(k_round_err, k, t, x, sum, out, k);
}

}  // namespace eot
