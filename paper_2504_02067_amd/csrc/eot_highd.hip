// Streaming passes for high-dimensional point clouds (d = 16, 32, 48, 64):
// C_ij = |x_i - y_j|^2 / s recomputed on the fly as |x_i|^2 + |y_j|^2 -
// 2 x_i . y_j, with the x . y contraction on the matrix cores. Three kernels:
//
//  * k_pass_hd_mx16 (mixed precision, every sum except cost-weighted ones):
//    FP32 coordinates split once per call as x = xh + xl (xh = bf16(x), xl =
//    bf16(x - xh)), stored zero-padded to whole 32-dimension chunks;
//    x . y ~ xh.yh + xh.yl + xl.yh, three v_mfma_f32_16x16x32_bf16 per chunk
//    with FP32 accumulation (the dropped xl.yl term is ~2^-16 relative).
//    Per-pass tables hold the rows' and columns' exponent parts; column
//    operands are copied global -> LDS by DMA, double-buffered. Details at the
//    kernel.
//  * k_pass_hd_f64 (FP64 mode and row maxima): x . y from
//    v_mfma_f64_16x16x4_f64, norms and exp in FP64.
//  * k_pass_hd (the mixed cost-weighted sums, and the fallback when a point
//    array is not 16-byte aligned): the 32 x 32 BF16 hi/lo products staged per
//    step in mixed mode, |x - y|^2 per entry in FP64 (difference form) in FP64.
//
// Lane layout of the 32 x 32 BF16 MFMA result used by k_pass_hd (checked on the
// target): lane l holds the entries (row 8 (r / 4) + 4 (l / 32) + r % 4, column
// l % 32), r = 0..15; operand A lane l supplies row l % 32, dimensions
// 8 (l / 32) + 0..7 of each 16-dimension chunk, operand B lane l the same
// dimensions of column l % 32.

#include <hip/hip_runtime.h>
#include <math.h>

#include "eot_internal.h"
#include "eot_lanes.h"

namespace eot {
namespace {

constexpr int kHdRows = kHdTileRows;        // 128: 4 waves x 32 rows
constexpr int kHdStep = 32;
constexpr int kHdMaxD = 64;
constexpr double kLog2eHd = 1.4426950408889634074;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ double hd_wave_max(double x)
{
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}


// OP = 0: the pass (sums); OP = 1: row maxima of u_i + v_j - beta C_ij (FP32,
// a range shift only), into part[blockIdx.x][n] or atomically into out32.
template <int PREC, int NR, int NC, int MODE2, int OP>
__global__ __launch_bounds__(256) void k_pass_hd(PassArgs A, float* out32)
{
    if (A.skip && *A.skip) return;
    constexpr bool MIXED = PREC == EOT_PREC_MIXED;
    constexpr bool MAXOP = OP == 1;
    constexpr int NRA = NR > 0 ? NR : 1, NCA = NC > 0 ? NC : 1;
    __shared__ float s_x[MIXED && !MAXOP ? 1 : kHdRows * kHdMaxD];   // FP64 / max: row points
    __shared__ float s_y[MIXED && !MAXOP ? 1 : kHdStep * kHdMaxD];   // FP64 / max: step columns
    __shared__ float s_xx[kHdRows];
    __shared__ float s_uh[kHdRows];
    __shared__ double s_A[kHdRows];
    __shared__ double s_rf[kHdRows];
    __shared__ double s_xw[2][kHdRows];
    __shared__ double s_rr[kHdRows];
    __shared__ double s_col[kWaves][NCA][kHdStep];
    __shared__ double s_wmax[kWaves];
    // mixed: the step's 32 columns as BF16 hi / lo, rows padded by 8 (no bank conflicts)
    constexpr int kLd = kHdMaxD + 8;
    __shared__ __attribute__((aligned(16))) __bf16 s_bh[MIXED && !MAXOP ? kHdStep * kLd : 1];
    __shared__ __attribute__((aligned(16))) __bf16 s_bl[MIXED && !MAXOP ? kHdStep * kLd : 1];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n = A.n, m = A.m;
    const int d = A.d;
    const int kch = d / 16;
    const int64_t i0 = (int64_t)blockIdx.y * kHdRows;
    const int64_t j0 = (int64_t)blockIdx.x * A.hd_cols;

    // ---- prologue: row values (LDS), the tile's exponent grid (mixed)
    const int64_t irow = i0 + tid;
    const bool rvalid = tid < kHdRows && irow < n;
    double arow = 0.0, Ud = 0.0, uh = 0.0, ul = 0.0, sc = 1.0, isc = 1.0;
    if (tid < kHdRows) {
        if constexpr (MIXED && !MAXOP) {
            s_xx[tid] = rvalid ? A.hd_xx[irow] : 0.0f;
        } else {
            for (int k = 0; k < d; ++k) s_x[tid * kHdMaxD + k] = rvalid ? A.X[irow * d + k] : 0.0f;
        }
    }
    if constexpr (MIXED && !MAXOP) {
        double mx = 0.0;
        for (int c = tid; c < A.hd_cols; c += 256) {
            const int64_t j = j0 + c;
            if (j < m) mx = fmax(mx, fabs(kLog2eHd * A.v[j]));
        }
        if (rvalid) {
            arow = A.a[irow];
            Ud = kLog2eHd * (A.u[irow] - arow);
            mx = fmax(mx, fabs(Ud));
        }
        mx = hd_wave_max(mx);
        if (lane == 0) s_wmax[wave] = mx;
        __syncthreads();
        mx = fmax(fmax(s_wmax[0], s_wmax[1]), fmax(s_wmax[2], s_wmax[3]));
        if (!(mx < 4.0e6)) mx = 4.0e6;
        int e2;
        frexp(2.0 * mx + 2.0, &e2);
        const int g = 23 - e2;
        sc = ldexp(1.0, g);
        isc = ldexp(1.0, -g);
        uh = rint(Ud * sc) * isc;
        ul = Ud - uh;
    } else if (rvalid) {
        arow = MAXOP ? 0.0 : A.a[irow];
    }
    if (tid < kHdRows) {
        if (rvalid) {
            const double rf = MIXED && !MAXOP ? exp2(ul) : 1.0;
            const double R = MAXOP ? 0.0 : exp(arow) * rf;
            s_uh[tid] = MAXOP ? (float)A.u[irow] : (float)uh;
            s_A[tid] = MIXED ? 0.0 : A.u[irow] - arow;
            s_rf[tid] = rf;
            s_rr[tid] = R;
            if constexpr (MODE2 == R2_HVP) {
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
    }
    __syncthreads();

    // ---- this wave's 32 rows: MFMA operand A (mixed) for every 16-dimension chunk
    const int rl = lane & 31, half = lane >> 5;
    const int64_t arow_i = i0 + wave * 32 + rl;
    bf16x8 ah[kHdMaxD / 16], al[kHdMaxD / 16];
    if constexpr (MIXED && !MAXOP) {
        const __bf16* xh = static_cast<const __bf16*>(A.hd_xh);
        const __bf16* xl = static_cast<const __bf16*>(A.hd_xl);
        const bool ok = arow_i < n;
#pragma unroll
        for (int kc = 0; kc < kHdMaxD / 16; ++kc) {
            if (kc < kch) {
                const int64_t off = arow_i * hd_padded_dim(d) + kc * 16 + 8 * half;
                if (ok) {
                    ah[kc] = *reinterpret_cast<const bf16x8*>(xh + off);
                    al[kc] = *reinterpret_cast<const bf16x8*>(xl + off);
                } else {
#pragma unroll
                    for (int t = 0; t < 8; ++t) ah[kc][t] = al[kc][t] = (__bf16)0.0f;
                }
            }
        }
    }
    // rows of the 16 result entries of this lane (tile-local)
    int rowl[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) rowl[r] = wave * 32 + 8 * (r / 4) + 4 * half + (r % 4);

    const double Bd = kLog2eHd * A.beta;
    const float Bh = (float)Bd;
    const float Bl = (float)(Bd - (double)Bh);
    const double beta = A.beta;
    const double srho = A.hvp_srho;

    double racc[NRA][16];
#pragma unroll
    for (int k = 0; k < NRA; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) racc[k][r] = MAXOP ? -INFINITY : 0.0;

    // mixed: one 16-byte chunk of a step's columns per thread (32 columns x d / 8 chunks <= 256)
    const int per = d / 8;
    const int sc_c = tid / (per > 0 ? per : 1), sc_q = tid % (per > 0 ? per : 1);
    const bool stager = tid < kHdStep * per;

    const int nsteps = A.hd_cols / kHdStep;
    for (int st = 0; st < nsteps; ++st) {
        const int64_t jc = j0 + (int64_t)st * kHdStep;
        if (jc >= m) break;                                  // uniform
        const int64_t j = jc + rl;                           // this lane's column
        const bool jok = j < m;
        // column values of this lane
        float vh = -INFINITY, vl = 0.0f, vf = -INFINITY;
        double vc = -INFINITY;
        double yw0 = 0.0, yw1 = 0.0;
        if (jok) {
            const double Vd = kLog2eHd * A.v[j];
            if constexpr (MIXED && !MAXOP) {
                const double h = rint(Vd * sc) * isc;
                vh = (float)h;
                vl = (float)(Vd - h);
            }
            vf = (float)A.v[j];
            vc = A.v[j];
            if constexpr (MODE2 == R2_HVP) {
                yw0 = A.yw1[j];
            } else {
                yw0 = A.yw0 ? A.yw0[j] : 1.0;
                yw1 = A.yw1 ? A.yw1[j] : 1.0;
            }
        }
        // squared distances of the lane's 16 entries
        float d2f[16];
        double d2d[16];
        if constexpr (MIXED && !MAXOP) {
            // stage the step's columns (BF16 hi / lo) once for the 4 waves
            __syncthreads();
            if (stager) {
                const int64_t jj = jc + sc_c;
                bf16x8 h8, l8;
                if (jj < m) {
                    const int64_t o = jj * hd_padded_dim(d) + sc_q * 8;
                    h8 = *reinterpret_cast<const bf16x8*>(static_cast<const __bf16*>(A.hd_yh) + o);
                    l8 = *reinterpret_cast<const bf16x8*>(static_cast<const __bf16*>(A.hd_yl) + o);
                } else {
#pragma unroll
                    for (int t = 0; t < 8; ++t) h8[t] = l8[t] = (__bf16)0.0f;
                }
                *reinterpret_cast<bf16x8*>(&s_bh[sc_c * kLd + sc_q * 8]) = h8;
                *reinterpret_cast<bf16x8*>(&s_bl[sc_c * kLd + sc_q * 8]) = l8;
            }
            __syncthreads();
            const float yy = jok ? A.hd_yy[j] : 0.0f;
            f32x16 acc = {};
#pragma unroll
            for (int kc = 0; kc < kHdMaxD / 16; ++kc) {
                if (kc < kch) {
                    const int o = rl * kLd + kc * 16 + 8 * half;
                    const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&s_bh[o]);
                    const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&s_bl[o]);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[kc], bh, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[kc], bl, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[kc], bh, acc, 0, 0, 0);
                }
            }
#pragma unroll
            for (int r = 0; r < 16; ++r)
                d2f[r] = fmaxf(s_xx[rowl[r]] + yy - 2.0f * acc[r], 0.0f);
        } else {
            // stage this step's 32 columns in LDS, then per-entry difference form
            __syncthreads();
            for (int e = tid; e < kHdStep * d; e += 256) {
                const int c = e / d, k = e % d;
                const int64_t jj = jc + c;
                s_y[c * kHdMaxD + k] = jj < m ? A.Y[jj * d + k] : 0.0f;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                if constexpr (MAXOP) {
                    float acc = 0.0f;
                    for (int k = 0; k < d; ++k) {
                        const float df = s_x[rowl[r] * kHdMaxD + k] - s_y[rl * kHdMaxD + k];
                        acc = fmaf(df, df, acc);
                    }
                    d2f[r] = acc;
                } else {
                    double acc = 0.0;
                    for (int k = 0; k < d; ++k) {
                        const double df =
                            (double)s_x[rowl[r] * kHdMaxD + k] - (double)s_y[rl * kHdMaxD + k];
                        acc = fma(df, df, acc);
                    }
                    d2d[r] = acc;
                }
            }
        }
        // epilogue: plan entries, row and column accumulation
        double cacc[NCA];
#pragma unroll
        for (int k = 0; k < NCA; ++k) cacc[k] = 0.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = rowl[r];
            if constexpr (MAXOP) {
                const float x = fmaf(-(float)beta, d2f[r], s_uh[row] + vf);
                racc[0][r] = fmax(racc[0][r], (double)x);
                continue;
            } else {
                double e64, cd;
                if constexpr (MIXED) {
                    const float c = d2f[r];
                    const float t = fmaf(-Bh, c, s_uh[row] + vh);
                    const float w = fmaf(-Bl, c, vl);
                    e64 = (double)__builtin_amdgcn_exp2f(t + w);
                    cd = (double)c;
                } else {
                    const double c = d2d[r];
                    e64 = exp(fma(-beta, c, s_A[row] + vc));
                    cd = c;
                }
                const double xw0 = s_xw[0][row], xw1 = s_xw[1][row];
                if constexpr (MODE2 == R2_HVP) {
                    racc[0][r] = fma(e64, fma(srho, yw0, xw1), racc[0][r]);
                    cacc[0] = fma(e64, fma(s_rr[row], yw0, xw0), cacc[0]);
                } else {
                    if constexpr (NR >= 1) racc[0][r] = fma(e64, yw0, racc[0][r]);
                    if constexpr (NR >= 2) {
                        double term = e64;
                        if constexpr (MODE2 == R2_SQUARE) term = e64 * e64;
                        if constexpr (MODE2 == R2_COST) term = e64 * cd;
                        racc[NR - 1][r] = fma(term, yw1, racc[NR - 1][r]);
                    }
                    if constexpr (NC >= 1) cacc[0] = fma(e64, xw0, cacc[0]);
                    if constexpr (NC >= 2) {
                        const double term = MODE2 == R2_COST ? e64 * cd : e64;
                        cacc[NC - 1] = fma(term, xw1, cacc[NC - 1]);
                    }
                }
            }
        }
        if constexpr (NC > 0 && !MAXOP) {
            // the wave's 32-row column sums: both lane halves, then the 4 waves
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const double tot = cacc[k] + __shfl_xor(cacc[k], 32, 64);
                if (half == 0) s_col[wave][k][rl] = tot;
            }
            __syncthreads();
            if (tid < kHdStep) {
                const int64_t jj = jc + tid;
                if (jj < m) {
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        const double v =
                            (s_col[0][k][tid] + s_col[1][k][tid]) + (s_col[2][k][tid] + s_col[3][k][tid]);
                        if (A.atomic)
                            atomicAdd(&A.col_part[(int64_t)k * m + jj], v);
                        else
                            A.col_part[((int64_t)k * A.tiles_n + blockIdx.y) * m + jj] = v;
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---- row outputs: reduce each of the lane's 16 rows over the 32 lanes of its half
    if constexpr (NR > 0 || MAXOP) {
#pragma unroll
        for (int k = 0; k < NRA; ++k) {
            if constexpr (!MAXOP) {
                if (k >= NR) break;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                double v = racc[k][r];
#pragma unroll
                for (int off = 16; off > 0; off >>= 1) {
                    const double o = __shfl_xor(v, off, 64);
                    v = MAXOP ? fmax(v, o) : v + o;
                }
                racc[k][r] = v;
            }
            if (rl == 0) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = rowl[r];
                    const int64_t i = i0 + row;
                    if (i >= n) continue;
                    if constexpr (MAXOP) {
                        const float x = (float)racc[0][r];
                        if (A.atomic) {
                            if (x >= 0.0f)
                                atomicMax(reinterpret_cast<int*>(&out32[i]), __float_as_int(x));
                            else
                                atomicMin(reinterpret_cast<unsigned int*>(&out32[i]), __float_as_uint(x));
                        } else {
                            A.row_part[(int64_t)blockIdx.x * n + i] = (double)x;
                        }
                    } else {
                        double fac = s_rf[row];
                        if (k == 1 && MODE2 == R2_SQUARE) fac *= fac;
                        const double v = racc[k][r] * fac;
                        if (A.atomic)
                            atomicAdd(&A.row_part[(int64_t)k * n + i], v);
                        else
                            A.row_part[((int64_t)k * A.tiles_m + blockIdx.x) * n + i] = v;
                    }
                }
            }
        }
    }
}


// ---- mixed precision: per-pass tables, then the matrix-core pass ---------------
// The norms are folded into the potentials before the hi / lo split:
//     log2 P_ij - a_i log2 e = (U_i - B |x_i|^2) + (V_j - B |y_j|^2) + 2 B x_i . y_j
// with B = log2(e) beta / s. Two small kernels per pass split every
// U_i - B |x_i|^2 and V_j - B |y_j|^2 into a hi part on one grid 2^-g (from
// the largest magnitude, so that Uh + Vh is exact in FP32) and a lo part,
// and store per row the hi part, the FP32 weights and the FP64 factor 2^Ul,
// per column a 16-byte record {Vh, 2^Vl, row weight(s)}. A plan entry then
// costs e = exp2(fma(2B, xy, Uh_i + Vh_j)) with xy the MFMA result (the lo
// part of 2B would move the exponent by at most 2^-24 2B |x . y|, far below
// the BF16 hi / lo error of xy, and is dropped), and 2^Vl_j multiplies the
// column weights and the column totals.

__global__ __launch_bounds__(256) void k_hd_grid_max(PassArgs A)
{
    const double Bd = kLog2eHd * A.beta;
    double mx = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += stride)
        mx = fmax(mx, fabs(kLog2eHd * (A.u[i] - A.a[i]) - Bd * (double)A.hd_xx[i]));
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < A.m; j += stride)
        mx = fmax(mx, fabs(kLog2eHd * A.v[j] - Bd * (double)A.hd_yy[j]));
    __shared__ double s_w[4];
    mx = hd_wave_max(mx);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) A.hd_gpart[blockIdx.x] = fmax(fmax(s_w[0], s_w[1]), fmax(s_w[2], s_w[3]));
}

// hvp: rows {Uh, x, R, R sqrt(rho) x}, columns {Vh, f, sqrt(rho) y f, y};
// otherwise rows {Uh, R xw0, R xw1}, columns {Vh, f, yw0 f, yw1 f (f^2 if sq)}.
__global__ __launch_bounds__(256) void k_hd_tables(PassArgs A, int nparts, int hvp, int nr, int nc,
                                                    int sq)
{
    __shared__ double s_w[4];
    double mx = 0.0;
    for (int t = threadIdx.x; t < nparts; t += blockDim.x) mx = fmax(mx, A.hd_gpart[t]);
    mx = hd_wave_max(mx);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(s_w[0], s_w[1]), fmax(s_w[2], s_w[3]));
    if (!(mx < 4.0e6)) mx = 4.0e6;             // non-finite input: results flagged later
    int e2;
    frexp(2.0 * mx + 2.0, &e2);
    const int g = 23 - e2;                       // |Uh + Vh| < 2^(23 - g) on a 2^-g grid: exact
    const double sc = ldexp(1.0, g), isc = ldexp(1.0, -g);
    const double Bd = kLog2eHd * A.beta;
    const double srho = A.hvp_srho;
    const int64_t np = A.hd_npad, mp = (int64_t)A.tiles_m * A.hd_cols;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    float* rt = A.hd_rt;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
        float r0 = -INFINITY, r1 = 0.0f, r2 = 0.0f, r3 = 0.0f;
        double rf = 0.0;
        if (i < A.n) {
            const double a = A.a[i];
            const double U = kLog2eHd * (A.u[i] - a) - Bd * (double)A.hd_xx[i];
            const double uh = rint(U * sc) * isc;
            rf = exp2(U - uh);
            const double R = exp(a) * rf;
            r0 = (float)uh;
            if (hvp) {
                const double x = A.xw1[i];
                r1 = (float)x;
                r2 = (float)R;
                r3 = (float)(R * srho * x);
            } else {
                if (nc >= 1) r1 = (float)(R * (A.xw0 ? A.xw0[i] : 1.0));
                if (nc >= 2) r2 = (float)(R * (A.xw1 ? A.xw1[i] : 1.0));
            }
        }
        rt[i] = r0;
        rt[np + i] = r1;
        rt[2 * np + i] = r2;
        rt[3 * np + i] = r3;
        A.hd_rf[i] = rf;
    }
    float4* ct = static_cast<float4*>(A.hd_ct);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < mp; j += stride) {
        float4 rec = make_float4(-INFINITY, 1.0f, 0.0f, 0.0f);
        if (j < A.m) {
            const double V = kLog2eHd * A.v[j] - Bd * (double)A.hd_yy[j];
            const double vh = rint(V * sc) * isc;
            const double f = exp2(V - vh);
            rec.x = (float)vh;
            rec.y = (float)f;
            if (hvp) {
                const double y = A.yw1[j];
                rec.z = (float)(srho * y * f);
                rec.w = (float)y;
            } else {
                if (nr >= 1) rec.z = (float)((A.yw0 ? A.yw0[j] : 1.0) * f);
                if (nr >= 2) rec.w = (float)((A.yw1 ? A.yw1[j] : 1.0) * (sq ? f * f : f));
            }
        }
        ct[j] = rec;
    }
}

// The pass, with v_mfma_f32_16x16x32_bf16 over the zero-padded 32-dimension
// chunks of the BF16 copies (d = 16 .. 64 -> 1 or 2 chunks). A workgroup owns
// 128 rows x hd_cols columns; each wave owns two 16-row blocks and takes 16
// columns per step, and each lane keeps the table values of its 8 result rows
// in registers for the whole tile. Lane layout (checked on the target): A[i][k]
// in lane i + 16 (k / 8), element k % 8; B[k][j] in lane j + 16 (k / 8), element
// k % 8; D[i][j] in lane j + 16 (i / 4), element i % 4. The columns go through
// LDS in blocks of 64 (4 steps), double-buffered: the next block (BF16 operands
// and the column records) is copied global -> LDS by the DMA path (no
// registers) while the current one is computed, one barrier per block. A block
// is stored as 1 KB fragments in the MFMA operand's lane order (the 64 records
// are one more fragment), so the copy writes linearly and the reads are
// conflict-free. Within a lane, the 8 entries of a step (column sums) and the
// tile's steps (row sums) accumulate in FP32; every sum across lanes, waves and
// tiles is FP64.
constexpr int kHd16Step = 16;
constexpr int kHd16Blk = 64;
constexpr int kHd16Steps = kHd16Blk / kHd16Step;

template <int NR, int NC, int MODE2, int KC2>
__global__ __launch_bounds__(256) EOT_HD_OCCUPANCY void k_pass_hd_mx16(PassArgs A)
{
    static_assert(KC2 == 1 || KC2 == 2, "KC2 = d / 32");
    if (A.skip && *A.skip) return;
    constexpr bool HVP = MODE2 == R2_HVP;
    constexpr int NV = HVP ? 4 : 1 + NC;
    constexpr int NRA = NR > 0 ? NR : 1, NCA = NC > 0 ? NC : 1;
    constexpr int d = KC2 * 32;
    // [buffer][hi, lo][step][chunk][lane]: 16 bytes each
    __shared__ __attribute__((aligned(16))) bf16x8 s_b[2][2][kHd16Steps][KC2][64];
    __shared__ __attribute__((aligned(16))) float4 s_rec[2][kHd16Blk];
    __shared__ float s_cp[2][NCA][kWaves][kHd16Blk];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int jl = lane & 15, g = lane >> 4;
    const int64_t n = A.n, m = A.m;
    const int64_t i0 = (int64_t)blockIdx.y * kHdRows;
    const int64_t j0 = (int64_t)blockIdx.x * A.hd_cols;
    const __bf16* yh = static_cast<const __bf16*>(A.hd_yh);
    const __bf16* yl = static_cast<const __bf16*>(A.hd_yl);
    const float4* ct = static_cast<const float4*>(A.hd_ct);

    auto copy_block = [&](int blk, int p) {
        const int64_t jb = j0 + (int64_t)blk * kHd16Blk;
        constexpr int NF = 2 * kHd16Steps * KC2;
#pragma unroll
        for (int f = wave; f < NF + 1; f += kWaves) {
            if (f == NF) {                                   // the block's records
                lds_dma16(ct + jb + lane, lds_addr(&s_rec[p][0]));
                continue;
            }
            const int hl = f / (kHd16Steps * KC2), st = (f / KC2) % kHd16Steps, kc = f % KC2;
            int64_t j = jb + st * kHd16Step + jl;
            j = j < m ? j : m - 1;                           // finite filler past m
            const __bf16* src = (hl ? yl : yh) + j * d + kc * 32 + 8 * g;
            lds_dma16(src, lds_addr(&s_b[p][hl][st][kc][0]));
        }
    };
    copy_block(0, 0);

    // the lane's 8 result rows: block b, rows 4 g + r
    float rv[NV][8];
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t i = i0 + wave * 32 + 16 * b + 4 * g;
            const float4 t4 = *reinterpret_cast<const float4*>(A.hd_rt + k * A.hd_npad + i);
            rv[k][4 * b + 0] = t4.x;
            rv[k][4 * b + 1] = t4.y;
            rv[k][4 * b + 2] = t4.z;
            rv[k][4 * b + 3] = t4.w;
        }
    // MFMA operand A: block b, row 16 b + jl, dimensions 32 kc + 8 g .. + 7
    bf16x8 ah[2][KC2], al[2][KC2];
    {
        const __bf16* xh = static_cast<const __bf16*>(A.hd_xh);
        const __bf16* xl = static_cast<const __bf16*>(A.hd_xl);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t ai = i0 + wave * 32 + 16 * b + jl;
#pragma unroll
            for (int kc = 0; kc < KC2; ++kc) {
                if (ai < n) {
                    const int64_t off = ai * d + kc * 32 + 8 * g;
                    ah[b][kc] = *reinterpret_cast<const bf16x8*>(xh + off);
                    al[b][kc] = *reinterpret_cast<const bf16x8*>(xl + off);
                } else {
#pragma unroll
                    for (int t = 0; t < 8; ++t) ah[b][kc][t] = al[b][kc][t] = (__bf16)0.0f;
                }
            }
        }
    }
    const float B2 = (float)(2.0 * kLog2eHd * A.beta);
    float racc[NRA][8];
#pragma unroll
    for (int k = 0; k < NRA; ++k)
#pragma unroll
        for (int r = 0; r < 8; ++r) racc[k][r] = 0.0f;
    __builtin_amdgcn_s_waitcnt(0);             // block 0 has landed in LDS
    __syncthreads();

    typedef float f32x4 __attribute__((ext_vector_type(4)));
    const int64_t cols = m - j0 < A.hd_cols ? m - j0 : A.hd_cols;
    const int nblk = (int)((cols + kHd16Blk - 1) / kHd16Blk);
    for (int blk = 0; blk < nblk; ++blk) {
        const int p = blk & 1;
        if (blk + 1 < nblk) copy_block(blk + 1, p ^ 1);
#pragma unroll 1
        for (int st = 0; st < kHd16Steps; ++st) {
            const int c = st * kHd16Step + jl;               // this lane's column in the block
            const float4 rec = s_rec[p][c];
            f32x4 acc[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[b] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kc = 0; kc < KC2; ++kc) {
                const bf16x8 bh = s_b[p][0][st][kc][lane];
                const bf16x8 bl = s_b[p][1][st][kc][lane];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[b][kc], bh, acc[b], 0, 0, 0);
                    acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[b][kc], bl, acc[b], 0, 0, 0);
                    acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[b][kc], bh, acc[b], 0, 0, 0);
                }
            }
            float cacc[NCA];
#pragma unroll
            for (int k = 0; k < NCA; ++k) cacc[k] = 0.0f;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
#pragma unroll
                for (int r4 = 0; r4 < 4; ++r4) {
                    const int r = 4 * b + r4;
                    const float e = __builtin_amdgcn_exp2f(fmaf(B2, acc[b][r4], rv[0][r] + rec.x));
                    if constexpr (HVP) {
                        racc[0][r] = fmaf(e, fmaf(rv[1][r], rec.y, rec.z), racc[0][r]);
                        cacc[0] = fmaf(e, fmaf(rv[2][r], rec.w, rv[3][r]), cacc[0]);
                    } else {
                        if constexpr (NR >= 1) racc[0][r] = fmaf(e, rec.z, racc[0][r]);
                        if constexpr (NR >= 2)
                            racc[1][r] = fmaf(MODE2 == R2_SQUARE ? e * e : e, rec.w, racc[1][r]);
                        if constexpr (NC >= 1) cacc[0] = fmaf(e, rv[1][r], cacc[0]);
                        if constexpr (NC >= 2) cacc[1] = fmaf(e, rv[2][r], cacc[1]);
                    }
                }
            }
            if constexpr (NC > 0) {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    const float tot = quad_total_f32(cacc[k]);
                    if (g == 0) s_cp[p][k][wave][c] = tot;
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);         // the next block has landed in LDS
        __syncthreads();
        if constexpr (NC > 0) {
            if (tid < kHd16Blk) {
                const int64_t j = j0 + (int64_t)blk * kHd16Blk + tid;
                if (j < m) {
                    const double f = (double)s_rec[p][tid].y;
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        const double t = ((double)s_cp[p][k][0][tid] + (double)s_cp[p][k][1][tid]) +
                                         ((double)s_cp[p][k][2][tid] + (double)s_cp[p][k][3][tid]);
                        if (A.atomic)
                            atomicAdd(&A.col_part[(int64_t)k * m + j], t * f);
                        else
                            A.col_part[((int64_t)k * A.tiles_n + blockIdx.y) * m + j] = t * f;
                    }
                }
            }
        }
    }

    // ---- row totals: the 16 lanes of a group g hold the same 8 rows
    if constexpr (NR > 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                double x = (double)racc[k][r];
                x += dpp_f64<kDppXor1>(x);
                x += dpp_f64<kDppXor2>(x);
                x += dpp_f64<kDppHalfMirror>(x);
                x += dpp_f64<kDppMirror>(x);
                if (jl == 0) {
                    const int64_t i = i0 + wave * 32 + 16 * (r / 4) + 4 * g + (r % 4);
                    if (i < n) {
                        double fac = A.hd_rf[i];
                        if (k == 1 && MODE2 == R2_SQUARE) fac *= fac;
                        if (A.atomic)
                            atomicAdd(&A.row_part[(int64_t)k * n + i], x * fac);
                        else
                            A.row_part[((int64_t)k * A.tiles_m + blockIdx.x) * n + i] = x * fac;
                    }
                }
            }
        }
    }
}

// ---- FP64: x . y on the FP64 matrix cores -----------------------------------
// v_mfma_f64_16x16x4_f64 (IEEE FP64 products and sums; lane layout checked on the
// target: A[i][k] from lane i + 16 k, B[k][j] from lane j + 16 k, D[i][j] in lane
// j + 16 (i % 4), element i / 4). The shared dimension is permuted so that lane
// group g = l / 16 supplies dimensions g D4 .. g D4 + D4 - 1 (one per product),
// which makes each lane's operand slice contiguous; the products are then
//     u_i - a_i + v_j - beta |x_i - y_j|^2
//   = ((u_i - a_i) - beta |x_i|^2) + (v_j - beta |y_j|^2) + 2 beta x_i . y_j
// with the norms in FP64, and exp in FP64. A workgroup owns 128 rows (the FP32
// points staged in LDS, converted exactly when read); each wave owns two 16-row
// blocks and walks the tile's columns 16 at a time, its next step's column
// operands loaded during the current step. Column sums reduce over the 4 lane
// groups in registers and over the waves in LDS, one barrier per 128 columns.
constexpr int kF64Blk = 128;
constexpr int kF64Step = 16;

// OP = 1: row maxima of u_i + v_j - beta C_ij (FP64; no row shift, no sums), into
// part[blockIdx.x][n] or atomically into out32 (FP32, a range shift only).
template <int NR, int NC, int MODE2, int D4, int OP = 0>
__global__ __launch_bounds__(256) void k_pass_hd_f64(PassArgs A, float* out32)
{
    constexpr bool MAXOP = OP == 1;
    if (A.skip && *A.skip) return;
    constexpr bool HVP = MODE2 == R2_HVP;
    constexpr int d = 4 * D4;
    constexpr int XS = d + 1;                          // padded row stride (floats)
    constexpr int NRA = NR > 0 ? NR : 1, NCA = NC > 0 ? NC : 1;
    __shared__ float s_x[kHdRows * XS];
    __shared__ double s_E[kHdRows];                    // (u - a) - beta |x|^2
    __shared__ double s_xx[kHdRows];                   // |x|^2
    __shared__ double s_w0[kHdRows], s_w1[kHdRows];    // column weights (R_i included)
    __shared__ double s_hx[kHdRows];                   // HVP: x_i
    __shared__ double s_cp[2][NCA][kWaves][kF64Blk];
    __shared__ __attribute__((aligned(16))) double s_exp[MAXOP ? 2 : kExpTabDoubles];  // exp_tab256

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int jl = lane & 15, g = lane >> 4;
    const int64_t n = A.n, m = A.m;
    const int64_t i0 = (int64_t)blockIdx.y * kHdRows;
    const int64_t j0 = (int64_t)blockIdx.x * A.hd_cols;
    const double beta = A.beta;                        // 1 / (temperature x scale)
    const double srho = A.hvp_srho;

    // ---- the tile's rows: points in LDS, per-row values
    if constexpr (!MAXOP) load_exp_table(s_exp);       // read after the barrier below
    for (int e = tid; e < kHdRows * d; e += 256) {
        const int r = e / d, k = e % d;
        const int64_t i = i0 + r;
        s_x[r * XS + k] = i < n ? A.X[i * d + k] : 0.0f;
    }
    __syncthreads();
    if (tid < kHdRows) {
        const int64_t i = i0 + tid;
        double xx = 0.0;
        for (int k = 0; k < d; ++k) {
            const double t = (double)s_x[tid * XS + k];
            xx = fma(t, t, xx);
        }
        s_xx[tid] = xx;
        if (i < n) {
            const double a = MAXOP ? 0.0 : A.a[i];
            const double R = MAXOP ? 0.0 : exp(a);
            s_E[tid] = (A.u[i] - a) - beta * xx;
            if constexpr (MAXOP) {
                s_hx[tid] = 0.0;
                s_w0[tid] = 0.0;
                s_w1[tid] = 0.0;
            } else if constexpr (HVP) {
                const double x = A.xw1[i];
                s_hx[tid] = x;
                s_w0[tid] = R * srho * x;
                s_w1[tid] = R;
            } else {
                s_hx[tid] = 0.0;
                s_w0[tid] = R * (A.xw0 ? A.xw0[i] : 1.0);
                s_w1[tid] = R * (A.xw1 ? A.xw1[i] : 1.0);
            }
        } else {
            s_E[tid] = -INFINITY;
            s_hx[tid] = 0.0;
            s_w0[tid] = 0.0;
            s_w1[tid] = 0.0;
        }
    }
    __syncthreads();

    // the lane's column operand slice (FP32) of step st of block blk
    auto load_cols = [&](int64_t jc, float (&yf)[D4]) {
        int64_t j = jc + jl;
        j = j < m ? j : m - 1;                         // finite filler past m
        const float4* src = reinterpret_cast<const float4*>(A.Y + j * d + g * D4);
#pragma unroll
        for (int q = 0; q < D4 / 4; ++q) {
            const float4 t = src[q];
            yf[4 * q + 0] = t.x;
            yf[4 * q + 1] = t.y;
            yf[4 * q + 2] = t.z;
            yf[4 * q + 3] = t.w;
        }
    };

    double racc[NRA][2][4];
#pragma unroll
    for (int k = 0; k < NRA; ++k)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) racc[k][b][r] = MAXOP ? -INFINITY : 0.0;

    const int64_t cols = m - j0 < A.hd_cols ? m - j0 : A.hd_cols;
    const int nblk = (int)((cols + kF64Blk - 1) / kF64Blk);
    const int ra = wave * 32 + jl;                     // MFMA operand A rows (block 0 / +16)
    float ycur[D4], ynext[D4];
    load_cols(j0, ycur);
    for (int blk = 0; blk < nblk; ++blk) {
        const int p = blk & 1;
        const int64_t jb = j0 + (int64_t)blk * kF64Blk;
#pragma unroll 1
        for (int st = 0; st < kF64Blk / kF64Step; ++st) {
            const int64_t jc = jb + st * kF64Step;
            const bool more = st + 1 < kF64Blk / kF64Step || blk + 1 < nblk;
            if (more) load_cols(jc + kF64Step, ynext);
            // x . y for the two 16-row blocks, and this lane's share of |y_j|^2
            typedef double d4 __attribute__((ext_vector_type(4)));
            d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
            double yy = 0.0;
#pragma unroll
            for (int kk = 0; kk < D4; ++kk) {
                const double b = (double)ycur[kk];
                const double a0 = (double)s_x[ra * XS + g * D4 + kk];
                const double a1 = (double)s_x[(ra + 16) * XS + g * D4 + kk];
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b, acc1, 0, 0, 0);
                yy = fma(b, b, yy);
            }
            yy = quad_total_f64(yy);
            const int64_t j = jc + jl;
            const bool jok = j < m;
            const double F = jok ? A.v[j] - beta * yy : -INFINITY;
            double yw0 = 0.0, yw1 = 0.0;
            if (jok && !MAXOP) {
                if constexpr (HVP) {
                    yw0 = A.yw1[j];
                } else {
                    yw0 = A.yw0 ? A.yw0[j] : 1.0;
                    yw1 = A.yw1 ? A.yw1[j] : 1.0;
                }
            }
            double cacc[NCA];
#pragma unroll
            for (int k = 0; k < NCA; ++k) cacc[k] = 0.0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wave * 32 + 16 * b + 4 * r + g;
                    const double xy = b == 0 ? acc0[r] : acc1[r];
                    if constexpr (MAXOP) {
                        racc[0][b][r] = fmax(racc[0][b][r], fma(2.0 * beta, xy, s_E[row] + F));
                        continue;
                    }
                    const double e = exp_tab256(fma(2.0 * beta, xy, s_E[row] + F), s_exp);
                    if constexpr (HVP) {
                        racc[0][b][r] = fma(e, fma(srho, yw0, s_hx[row]), racc[0][b][r]);
                        cacc[0] = fma(e, fma(s_w1[row], yw0, s_w0[row]), cacc[0]);
                    } else {
                        double cd = 0.0;
                        if constexpr (MODE2 == R2_COST) cd = fmax(s_xx[row] + yy - 2.0 * xy, 0.0);
                        if constexpr (NR >= 1) racc[0][b][r] = fma(e, yw0, racc[0][b][r]);
                        if constexpr (NR >= 2) {
                            double term = e;
                            if constexpr (MODE2 == R2_SQUARE) term = e * e;
                            if constexpr (MODE2 == R2_COST) term = e * cd;
                            racc[NR - 1][b][r] = fma(term, yw1, racc[NR - 1][b][r]);
                        }
                        if constexpr (NC >= 1) cacc[0] = fma(e, s_w0[row], cacc[0]);
                        if constexpr (NC >= 2) {
                            const double term = MODE2 == R2_COST ? e * cd : e;
                            cacc[NC - 1] = fma(term, s_w1[row], cacc[NC - 1]);
                        }
                    }
                }
            }
            if constexpr (NC > 0) {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    const double tot = quad_total_f64(cacc[k]);
                    if (g == 0) s_cp[p][k][wave][st * kF64Step + jl] = tot;
                }
            }
            if (more) {
#pragma unroll
                for (int kk = 0; kk < D4; ++kk) ycur[kk] = ynext[kk];
            }
        }
        __syncthreads();
        if constexpr (NC > 0) {
            if (tid < kF64Blk) {
                const int64_t j = jb + tid;
                if (j < m) {
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        const double t = (s_cp[p][k][0][tid] + s_cp[p][k][1][tid]) +
                                         (s_cp[p][k][2][tid] + s_cp[p][k][3][tid]);
                        if (A.atomic)
                            atomicAdd(&A.col_part[(int64_t)k * m + j], t);
                        else
                            A.col_part[((int64_t)k * A.tiles_n + blockIdx.y) * m + j] = t;
                    }
                }
            }
        }
    }

    // ---- row totals: the 16 lanes of a group g hold the same rows (4 r + g) of each block
    if constexpr (NR > 0) {
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double x = racc[k][b][r];
                    if constexpr (MAXOP) {
                        x = fmax(x, dpp_f64<kDppXor1>(x));
                        x = fmax(x, dpp_f64<kDppXor2>(x));
                        x = fmax(x, dpp_f64<kDppHalfMirror>(x));
                        x = fmax(x, dpp_f64<kDppMirror>(x));
                    } else {
                        x += dpp_f64<kDppXor1>(x);
                        x += dpp_f64<kDppXor2>(x);
                        x += dpp_f64<kDppHalfMirror>(x);
                        x += dpp_f64<kDppMirror>(x);
                    }
                    racc[k][b][r] = x;
                }
        if (jl == 0) {
#pragma unroll
            for (int k = 0; k < NR; ++k)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int64_t i = i0 + wave * 32 + 16 * b + 4 * r + g;
                        if (i < n && MAXOP) {
                            const float xf = (float)racc[k][b][r];
                            if (A.atomic) {
                                if (xf >= 0.0f)
                                    atomicMax(reinterpret_cast<int*>(&out32[i]), __float_as_int(xf));
                                else
                                    atomicMin(reinterpret_cast<unsigned int*>(&out32[i]), __float_as_uint(xf));
                            } else {
                                A.row_part[(int64_t)blockIdx.x * n + i] = (double)xf;
                            }
                        } else if (i < n) {
                            if (A.atomic)
                                atomicAdd(&A.row_part[(int64_t)k * n + i], racc[k][b][r]);
                            else
                                A.row_part[((int64_t)k * A.tiles_m + blockIdx.x) * n + i] = racc[k][b][r];
                        }
                    }
        }
    }
}

template <int NR, int NC, int MODE2>
hipError_t launch_hd(const PassArgs& a, int prec, hipStream_t s)
{
    dim3 grid((unsigned)a.tiles_m, (unsigned)a.tiles_n);
    if constexpr (MODE2 != R2_COST) {
        if (prec == EOT_PREC_MIXED) {
            const int64_t work = a.n > a.m ? a.n : a.m;
            int nb = (int)((work + 255) / 256);
            nb = nb < 1 ? 1 : (nb > kHdMaxPart ? kHdMaxPart : nb);
            hipLaunchKernelGGL(k_hd_grid_max, dim3(nb), dim3(256), 0, s, a);
            const int64_t tw = a.hd_npad > (int64_t)a.tiles_m * a.hd_cols ? a.hd_npad
                                                                          : (int64_t)a.tiles_m * a.hd_cols;
            const unsigned tb = (unsigned)((tw + 255) / 256 < 4096 ? (tw + 255) / 256 : 4096);
            hipLaunchKernelGGL(k_hd_tables, dim3(tb), dim3(256), 0, s, a, nb, MODE2 == R2_HVP ? 1 : 0,
                               NR, NC, MODE2 == R2_SQUARE ? 1 : 0);
            if (hd_padded_dim(a.d) == 32)
                hipLaunchKernelGGL((k_pass_hd_mx16<NR, NC, MODE2, 1>), grid, dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_pass_hd_mx16<NR, NC, MODE2, 2>), grid, dim3(256), 0, s, a);
            return hipGetLastError();
        }
    }
    if (prec == EOT_PREC_MIXED) {
        hipLaunchKernelGGL((k_pass_hd<EOT_PREC_MIXED, NR, NC, MODE2, 0>), grid, dim3(256), 0, s, a,
                           nullptr);
    } else if (reinterpret_cast<uintptr_t>(a.Y) % 16 != 0) {   // the FP64 kernel reads Y as float4
        hipLaunchKernelGGL((k_pass_hd<EOT_PREC_FP64, NR, NC, MODE2, 0>), grid, dim3(256), 0, s, a,
                           nullptr);
    } else {
        switch (a.d) {
        case 16: hipLaunchKernelGGL((k_pass_hd_f64<NR, NC, MODE2, 4>), grid, dim3(256), 0, s, a, nullptr); break;
        case 32: hipLaunchKernelGGL((k_pass_hd_f64<NR, NC, MODE2, 8>), grid, dim3(256), 0, s, a, nullptr); break;
        case 48: hipLaunchKernelGGL((k_pass_hd_f64<NR, NC, MODE2, 12>), grid, dim3(256), 0, s, a, nullptr); break;
        default: hipLaunchKernelGGL((k_pass_hd_f64<NR, NC, MODE2, 16>), grid, dim3(256), 0, s, a, nullptr); break;
        }
    }
    return hipGetLastError();
}

// BF16 hi / lo parts (rows of hd_padded_dim(d), zeros beyond d) and squared norm of
// each of k points (one thread per point)
__global__ void k_hd_prep(const float* __restrict__ P, int64_t k, int d, __bf16* hi, __bf16* lo,
                          float* sq)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int dp = hd_padded_dim(d);
        float s2 = 0.0f;
        for (int t = 0; t < d; ++t) {
            const float v = P[i * d + t];
            const __bf16 h = (__bf16)v;
            hi[i * dp + t] = h;
            lo[i * dp + t] = (__bf16)(v - (float)h);
            s2 = fmaf(v, v, s2);
        }
        for (int t = d; t < dp; ++t) hi[i * dp + t] = lo[i * dp + t] = (__bf16)0.0f;
        sq[i] = s2;
    }
}

__global__ void k_hd_fill_f32(float* x, float v, int64_t k)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

__global__ void k_hd_to_f64(const float* x, double* y, int64_t k)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}

__global__ void k_hd_merge_max(const double* part, int tiles, int64_t n, double* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = part[i];
    for (int t = 1; t < tiles; ++t) r = fmax(r, part[(int64_t)t * n + i]);
    out[i] = r;
}


// Row sums of the point-cloud cotangent G_ij = P_ij (ra_i + cb_j + kappa D_ij),
// D_ij = |x_i - y_j|^2 (cost scale folded into beta and kappa), for d = 16 .. 64,
// in FP64 with the difference form: g0_i += sum_j G_ij and gy_ik += sum_j G_ij
// y_jk over this block's column slice, accumulated atomically. TPR adjacent
// lanes share a row, each owning 16 dimensions (zero beyond d); the partial
// squared distances are summed across them by lane exchanges, so all TPR lanes
// hold the same D_ij and G_ij, and each accumulates its own 16 dimensions.
// Column points are staged in LDS as FP64, 64 at a time, dimension-interleaved
// (dimension 16 q + k at k TPR + q) so that the TPR lanes of a row read
// adjacent words.
template <int TPR>
__global__ __launch_bounds__(256) void k_points_grad_rows_hd(
    const float* __restrict__ Xr, const float* __restrict__ Yc, int d, int64_t n, int64_t m,
    const double* __restrict__ u, const double* __restrict__ v, double beta,
    const double* __restrict__ ra, const double* __restrict__ cb, double kappa, int64_t slice,
    double* g0, double* gy)
{
    constexpr int kCols = 64;
    constexpr int kDim = 16 * TPR;
    __shared__ double s_y[kCols][kDim];
    __shared__ double s_v[kCols], s_b[kCols];
    const int tid = threadIdx.x;
    const int q = tid % TPR;
    const int64_t i = (int64_t)blockIdx.x * (256 / TPR) + tid / TPR;
    const bool ok = i < n;
    double xi[16], accy[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int e = 16 * q + k;
        xi[k] = ok && e < d ? (double)Xr[i * d + e] : 0.0;
        accy[k] = 0.0;
    }
    const double ui = ok ? u[i] : 0.0, ai = ok ? ra[i] : 0.0;
    double acc0 = 0.0;
    const int64_t jb = (int64_t)blockIdx.y * slice;
    const int64_t je = jb + slice < m ? jb + slice : m;
    for (int64_t j0 = jb; j0 < je; j0 += kCols) {
        __syncthreads();
        for (int idx = tid; idx < kCols * kDim; idx += 256) {
            const int c = idx / kDim, e = idx % kDim;
            const int64_t j = j0 + c;
            s_y[c][(e % 16) * TPR + e / 16] = j < je && e < d ? (double)Yc[j * d + e] : 0.0;
        }
        if (tid < kCols) {
            const int64_t j = j0 + tid;
            s_v[tid] = j < je ? v[j] : -INFINITY;
            s_b[tid] = j < je ? cb[j] : 0.0;
        }
        __syncthreads();
        const int cnt = (int)(je - j0 < kCols ? je - j0 : kCols);
        for (int t = 0; t < cnt; ++t) {
            double d2 = 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const double df = xi[k] - s_y[t][k * TPR + q];
                d2 = fma(df, df, d2);
            }
            if constexpr (TPR >= 2) d2 += __shfl_xor(d2, 1);
            if constexpr (TPR >= 4) d2 += __shfl_xor(d2, 2);
            const double P = exp(fma(-beta, d2, ui + s_v[t]));
            const double Gv = P * fma(kappa, d2, ai + s_b[t]);
            acc0 += Gv;
#pragma unroll
            for (int k = 0; k < 16; ++k) accy[k] = fma(Gv, s_y[t][k * TPR + q], accy[k]);
        }
    }
    if (!ok) return;
    if (q == 0) atomicAdd(&g0[i], acc0);
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (16 * q + k < d) atomicAdd(&gy[i * d + 16 * q + k], accy[k]);
}

// out_ik = two_over_s (x_ik g0_i - out_ik) in place, row-major n x d.
__global__ void k_points_grad_finish_hd(const float* X, int64_t n, int d, double two_over_s,
                                        const double* g0, double* out)
{
    const int64_t total = n * d;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x)
        out[idx] = two_over_s * ((double)X[idx] * g0[idx / d] - out[idx]);
}

}  // namespace

bool is_high_d(const PassArgs& a) { return a.kind == EOT_COST_SQEUCLID_POINTS && a.d > 3; }

hipError_t launch_hd_prep(const float* P, int64_t k, int d, void* hi, void* lo, float* sq,
                          hipStream_t s)
{
    const int64_t b = (k + 255) / 256;
    hipLaunchKernelGGL(k_hd_prep, dim3((unsigned)(b < 4096 ? (b < 1 ? 1 : b) : 4096)), dim3(256), 0,
                       s, P, k, d, static_cast<__bf16*>(hi), static_cast<__bf16*>(lo), sq);
    return hipGetLastError();
}

hipError_t launch_pass_hd(const PassArgs& a, int prec, int nr, int nc, int mode2, hipStream_t s)
{
    if (a.d % 16 != 0 || a.d < 16 || a.d > kHdMaxD) return hipErrorInvalidValue;
    if (nr == 1 && nc == 1 && mode2 == R2_HVP) return launch_hd<1, 1, R2_HVP>(a, prec, s);
    if (nr == 1 && nc == 1) return launch_hd<1, 1, R2_WEIGHT>(a, prec, s);
    if (nr == 2 && nc == 1 && mode2 == R2_SQUARE) return launch_hd<2, 1, R2_SQUARE>(a, prec, s);
    if (nr == 2 && nc == 2 && mode2 == R2_WEIGHT) return launch_hd<2, 2, R2_WEIGHT>(a, prec, s);
    if (nr == 2 && nc == 1 && mode2 == R2_COST) return launch_hd<2, 1, R2_COST>(a, prec, s);
    if (nr == 2 && nc == 2 && mode2 == R2_COST) return launch_hd<2, 2, R2_COST>(a, prec, s);
    if (nr == 2 && nc == 0 && mode2 == R2_SQUARE) return launch_hd<2, 0, R2_SQUARE>(a, prec, s);
    if (nr == 2 && nc == 0 && mode2 == R2_COST) return launch_hd<2, 0, R2_COST>(a, prec, s);
    if (nr == 1 && nc == 0) return launch_hd<1, 0, R2_WEIGHT>(a, prec, s);
    if (nr == 0 && nc == 1) return launch_hd<0, 1, R2_WEIGHT>(a, prec, s);
    return hipErrorInvalidValue;
}

hipError_t launch_rowmax_hd(const PassArgs& a, double* part, double* out, hipStream_t s)
{
    if (a.d % 16 != 0 || a.d < 16 || a.d > kHdMaxD) return hipErrorInvalidValue;
    dim3 grid((unsigned)a.tiles_m, (unsigned)a.tiles_n);
    float* out32 = reinterpret_cast<float*>(part);
    const unsigned eb = (unsigned)((a.n + 255) / 256 < 1024 ? (a.n + 255) / 256 : 1024);
    if (a.atomic)
        hipLaunchKernelGGL(k_hd_fill_f32, dim3(eb), dim3(256), 0, s, out32, -INFINITY, a.n);
    if (reinterpret_cast<uintptr_t>(a.Y) % 16 != 0) {   // the matrix-core kernel reads Y as float4
        hipLaunchKernelGGL((k_pass_hd<EOT_PREC_FP64, 1, 0, R2_WEIGHT, 1>), grid, dim3(256), 0, s, a,
                           out32);
    } else {
        switch (a.d) {
        case 16: hipLaunchKernelGGL((k_pass_hd_f64<1, 0, R2_WEIGHT, 4, 1>), grid, dim3(256), 0, s, a, out32); break;
        case 32: hipLaunchKernelGGL((k_pass_hd_f64<1, 0, R2_WEIGHT, 8, 1>), grid, dim3(256), 0, s, a, out32); break;
        case 48: hipLaunchKernelGGL((k_pass_hd_f64<1, 0, R2_WEIGHT, 12, 1>), grid, dim3(256), 0, s, a, out32); break;
        default: hipLaunchKernelGGL((k_pass_hd_f64<1, 0, R2_WEIGHT, 16, 1>), grid, dim3(256), 0, s, a, out32); break;
        }
    }
    if (a.atomic)
        hipLaunchKernelGGL(k_hd_to_f64, dim3(eb), dim3(256), 0, s, out32, out, a.n);
    else
        hipLaunchKernelGGL(k_hd_merge_max, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s,
                           part, a.tiles_m, a.n, out);
    return hipGetLastError();
}

hipError_t launch_points_grad_rows_hd(const float* Xr, const float* Yc, int d, int64_t n,
                                      int64_t m, const double* u, const double* v, double beta,
                                      const double* ra, const double* cb, double kappa, double* g0,
                                      double* gy, hipStream_t s)
{
    if (d < 4 || d > kHdMaxD) return hipErrorInvalidValue;
    const int tpr = d <= 16 ? 1 : d <= 32 ? 2 : 4;
    const int64_t rows = 256 / tpr;
    const int64_t bx = (n + rows - 1) / rows;
    const int64_t col_blocks = (m + 63) / 64;
    int64_t by = (4096 + bx - 1) / bx;                 // aim at >= 4096 workgroups
    by = by < 1 ? 1 : (by > col_blocks ? col_blocks : by);
    const int64_t slice = ((m + by - 1) / by + 63) / 64 * 64;
    by = (m + slice - 1) / slice;
    dim3 grid((unsigned)bx, (unsigned)by);
    if (tpr == 1)
        hipLaunchKernelGGL((k_points_grad_rows_hd<1>), grid, dim3(256), 0, s, Xr, Yc, d, n, m, u, v,
                           beta, ra, cb, kappa, slice, g0, gy);
    else if (tpr == 2)
        hipLaunchKernelGGL((k_points_grad_rows_hd<2>), grid, dim3(256), 0, s, Xr, Yc, d, n, m, u, v,
                           beta, ra, cb, kappa, slice, g0, gy);
    else
        hipLaunchKernelGGL((k_points_grad_rows_hd<4>), grid, dim3(256), 0, s, Xr, Yc, d, n, m, u, v,
                           beta, ra, cb, kappa, slice, g0, gy);
    return hipGetLastError();
}

hipError_t launch_points_grad_finish_hd(const float* X, int64_t n, int d, double two_over_s,
                                        const double* g0, double* out, hipStream_t s)
{
    const int64_t total = n * d;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_points_grad_finish_hd, dim3((unsigned)blocks), dim3(256), 0, s, X, n, d,
                       two_over_s, g0, out);
    return hipGetLastError();
}

}  // namespace eot
