// Internal interface between the ABI/driver (eot_api.hip) and the device
// kernels (eot_kernels.hip). Not installed; not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cmath>

#include "eot.h"

namespace eot {

// Tile geometry of the streaming pass (see eot_kernels.hip).
constexpr int kPassThreads = 256;        // 4 wave64 per workgroup
constexpr int kVec = 4;                  // consecutive columns per thread per row
constexpr int kChunks = 2;               // column chunks of 1024 per tile
constexpr int kTileCols = kPassThreads * kVec * kChunks;   // 2048
constexpr int kTileRows = 256;           // maximum rows per tile (column partials per band);
                                         // a launch uses PassArgs::rb <= kTileRows rows
// Rows per chunk in flight per thread: passes with one kind of sum, and passes
// with both row and column sums (more accumulators). Build-time tunables.
#ifndef EOT_SUB_ROWS
#define EOT_SUB_ROWS 4
#endif
#ifndef EOT_SUB_ROWS_FUSED
#define EOT_SUB_ROWS_FUSED 4
#endif
constexpr int kSubRows = EOT_SUB_ROWS;
constexpr int kSubRowsFused = EOT_SUB_ROWS_FUSED;
// The same for the mixed point-cloud passes (arithmetic-bound; 8 rows per
// sub-band made the single-sum passes a few percent faster, the fused ones
// slower).
#ifndef EOT_PTS_SUB_ROWS
#define EOT_PTS_SUB_ROWS 8
#endif
#ifndef EOT_PTS_SUB_ROWS_FUSED
#define EOT_PTS_SUB_ROWS_FUSED 4
#endif
constexpr int kPtsSubRows = EOT_PTS_SUB_ROWS;
constexpr int kPtsSubRowsFused = EOT_PTS_SUB_ROWS_FUSED;
// Optional occupancy request (waves per SIMD) for the fused passes, build-time.
#if defined(EOT_FUSED_WAVES_PER_EU) && EOT_FUSED_WAVES_PER_EU > 0
#define EOT_FUSED_OCCUPANCY __attribute__((amdgpu_waves_per_eu(EOT_FUSED_WAVES_PER_EU)))
#else
#define EOT_FUSED_OCCUPANCY
#endif
// Optional occupancy target of the mixed high-dimensional pass (waves per SIMD).
#if defined(EOT_HD_WAVES_PER_EU) && EOT_HD_WAVES_PER_EU > 0
#define EOT_HD_OCCUPANCY __attribute__((amdgpu_waves_per_eu(EOT_HD_WAVES_PER_EU)))
#else
#define EOT_HD_OCCUPANCY
#endif
constexpr int kWaves = kPassThreads / 64;
// Row partials are written per wave: [nr][tiles_m * kWaves][n].
inline int row_tiles(int tiles_m) { return tiles_m * kWaves; }
constexpr int kVecThreads = 256;         // O(n) vector kernels
constexpr int kMaxRedBlocks = 1024;      // partial sums per reduction

// Weighting of the second row accumulator.
// R2_HVP: one row and one column sum with the fused Hessian weights
// (x_i + sqrt(rho) y_j) and (sqrt(rho) x_i + y_j); x in xw1, y in yw1.
enum RowMode2 : int { R2_WEIGHT = 0, R2_SQUARE = 1, R2_COST = 2, R2_HVP = 3 };

struct PassArgs {
    int32_t kind;          // eot_cost_kind
    const void* C;
    int64_t n, m, ldc;
    int32_t vec_ok;        // 16-byte aligned rows: vector loads allowed
    const double* u;       // log-unit row potentials
    const double* a;       // row shifts (~log r(P))
    const double* v;       // log-unit column potentials
    double beta;           // inverse temperature
    const double* xw0;     // per-row weights of column sum 0 (nullable = 1)
    const double* xw1;     // per-row weights of column sum 1 (nullable = 1)
    const double* yw0;     // per-column weights of row sum 0 (nullable = 1)
    const double* yw1;     // per-column weights of row sum 1 (nullable = 1)
    double* row_part;      // [nr][tiles_m][n]
    double* col_part;      // [nc][tiles_n][m]
    int32_t tiles_m, tiles_n;
    double hvp_srho;       // sqrt(rho) for R2_HVP
    const int32_t* skip;   // nullable device flag: the whole pass is skipped when set
    const float* X;        // points: n x d
    const float* Y;        // points: m x d
    int32_t d;             // point dimension (2 or 3)
    int32_t rb;            // rows per tile: 8, 16, ..., kTileRows (grid.y = ceil(n / rb))
    // high-dimensional point clouds, mixed precision: BF16 hi / lo parts of X, Y
    // (n x d, m x d) and the squared norms, prepared once per call
    const void* hd_xh;
    const void* hd_xl;
    const void* hd_yh;
    const void* hd_yl;
    const float* hd_xx;
    const float* hd_yy;
    int32_t exact_sums;    // 1: the mixed point-cloud row-sum pass keeps FP64 sums per entry
                           //    (tight CG solves); 0: FP32 over runs of 16 columns
    int32_t atomic;        // 1: row_part = [nr][n], col_part = [nc][m], pre-zeroed, atomically
                           //    accumulated (problems whose per-tile partials would not fit)
    // high-dimensional point clouds: columns per tile, and the per-pass tables of
    // the mixed pass (rows padded to whole tiles: [4][hd_npad] FP32 + [hd_npad]
    // FP64; columns padded to whole tiles: 16-byte records) and its grid maxima
    int32_t hd_cols;
    int64_t hd_npad;
    float* hd_rt;
    double* hd_rf;
    void* hd_ct;
    double* hd_gpart;
};

// High-dimensional point clouds (d = 16 .. 64, x . y on the matrix cores):
// 128-row tiles of 512 .. 2048 columns, one row partial per tile.
constexpr int kHdTileRows = 128;
constexpr int kHdTileCols = 512;
constexpr int kHdTileColsMax = 2048;
constexpr int kHdMaxPart = 1024;         // grid-maximum partials of the mixed pass
// Row stride of the BF16 hi / lo copies of high-dimensional points: d rounded up
// to whole 32-dimension MFMA chunks (zeros beyond d).
__host__ __device__ constexpr int hd_padded_dim(int d) { return (d + 31) / 32 * 32; }

inline int64_t tiles_m_of(int64_t m) { return (m + kTileCols - 1) / kTileCols; }
inline int64_t tiles_n_of(int64_t n, int rb) { return (n + rb - 1) / rb; }

// One streaming pass: nr row sums (0..2), nc column sums (0..2).
hipError_t launch_pass(const PassArgs& a, int prec, int nr, int nc, int mode2, hipStream_t s);
// Opt-in event timing of every launch_pass (see eot_pass_timing in eot.h).
hipError_t set_pass_timing(bool on);
bool pass_timing_on();
hipError_t read_pass_timing(int nr, int nc, int prec, int hvp, int64_t* launches, double* ms);
// Row shifts ~ max_j (u_i + v_j - beta C_ij): out[n].
hipError_t launch_rowmax(const PassArgs& a, double* part, double* out, hipStream_t s);
// High-dimensional point clouds (eot_highd.hip).
bool is_high_d(const PassArgs& a);
hipError_t launch_pass_hd(const PassArgs& a, int prec, int nr, int nc, int mode2, hipStream_t s);
hipError_t launch_rowmax_hd(const PassArgs& a, double* part, double* out, hipStream_t s);
// BF16 hi / lo split of k points of dimension d (hi = bf16(p), lo = bf16(p - hi))
// and their squared norms.
hipError_t launch_hd_prep(const float* P, int64_t k, int d, void* hi, void* lo, float* sq,
                          hipStream_t s);     // hi / lo rows of hd_padded_dim(d), zero-padded

// ---- merges / epilogues (all FP64) ----------------------------------------
// out_k[i] = exp(a_i) * sum_t part[k][t][i]   (nr row sums)
// out1 carries exp(2 a_i) instead when sq1 (sums of squared plan entries)
hipError_t launch_merge_rows(const double* part, int tiles, int64_t n, int nr,
                             const double* a, double* out0, double* out1, int sq1, hipStream_t s);
// out_k[j] = sum_t part[k][t][j]
hipError_t launch_merge_cols(const double* part, int tiles, int64_t m, int nc,
                             double* out0, double* out1, hipStream_t s);

// ---- vector kernels ---------------------------------------------------------
hipError_t launch_scale(const double* x, double alpha, double* y, int64_t k, hipStream_t s);
hipError_t launch_divs(const double* x, double d, double* y, int64_t k, hipStream_t s);
// v = va + log_ct - log colsum (columns whose sum is 0 / not finite keep va, flags[1] = 1)
hipError_t launch_log_ratio_fix(double* v, const double* va, const double* log_ct,
                                const double* colsum, int64_t m, int32_t* flags, hipStream_t s);
hipError_t launch_hvp_finish(const double* row_part, int tiles_m, const double* col_part,
                             int tiles_n, int64_t n, int64_t m, const double* a, double* Hx,
                             double* Hy, hipStream_t s);
// Hx = exp(log_rP) x + srho exp(a) (row sums), Hy = srho (column sums) + exp(log_cP) y
hipError_t launch_hvp_finish_diag(const double* row_part, int tiles_m, const double* col_part,
                                  int tiles_n, int64_t n, int64_t m, const double* a, double srho,
                                  const double* log_rP, const double* log_cP, const double* x,
                                  const double* y, double* Hx, double* Hy, hipStream_t s);
hipError_t launch_log_row_from_sums(const double* part, int tiles, int64_t n, const double* a,
                                    double* log_rP, int32_t* flags, hipStream_t s);
// Block partial sums of an elementwise expression: writes nb partials to red.
enum VecRed : int {
    RED_L1_DIFF_EXP = 0,   // |x_i - exp(y_i)|
    RED_CHI2 = 1,          // (x_i - exp(y_i))^2 / exp(y_i)
    RED_DOT = 2,           // x_i * y_i
    RED_SUM_EXP = 3,       // exp(y_i)
    RED_SUM = 4,           // x_i
    RED_ENTROPY = 5,       // -x_i log x_i
    RED_L1 = 6,            // |x_i|
    RED_BAD = 7,           // 1 if x_i is not finite and positive
    RED_MAXABS2 = 8        // max_i |x_i| + |y_i| (a maximum, not a sum)
};
hipError_t launch_reduce(int op, const double* x, const double* y, int64_t k, double* red,
                         int* nb_out, hipStream_t s);
// FP64 resolution of the line search's mass (Alg. 4's Armijo test on
// ||c(P(alpha))||_1 - 1): the mass sums exponentials whose arguments
// u_i + v_j - beta C_ij carry rounding errors of a few units in the last place
// of the potentials (for every entry that is not negligible,
// |beta C_ij| <= |u_i| + |v_j| + 745), so it is known only to within
// 2^-50 mass (max_i(|u_i| + |du_i|) + max_j(|v_j| + |dv_j|) + 745); span is
// the sum of the two maxima. A test that fails by less cannot be decided in
// FP64, and the trial is taken.
__host__ __device__ inline double armijo_resolution(double mass, double span)
{
    return ldexp(mass * (span + 745.0), -50);
}

// Host-visible scalar: sum of nb partials written to dst[0] (device).
hipError_t launch_finish_sum(const double* red, int nb, double* dst, hipStream_t s);
// The same for RED_MAXABS2: the largest of nb partials.
hipError_t launch_finish_max(const double* red, int nb, double* dst, hipStream_t s);

// Elementwise updates used by the drivers.
hipError_t launch_axpy(double alpha, const double* x, double* y, int64_t k, hipStream_t s);
hipError_t launch_fix_cols(double* v, const double* log_ct, const double* colsum, int64_t m,
                           int32_t* flags, hipStream_t s);            // v += log ct - log colsum
hipError_t launch_add_logdiff(double* x, const double* la, const double* lb, int64_t k,
                              hipStream_t s);                        // x += la - lb
hipError_t launch_log(const double* x, double* y, int64_t k, hipStream_t s);
hipError_t launch_exp(const double* x, double* y, int64_t k, hipStream_t s);
hipError_t launch_recip(const double* x, double* y, int64_t k, hipStream_t s);
hipError_t launch_smooth(const double* x, double w, double k_inv, double* out, double* log_out,
                         int64_t k, hipStream_t s);
hipError_t launch_extrapolate(double* z, double* z_prev, double ratio, int64_t k, hipStream_t s);
hipError_t launch_shifted(const double* base, double alpha, const double* d, double* out,
                          int64_t k, hipStream_t s);                 // out = base + alpha d
hipError_t launch_newton_init(const double* log_rP, const double* r, double* rP, double* grad,
                              double* b, double* d, int64_t n, hipStream_t s);
hipError_t launch_forcing_resid(const double* rP, const double* d, const double* pcptd,
                                const double* grad, double* e, int64_t n, hipStream_t s);
hipError_t launch_div(const double* x, const double* y, double* out, double sign, int64_t k,
                      hipStream_t s);                                // out = sign * x / y
hipError_t launch_copy(const double* x, double* y, int64_t k, hipStream_t s);
hipError_t launch_fill(double* x, double val, int64_t k, hipStream_t s);
// out = alpha x + beta y + c0 (x, y nullable)
hipError_t launch_lincomb(double* out, int64_t k, double alpha, const double* x, double beta,
                          const double* y, double c0, hipStream_t s);

// Rounding onto U(r, c) (the last step of Alg. 1): out = min(1, t / sum) (1 where sum = 0);
// out = t - x o sum (x nullable = 1); dense rounded plan x_i P_ij y_j + er_i ec_j inv_nr.
hipError_t launch_round_scale(const double* t, const double* sum, double* out, int64_t k,
                              hipStream_t s);
hipError_t launch_round_err(const double* t, const double* x, const double* sum, double* out,
                            int64_t k, hipStream_t s);
hipError_t launch_plan_round(const PassArgs& a, const double* x, const double* y, const double* er,
                             const double* ec, double inv_nr, double* out, int64_t ldo,
                             hipStream_t s);

// Gradients. Dense cotangent G_ij = P_ij (ra_i + cb_j + kappa C_ij) into G (ldg).
hipError_t launch_plan_grad(const PassArgs& a, const double* ra, const double* cb, double kappa,
                            double* G, int64_t ldg, hipStream_t s);
// Point clouds: g0_i += sum_j G_ij, gy[k]_i += sum_j G_ij y_jk with D_ij = |x_i - y_j|^2
// (beta and kappa already divided by the cost scale); outputs pre-zeroed.
hipError_t launch_points_grad_rows(const float* Xr, const float* Yc, int d, int64_t n, int64_t m,
                                   const double* u, const double* v, double beta, const double* ra,
                                   const double* cb, double kappa, double* g0, double* gy0,
                                   double* gy1, double* gy2, hipStream_t s);
// out_ik = two_over_s (x_ik g0_i - gy[k]_i), row-major n x d.
hipError_t launch_points_grad_finish(const float* X, int64_t n, int d, double two_over_s,
                                     const double* g0, const double* gy0, const double* gy1,
                                     const double* gy2, double* out, hipStream_t s);
// The same for d = 16 .. 64: gy is row-major n x d (pre-zeroed, like g0), and the
// finish turns it into the gradient in place.
hipError_t launch_points_grad_rows_hd(const float* Xr, const float* Yc, int d, int64_t n,
                                      int64_t m, const double* u, const double* v, double beta,
                                      const double* ra, const double* cb, double kappa, double* g0,
                                      double* gy, hipStream_t s);
hipError_t launch_points_grad_finish_hd(const float* X, int64_t n, int d, double two_over_s,
                                        const double* g0, double* out, hipStream_t s);

// CG building blocks (state lives in device scalars `sc`).
struct CgScalars {
    double rz, pq, alpha, beta, res_l1, rz_new, tol;
    int32_t done;      // set by the iteration that converged / broke down / hit max_iter
    int32_t iters;     // CG iterations performed
    int32_t broke;     // <p, F p> <= 0 or a non-finite step
    int32_t max_iter;
};
// `mirror` (nullable, pinned coherent host memory, two int32): the kernels
// that run the stop test also store {iterations done, done flag} there, so the
// host can watch the loop's progress without synchronising the stream.
hipError_t launch_cg_init(const double* b, const double* rP, const double* s, double rho,
                          double* d, double* res, double* z, double* p, double* M, double* ptd,
                          double* pcptd, int64_t n, int64_t m, double* red, CgScalars* sc,
                          double tol, int32_t max_iter, int32_t* mirror, hipStream_t st);
// after pass A (column sums of P p): w = raw column sums, wc = w / c
hipError_t launch_cg_colstep(const double* part, int tiles, int64_t m, const double* c,
                             double* w, double* wc, const CgScalars* sc, hipStream_t st);
// after pass B (row sums of P wc): t = row sums, q = rP p - rho t; partial <p, q>
hipError_t launch_cg_rowstep(const double* part, int tiles, int64_t n, const double* a,
                             const double* rP, const double* p, double rho, double* t,
                             double* q, double* red, int* nb, const CgScalars* sc,
                             hipStream_t st);
hipError_t launch_cg_update(const double* red_pq, int nb_pq, double* d, double* res, double* z,
                            const double* p, const double* q, const double* M, const double* t,
                            double* pcptd, const double* w, double* ptd, int64_t n, int64_t m,
                            double* red, int* nb, CgScalars* sc, hipStream_t st);
hipError_t launch_cg_direction(const double* red, int nb, const double* z, double* p,
                               int64_t n, CgScalars* sc, int32_t* mirror, hipStream_t st);
// Small problems (n, m <= kCgSmallMax): row step, update, direction and stop
// test of one CG iteration in a single workgroup launch.
constexpr int64_t kCgSmallMax = 8192;
hipError_t launch_cg_small(const double* part, int tiles, int64_t n, int64_t m, const double* a,
                           const double* rP, double* p, double rho, double* t, double* q,
                           double* d, double* res, double* z, const double* M, double* pcptd,
                           const double* w, double* ptd, CgScalars* sc, int32_t* mirror,
                           hipStream_t s);

// ---- batched solves in one persistent launch (eot_team.hip)
constexpr int kTeamThreads = 256;        // threads per workgroup
constexpr int kTeamVecs = 26;            // FP64 row vectors per team (members own row blocks)
constexpr int kTeamColVecs = 12;         // FP64 column vectors, private to each workgroup
constexpr int kTeamPriv = 3;             // FP64 scratch vectors per workgroup
constexpr int kTeamMaxGrid = 1024;       // workgroups per launch at most
constexpr int64_t kTeamMaxDim = 16384;   // n, m of a problem the team solver takes
constexpr int kTeamSyncWords = 160;      // barrier / queue words per team (8 + 2 per sub-team)
constexpr int kTeamMaxK = 64;            // workgroups per team at most
constexpr int64_t kTeamEntriesPerWg = int64_t(1) << 18;   // plan entries per workgroup and pass
                                                         // below which a team splits
struct TeamProblem {
    int32_t kind, d;
    int64_t n, m, ldc;
    const void* C;
    const float* X;
    const float* Y;
    double scale;
    const double* r;
    const double* c;
    double* f;
    double* g;
};
struct TeamLaunch {
    const TeamProblem* probs;   // device table
    const int32_t* order;       // problem indices, largest first (device)
    int32_t nprob;              // entries of order
    int32_t K;                  // workgroups per team
    int32_t nteams;
    eot_solve_stats* out;       // device, indexed like probs
    double* vec;                // [nteams][team_doubles]
    int64_t vstride;            // doubles per vector (>= every n, m; multiple of 64)
    int64_t team_doubles;       // kTeamVecs * vstride + K vstride + 2 K 8, rounded up
    double* priv;               // [grid][kTeamPriv + kTeamColVecs][vstride]
    uint32_t* sync;             // [nteams][kTeamSyncWords], zeroed before the launch
    int32_t* queue;             // next entry of order (zeroed)
    int32_t* abort;             // set when a team wait timed out (zeroed)
    int64_t entries_per_wg;     // sub-team sizing: plan entries per workgroup and pass
    eot_solve_opts opts;
};
inline int64_t team_doubles_of(int64_t vstride, int K)
{
    return ((int64_t)kTeamVecs * vstride + (int64_t)K * vstride + 2 * (int64_t)K * 8 + 63) / 64 *
           64;
}
// kind: 0 dense FP32, 1 dense FP64, 2 / 3 points in R^2 / R^3; grid a multiple of 8 K,
// at most the co-resident capacity (team_max_grid). Cooperative launch.
// One preconditioned CG solve of NewtonSolve (Alg. 2's inner loop) in a single
// cooperative launch, for small problems (n, m <= kCgpMaxDim): the iterations
// run on the device, two exchanges each (the column sums, then the row sums)
// through iteration-tagged values, instead of four launches per iteration. Workgroup g
// owns a block of at most 8 columns in the column-sum pass and of at most 8
// rows in the row-sum pass (so the grid has at least max(n, m) / 8
// workgroups); every workgroup keeps its own copy of the n-side CG vectors and
// updates all of them in the same order, so all take the same decisions.
constexpr int64_t kCgpMaxDim = 1024;
constexpr int kCgpMaxGrid = 128;
struct CgpArgs {
    TeamProblem P;                // cost (kind, d, n, m, ldc, C, X, Y, scale)
    int32_t KIND;                 // 0 dense FP32, 1 dense FP64, 2 points in R^2
    int32_t mixed;
    double beta;                  // inverse temperature (points: not divided by scale)
    const double *u, *a, *v;      // potentials (log units) and the row shift (log r(P))
    const double *c, *rP, *s, *b; // column marginal, r(P), s_i, right-hand side
    double rho, tol;
    int32_t max_cg;
    double *d, *ptd, *pcptd;      // outputs: solution, P^T d (m), P (P^T d / c) (n)
    CgScalars* sc;                // output scalars
    double *wc, *t;               // exchange: (P^T p) / c (m), P ((P^T p) / c) (n), tagged;
                                  // zeroed before the launch
    int32_t* abort;               // set when a wait timed out; zeroed before the launch
};
hipError_t launch_cg_persist(const CgpArgs& A, int grid, hipStream_t s);
hipError_t cg_persist_max_grid(int kind, int mixed, int* grid);

hipError_t launch_team_solve(int kind, const TeamLaunch& L, int grid, hipStream_t s);
hipError_t team_max_grid(int kind, int* blocks_per_cu, int* cus);

}  // namespace eot
