/*
 * eot.h -- C ABI of the MI355X (gfx950) truncated-Newton entropic-OT library.
 *
 * The method is the one of Kemertas, Farahmand & Jepson, "A Truncated Newton
 * Method for Optimal Transport" (ICLR 2025): MDOT temperature annealing
 * (Alg. 1) around TruncatedNewtonProject (Alg. 4), whose Newton direction
 * comes from NewtonSolve (Alg. 2), a diagonally preconditioned conjugate-
 * gradient solve of the discounted reduced Newton system (Sec. 3.1).
 *
 * Problem statement (Sec. 2.1): cost C (n x m, entries in [0, 1], eq.
 * opt:original-OT-problem), marginals r (n) and c (m) on the simplex, and a
 * temperature gamma > 0. NOTE: the paper's "gamma" is the inverse
 * temperature; here `gamma` is the temperature itself (beta = 1/gamma is the
 * paper's gamma). Potentials at this interface are in cost units:
 *
 *     P_ij = exp((f_i + g_j - C_ij) / gamma)          (eq. lagrangian-closed-form)
 *
 * i.e. f = u / beta, g = v / beta with the paper's log-unit (u, v).
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller (e.g. PyTorch
 *    tensors); the library never allocates or frees them. Struct pointers
 *    marked "host" point to host memory.
 *  - Scratch memory comes from the caller-provided `ws` (device, 256-byte
 *    aligned) of at least the size eot_workspace_size() reports; the library
 *    calls no hipMalloc. The only memory it takes itself is two small pools
 *    of pinned host buffers, one per concurrently running call each, reused
 *    and never freed: 512-byte buffers that receive the scalars a call reads
 *    back, and 64-byte coherent buffers into which the CG kernels store their
 *    progress (iterations done, done flag) for the host to pace its launches.
 *  - `stream` is a hipStream_t (NULL = the default stream). eot_marginals
 *    and eot_hvp are asynchronous on it; eot_newton_cg and eot_solve make
 *    host-side decisions and return after their work on `stream` finished.
 *  - Errors are returned as eot_status; nothing throws across the ABI. On
 *    an error the contents of output arrays are unspecified, except
 *    EOT_ERR_NOT_CONVERGED, which leaves the last iterate in the outputs.
 *  - Vectors are FP64. Dense costs are row-major with leading dimension
 *    ldc >= m (elements).
 *  - Calls on different streams with different workspaces are independent;
 *    the library keeps no global mutable state apart from the opt-in pass
 *    timer (guarded by a mutex), the tile-height override below (an atomic)
 *    and the pinned-buffer pools (guarded by mutexes).
 */
#ifndef EOT_H
#define EOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EOT_OK = 0,
    EOT_ERR_INVALID_ARG = 1,   /* null pointer, n or m < 1, gamma <= 0 or not finite, bad option */
    EOT_ERR_BAD_MARGINALS = 2, /* an entry <= 0 or not finite, or |sum - 1| > 1e-9              */
    EOT_ERR_NONFINITE = 3,     /* a NaN / Inf appeared and the range fallback failed            */
    EOT_ERR_NOT_CONVERGED = 4, /* an iteration cap was hit; outputs hold the last iterate       */
    EOT_ERR_WORKSPACE = 5,     /* ws NULL or smaller than eot_workspace_size() / misaligned     */
    EOT_ERR_UNSUPPORTED = 6,   /* e.g. mixed precision on an FP64 dense cost                    */
    EOT_ERR_HIP = 7            /* a HIP runtime call failed                                     */
} eot_status;

typedef enum {
    EOT_PREC_FP64 = 0,  /* every operation in FP64 (exp included)                          */
    EOT_PREC_MIXED = 1  /* plan entries, exp and cost in FP32 (exponent assembled exactly
                           from FP64 potentials), all sums, CG inner products, residual
                           norms, potentials and the line search in FP64                   */
} eot_precision;

typedef enum {
    EOT_COST_DENSE_F32 = 0,       /* C: float[n * ldc]                                       */
    EOT_COST_DENSE_F64 = 1,       /* C: double[n * ldc]                                      */
    EOT_COST_SQEUCLID_POINTS = 2  /* C_ij = |x_i - y_j|^2 / scale, recomputed on the fly
                                     from X: float[n * d], Y: float[m * d] (Sec. 4.2: the
                                     O(n)-memory variant)                                    */
} eot_cost_kind;

typedef struct {
    int32_t kind;      /* eot_cost_kind                                            */
    int32_t d;         /* point dimension (points only): 2, 3 (vector units) or     */
                       /* 16, 32, 48, 64 (x . y on the matrix cores)               */
    int64_t n;         /* rows    (length of r, f)                                  */
    int64_t m;         /* columns (length of c, g)                                  */
    int64_t ldc;       /* dense: leading dimension in elements, >= m                */
    const void* C;     /* dense: device pointer                                     */
    const float* X;    /* points: device, n x d row-major                           */
    const float* Y;    /* points: device, m x d row-major                           */
    double scale;      /* points: normaliser (> 0), e.g. max_ij |x_i - y_j|^2        */
} eot_cost;

typedef enum {
    EOT_OP_MARGINALS = 0,
    EOT_OP_HVP = 1,
    EOT_OP_NEWTON_CG = 2,
    EOT_OP_SOLVE = 3,
    EOT_OP_GRADIENT = 4,
    EOT_OP_ROUND = 5
} eot_op;

/* Scratch bytes that `op` needs for `cost` in precision `prec`.
 * Returns EOT_ERR_INVALID_ARG for a malformed cost. */
eot_status eot_workspace_size(int32_t op, const eot_cost* cost, int32_t prec, size_t* bytes);

/* Row and column marginals of the plan (Sec. 2 Notation, LSE_r / LSE_c):
 *   log_rP[i] = log sum_j P_ij,  log_cP[j] = log sum_i P_ij,
 *   mass[0]   = sum_ij P_ij                       (device scalar),
 *   s[i]      = sum_j P_ij^2 / c[j]   with c = c_for_s (the diagonal term of
 *               the CG preconditioner diag F_r(rho) = r(P) - rho s, lemma
 *               "condo" in App. A).
 * One streaming pass over C computes all requested outputs.
 * row_shift (nullable): an estimate of log r(P) used only to keep the
 * exponentials in range (any value within ~80 of the truth works in mixed
 * precision, ~700 in FP64); NULL makes the library compute the exact row
 * maximum first (one extra pass).
 * log_rP, log_cP, mass, s are nullable (skip); s needs c_for_s.
 * f: n, g: m, log_rP/s: n, log_cP: m. */
eot_status eot_marginals(const eot_cost* cost, double gamma, const double* f, const double* g,
                         const double* row_shift, double* log_rP, double* log_cP, double* mass,
                         const double* c_for_s, double* s, int32_t prec,
                         void* ws, size_t ws_bytes, void* stream);

/* Discounted Hessian-vector product of the dual g(u, v) (eqs. hessian and
 * discounted-hessian), in the paper's log units, at P(f, g):
 *   Hx = r(P) * x + sqrt(rho) * P y,    Hy = sqrt(rho) * P^T x + c(P) * y.
 * rho in [0, 1]; rho = 1 is the undiscounted Hessian. One pass over C serves
 * both the row (P y, r(P)) and the column (P^T x, c(P)) reductions.
 * x, Hx: n; y, Hy: m. row_shift as for eot_marginals. */
eot_status eot_hvp(const eot_cost* cost, double gamma, const double* f, const double* g,
                   const double* row_shift, double rho, const double* x, const double* y,
                   double* Hx, double* Hy, int32_t prec, void* ws, size_t ws_bytes,
                   void* stream);

/* eot_hvp without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same operation, arguments, kernels and results as
 * eot_hvp; the scratch comes from a library-owned device array of 64 MiB
 * (one copy per GPU, taken when the library's code object is loaded on that
 * GPU and held until the process ends; its address is looked up at the first
 * call on each GPU). The call allocates nothing: no hipMalloc / hipFree, no
 * pinned host memory. It uses the array of the CURRENT device, so `stream`
 * must belong to that device. Every call on one GPU shares that array, which
 * keeps the last call's contents (each call initialises what it reads), so
 * calls that overlap on one GPU (different streams, or host threads) race
 * and must be serialised by the caller. Returns EOT_ERR_WORKSPACE when the
 * problem needs more than 64 MiB of scratch (eot_workspace_size(EOT_OP_HVP)
 * > 64 MiB: a dense n = m = 16384 cost needs 25 MiB, n = m = 32768 needs
 * 98 MiB), before any device work. */
eot_status eot_hvp_noalloc(const eot_cost* cost, double gamma, const double* f, const double* g,
                           const double* row_shift, double rho, const double* x, const double* y,
                           double* Hx, double* Hy, int32_t prec, void* stream);

/* The same discounted Hessian-vector product with the plan's marginals given,
 * as a Newton solver has them at its current iterate (eqs. hessian and
 * discounted-hessian: the diagonal blocks are D(r(P)) and D(c(P))):
 *   Hx = exp(log_rP) * x + sqrt(rho) * P y,    Hy = sqrt(rho) * P^T x + exp(log_cP) * y.
 * The pass then carries one weighted sum per direction instead of two (P y
 * over rows, P^T x over columns), which matters where the pass is bound by
 * arithmetic rather than memory (point clouds). log_rP (n) and log_cP (m) are
 * log r(P) and log c(P) at (f, g), e.g. from eot_marginals; log_rP also serves
 * as the row shift (the same range requirement as row_shift of
 * eot_marginals). Results equal eot_hvp's up to rounding when the marginals
 * are exact; other marginals give the operator with those diagonal blocks.
 * All pointers are device memory, none nullable; x, Hx: n; y, Hy: m.
 * Workspace: eot_workspace_size(EOT_OP_HVP, ...). Returns EOT_ERR_INVALID_ARG
 * for a NULL pointer, gamma <= 0 or rho outside [0, 1]. */
eot_status eot_hvp_with_marginals(const eot_cost* cost, double gamma, const double* f,
                                  const double* g, const double* log_rP, const double* log_cP,
                                  double rho, const double* x, const double* y, double* Hx,
                                  double* Hy, int32_t prec, void* ws, size_t ws_bytes,
                                  void* stream);

typedef struct {
    double rho_out;     /* discount at exit (after the update following the last solve, Alg. 2)          */
    int32_t cg_iters;   /* CG iterations over all discount levels                     */
    int32_t levels;     /* discount levels solved                                     */
    int32_t forcing_miss; /* 1 if the forcing test was unmet at the discount cap      */
    int32_t status;
    int64_t passes;     /* streaming passes over C                                    */
    double forcing_ratio; /* ||F_r(1) d + grad_u g||_1 / ||grad g||_1 at exit         */
} eot_newton_stats;

/* NewtonSolve (Alg. 2) with the warm discount of App. B: diagonally
 * preconditioned CG on F_r(rho) d = -grad_u g from d = 0, stopped at
 * ||F_r(rho) d + grad_u g||_1 <= (eta/4) ||grad g||_1, rho annealed
 * rho <- 1 - (1 - rho)/4 from rho0 until ||F_r(1) d + grad_u g||_1 <=
 * eta ||grad g||_1, then d_v = -P_c d_u (as in Alg. 4). Here
 * F_r(rho) = D(r(P)) - rho P D(c)^-1 P^T (eq. matrix-definitions).
 * Precondition (as in Alg. 4): the columns are fixed, c(P) = c.
 * r: n, c: m (targets); outputs dir_f: n, dir_g: m in cost units
 * (gamma * d_u, gamma * d_v). The discount is capped at 1 - 2^-30; if the
 * forcing test is still unmet there (nearly decomposable P_rc) or a CG solve
 * hits max_cg, the last converged CG direction is returned and
 * stats->forcing_miss = 1. stats: host pointer, nullable. */
eot_status eot_newton_cg(const eot_cost* cost, double gamma, const double* f, const double* g,
                         const double* r, const double* c, double eta, double rho0,
                         int32_t max_cg, int32_t max_levels, double* dir_f, double* dir_g,
                         eot_newton_stats* stats, int32_t prec, void* ws, size_t ws_bytes,
                         void* stream);

typedef enum { EOT_PROJ_TNP = 0, EOT_PROJ_SINKHORN = 1 } eot_projection;

typedef struct {
    double gamma_init;      /* initial temperature (1/beta_i); default 1/32            */
    double gamma_final;     /* final temperature (1/beta_f)                            */
    double tol;             /* target L1 marginal error vs the given r, c; 1e-6        */
    double p;               /* eps_d = min(H(r), H(c)) / beta^p (Alg. 1); 1.5       */
    double q1;              /* initial decay factor q^(1); 2                           */
    double w_r;             /* row smoothing weight (Sec. 3.4), w_c = 1/2 - w_r; 0.45  */
    int32_t adaptive_q;     /* AdjustSchedule (Sec. 3.3) on; 1                         */
    int32_t adaptive_rho0;  /* warm discount of App. B on; 1                           */
    int32_t max_cg;         /* 1000 */
    int32_t max_levels;     /* 30   */
    int32_t max_backtrack;  /* 60   */
    int32_t max_newton;     /* 200  */
    int32_t max_sinkhorn;   /* 10000 */
    int32_t max_mdot;       /* 500  */
    int32_t precision;      /* eot_precision                                           */
    int32_t verify_fp64;    /* mixed: check (and if needed finish) the last projection
                               with FP64 passes so the reported error is exact; 1     */
    int32_t projection;     /* Bregman projection inside MDOT: EOT_PROJ_TNP (Alg. 4, the
                               paper's method) or EOT_PROJ_SINKHORN (alternating row and
                               column fits to the same tolerance: the baseline the paper
                               compares against); EOT_PROJ_TNP                         */
    int32_t cg_graph;       /* 1: each CG solve records one chunk of 8 iterations as a HIP
                               graph and replays it (streams other than the legacy default
                               stream, pass timing off; otherwise direct launches); 0    */
    int32_t verbose;        /* 1: one line on stderr after each MDOT step (temperature,
                               Newton steps, CG iterations, passes, seconds so far); 0  */
    int32_t warm_start;     /* 1: f, g on input are the potentials that start the first
                               projection (Alg. 1's z^(1), converted to log units at
                               gamma_init) instead of (log r~, log c~); 0             */
    int32_t batch_persistent; /* eot_solve_batched: 1 solves every problem it can (dense or
                               d = 2, 3 points, n, m <= 16384, TNP projection, no warm
                               start) in one persistent launch on the device; 0 uses
                               host worker threads for every problem; 1               */
} eot_solve_opts;

typedef struct {
    int32_t status;
    int32_t mdot_steps, newton_steps, cg_iters, backtracks, sinkhorn_iters, levels;
    int32_t forcing_misses, range_retries;
    int32_t mixed_stalls;   /* mixed projections ended at the FP32 error floor (the last
                               one is then finished in FP64 when verify_fp64 is set)   */
    int32_t linesearch_unresolved; /* line searches that took a trial whose Armijo test
                               failed by less than the FP64 resolution of the mass
                               (2^-50 mass (max|u| + |du| + max|v| + |dv| + 745)):
                               the inequality is undecidable there, near the
                               projection's optimum                                    */
    int64_t passes_newton, passes_linesearch, passes_sinkhorn, passes_projection, passes_other;
    double final_gamma;
    double err_r, err_c;    /* L1 marginal errors vs the unsmoothed r, c, FP64 pass     */
    double cost;            /* <P, C> at the output potentials, FP64                    */
    double dual_value;      /* W = gamma (<u, r> + <v, c> - sum P + 1), cost units      */
    double rho_last, delta_min_last;
    double seconds;         /* wall-clock of the solve: the host's, or in the persistent
                               batch the device's from the team's start of the problem
                               to its end                                              */
} eot_solve_stats;

void eot_solve_opts_default(eot_solve_opts* opts);

/* MDOT (Alg. 1) with AdjustSchedule (Sec. 3.3), asymmetric smoothing
 * (Sec. 3.4) and TruncatedNewtonProject (Alg. 4) as the Bregman projection;
 * returns the potentials at gamma_final in cost units (f: n, g: m). The
 * plan at the output is exp((f_i + g_j - C_ij)/gamma_final); rounding onto
 * U(r, c) (the last step of Alg. 1) is not applied. r: n, c: m on the simplex.
 * f, g are also inputs when opts->warm_start is set (cost units at
 * gamma_init). When the solve stops at opts->max_mdot (EOT_ERR_NOT_CONVERGED)
 * f, g hold the extrapolated potentials of the next temperature, in cost
 * units of that temperature (stats->final_gamma).
 * opts, stats: host pointers (stats nullable). */
eot_status eot_solve(const eot_cost* cost, const double* r, const double* c,
                     const eot_solve_opts* opts, double* f, double* g,
                     eot_solve_stats* stats, void* ws, size_t ws_bytes, void* stream);

/* The state Alg. 1 carries from one temperature to the next, so that a solve
 * stopped after some temperatures (opts.max_mdot) can be resumed exactly:
 * z^(t) = (u, v), the potentials that start projection t (already
 * extrapolated), the last projected z^(t-1) = (u_prev, v_prev), the inverse
 * temperatures beta^(t) and beta^(t-1) (0 before the first projection), the
 * decay factor q and the warm discount rho0 of the next NewtonSolve (App. B).
 * Vectors are DEVICE arrays owned by the caller (u, u_prev: n; v, v_prev: m)
 * in the paper's LOG units (u = f / gamma), so that a resumed solve takes
 * bitwise the same steps as an uninterrupted one. */
typedef struct {
    int32_t t;                /* MDOT step that starts next (1-based)                 */
    double beta, beta_prev;   /* beta^(t), beta^(t-1)                                 */
    double q, rho0;
    double* u;
    double* v;
    double* u_prev;
    double* v_prev;
} eot_solve_state;

/* Record of what Algs. 1 and 4 decided, step by step (instrumentation for
 * tests and tuning). Arrays are HOST memory owned by the caller, each nullable,
 * with the capacities given; n_steps and n_newton count every step, also
 * those beyond the capacity, which are not stored. */
typedef struct {
    int32_t cap_steps, cap_newton;  /* in                                            */
    int32_t n_steps, n_newton;      /* out                                           */
    /* per MDOT step t = 1, 2, ... */
    double* beta;        /* inverse temperature of the projection                       */
    double* eps_d;       /* eps_d of Alg. 1 (the projection stops at eps_d / 2)         */
    double* start_err;   /* ||r~ - r(P)||_1 after the projection's first column fix     */
    double* delta_min;   /* smallest Newton decrease ratio (+inf: no Newton step)       */
    double* q;           /* decay factor after AdjustSchedule at the end of the step    */
    int32_t* newton;     /* Newton steps of the step (mixed: with the FP64 finish)      */
    int32_t* sweeps;     /* ChiSinkhorn sweeps of the step                              */
    /* per Newton step over the whole solve */
    int32_t* step_of;    /* MDOT step it belongs to                                     */
    double* gnorm;       /* ||grad g||_1 after ChiSinkhorn                              */
    double* eta;         /* forcing term of Alg. 4                                      */
    double* cg_tol;      /* L1 residual tolerance of its CG solves (eta/4 ||grad g||_1) */
    double* rho0;        /* discount NewtonSolve starts from                            */
    double* rho_out;     /* discount NewtonSolve returns                                */
    int32_t* cg_iters;   /* CG iterations of the NewtonSolve                            */
    int32_t* levels;     /* discount levels solved                                      */
    double* alpha;       /* accepted line-search step                                   */
    double* gnorm_next;  /* ||r~ - r(P)||_1 after the row refresh                       */
} eot_solve_trace;

/* eot_solve with the carried state and the step trace: `resume` (host struct
 * with device vectors, nullable) continues a solve from a saved state (f, g
 * and opts.warm_start are then ignored on input); `state_out` (nullable; its
 * vectors must be allocated by the caller) receives the state at exit, also
 * when the solve stopped at opts.max_mdot with EOT_ERR_NOT_CONVERGED;
 * `trace` (nullable) records the steps. Solving with max_mdot = k and
 * resuming from the saved state with a larger cap gives bitwise the potentials
 * of one uninterrupted solve (same kernels, same order). */
eot_status eot_solve_ex(const eot_cost* cost, const double* r, const double* c,
                        const eot_solve_opts* opts, const eot_solve_state* resume,
                        eot_solve_state* state_out, eot_solve_trace* trace, double* f,
                        double* g, eot_solve_stats* stats, void* ws, size_t ws_bytes,
                        void* stream);

/* Rounding onto the transport polytope U(r, c) (the last step of Alg. 1; the procedure of
 * Altschuler et al. that the paper cites for it): with P the plan at (f, g),
 *   x = min(1, r / r(P)),  y = min(1, c / c(D(x) P)),
 *   X = D(x) P D(y) + er ec^T / |er|_1,  er = r - r(D(x) P D(y)),  ec = c - c(D(x) P D(y)),
 * which has marginals exactly r and c. X is returned implicitly by x (n), y (m),
 * er (n), ec (m) (device, nullable) and, for dense costs, optionally as a dense
 * FP64 n x m matrix `plan` with leading dimension ldp >= m (nullable). `info`
 * (host, required) receives <X, C>, <P, C>, the L1 marginal errors of P, and
 * |er|_1 (the mass moved by the rank-one correction). Every pass is FP64; the
 * correction's cost er^T C ec is one extra pass over C with beta = 0.
 * EOT_ERR_INVALID_ARG for `plan` with a point cloud. */
typedef struct {
    double cost_round;   /* <X, C> */
    double cost_plan;    /* <P, C> */
    double err_r, err_c; /* |r(P) - r|_1, |c(P) - c|_1 */
    double mass_fix;     /* |er|_1 = |ec|_1 */
} eot_round_info;

eot_status eot_round(const eot_cost* cost, double gamma, const double* f, const double* g,
                     const double* r, const double* c, double* x, double* y, double* er,
                     double* ec, double* plan, int64_t ldp, eot_round_info* info, void* ws,
                     size_t ws_bytes, void* stream);

/* Batched solves: many independent problems (any mix of sizes and cost kinds)
 * solved with one shared option set.
 * Persistent path (opts->batch_persistent, default): every problem with a dense
 * cost or d = 2, 3 points and n, m <= 16384 is solved by ONE cooperative kernel
 * launch per cost kind. The grid (the co-resident capacity, at most 1024
 * workgroups) is split into teams of K workgroups (K from the largest n m);
 * each team takes problems from a device queue, largest n m first, and runs
 * the whole solve (Algs. 1-4, the CG iterations, the line search and the FP64
 * report) on the device with team barriers, without host round trips. Same
 * algorithm, decisions and tolerances as eot_solve; the passes are the
 * persistent kernel's own (fixed summation order, reproducible run to run, not
 * bitwise those of eot_solve). Wait bound: a team barrier that waits longer
 * than ~16 s aborts the launch and the affected problems report EOT_ERR_HIP.
 * Host-worker path (the other problems, or all with batch_persistent = 0): a
 * native scheduler runs `workers` host threads, each with its own non-blocking
 * HIP stream (default priority) and its own slice of the workspace; problems
 * are dealt largest n m first to whichever worker is free. Each problem's
 * arithmetic is exactly that of eot_solve on it: bitwise identical results.
 * probs: host array of nprob entries (device pointers inside); stats and
 * status: host arrays of nprob entries (nullable). Work on the caller's stream
 * that precedes the call is waited for; the call returns when every problem
 * is done, and the caller's stream is ordered after all of them. Returns
 * EOT_OK, or the status of the lowest-numbered problem that failed (the
 * others are still solved). ws: eot_workspace_size_batched bytes, 256-byte
 * aligned. */
typedef struct {
    eot_cost cost;
    const double* r;   /* device, n, on the simplex */
    const double* c;   /* device, m, on the simplex */
    double* f;         /* device, n, out (cost units) */
    double* g;         /* device, m, out */
} eot_batch_problem;

eot_status eot_workspace_size_batched(int32_t nprob, const eot_batch_problem* probs,
                                      int32_t workers, size_t* bytes);
eot_status eot_solve_batched(int32_t nprob, const eot_batch_problem* probs,
                             const eot_solve_opts* opts, int32_t workers,
                             eot_solve_stats* stats, int32_t* status, void* ws, size_t ws_bytes,
                             void* stream);

/* Derivatives at potentials (f, g) of the entropic value
 *   W = gamma (<u, r> + <v, c> - sum_ij P_ij + 1)      (u = f / gamma, v = g / gamma;
 *                                                      the negated dual of Sec. 2)
 * and of the sharp transport cost S = <P, C>, combined with the weights w_W and
 * w_S (a vector-Jacobian product; pass the upstream gradients of W and S).
 * With G = w_W dW/dC + w_S dS/dC:
 *   dW/dC = P, dW/dr = f, dW/dc = g               (envelope theorem, at the optimum);
 *   dS/dC_ij = P_ij (1 + (lam_i + mu_j - C_ij) / gamma), dS/dr = lam, dS/dc = mu,
 * where [lam; mu] solves H [lam; mu] = [(P o C) 1; (P o C)^T 1] with H the dual
 * Hessian [[D(r(P)), P], [P^T, D(c(P))]] (Sec. 2; implicit differentiation of
 * r(P) = r, c(P) = c). The system is solved through its row Schur complement
 * F_r(1) lam = (P o C) 1 - P D(c(P))^-1 (P o C)^T 1 by the preconditioned CG of
 * Alg. 2 at rho = 1, then mu = ((P o C)^T 1 - P^T lam) / c(P); skipped when
 * w_S = 0.
 * Outputs (device, all nullable, FP64):
 *   grad_C: dense costs only, n x m row-major with leading dimension ldg >= m,
 *           G itself;
 *   grad_X, grad_Y: point clouds only, n x d and m x d row-major,
 *           (2/s) (x_i sum_j G_ij - sum_j G_ij y_j) and the transpose analogue;
 *   grad_r, grad_c: w_W f + w_S lam and w_W g + w_S mu with their means removed
 *           (r and c live on the simplex; the constant part is not defined).
 * `info` (host, required): in tol (CG stop: L1 residual <= tol * L1 of the
 * right-hand side; FP64 1e-11 reaches ~1e-10 relative accuracy, mixed needs
 * >= 1e-5) and max_cg; out cg_iters, the relative residual reached, and S.
 * prec selects the CG passes' precision; the other passes are FP64.
 * Returns EOT_ERR_NOT_CONVERGED (outputs written) when CG hits max_cg, and
 * EOT_ERR_INVALID_ARG for grad_C with a point cloud or grad_X / grad_Y with a
 * dense cost. Gradient atomics make the point-cloud outputs reproducible to
 * rounding, not bitwise. */
typedef struct {
    double tol;              /* in  */
    int32_t max_cg;          /* in  */
    int32_t cg_iters;        /* out */
    double cg_residual;      /* out */
    double S;                /* out: <P, C> at (f, g) */
} eot_grad_info;

eot_status eot_gradient(const eot_cost* cost, double gamma, const double* f, const double* g,
                        double w_W, double w_S, double* grad_C, int64_t ldg, double* grad_X,
                        double* grad_Y, double* grad_r, double* grad_c, eot_grad_info* info,
                        int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* eot_gradient over a batch of independent problems (the backward of a batch
 * of solves), with one pair of weights (w_W, w_S) and one precision. Each
 * problem's outputs, formulas, validation and info (tol, max_cg in; cg_iters,
 * cg_residual, S out) are those of eot_gradient on it. A native scheduler runs
 * `workers` host threads, each with its own non-blocking HIP stream (default
 * priority) and its own workspace slice, largest n m first; per problem the
 * arithmetic is that of eot_gradient with the single-launch CG switched off
 * (eot_set_cg_persist(0)), so results are bitwise equal to such calls on dense
 * costs and equal to rounding on point clouds (their gradient atomics).
 * probs, info: host arrays of nprob entries (device pointers inside); status:
 * host array of nprob entries (nullable). Work on the caller's stream that
 * precedes the call is waited for; the call returns when every problem is
 * done, with the caller's stream ordered after them. Returns EOT_OK, the first
 * argument error before any device work, or the status of the lowest-numbered
 * problem that failed (the others are still computed). ws:
 * eot_workspace_size_gradient_batched bytes, 256-byte aligned. */
typedef struct {
    eot_cost cost;
    double gamma;        /* temperature of the problem's potentials            */
    const double* f;     /* device, n, in (cost units)                          */
    const double* g;     /* device, m, in                                       */
    double* grad_C;      /* device, dense costs only, n x ldg (nullable)        */
    int64_t ldg;
    double* grad_X;      /* device, point clouds only, n x d (nullable)         */
    double* grad_Y;      /* device, point clouds only, m x d (nullable)         */
    double* grad_r;      /* device, n (nullable)                                */
    double* grad_c;      /* device, m (nullable)                                */
} eot_grad_problem;

eot_status eot_workspace_size_gradient_batched(int32_t nprob, const eot_grad_problem* probs,
                                               int32_t workers, size_t* bytes);
eot_status eot_gradient_batched(int32_t nprob, const eot_grad_problem* probs, double w_W,
                                double w_S, eot_grad_info* info, int32_t prec, int32_t workers,
                                int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Rows per tile of the streaming passes (a power of two in [8, 256]) used by
 * every later call in this process, or 0 to restore the default choice (the
 * measured table compiled into the library, else the smallest halving of 256
 * that launches at least 512 workgroups). For the autotuner and tests; size
 * workspaces after changing it. */
eot_status eot_set_rows_per_tile(int32_t rows);

/* Workgroups per team of the persistent batched solver (a power of two up to
 * 64) used by every later call in this process, or 0 to restore the default
 * choice from the largest problem (16 from n m >= 4M, 8 from 1M, 4 from 256k,
 * 2 from 64k, else 1); and the plan entries per workgroup and pass below
 * which a team splits into sub-teams for a problem (0: the default 2^18).
 * For tuning and tests; size workspaces after changing it. */
eot_status eot_set_team_size(int32_t k, int64_t entries_per_wg);

/* The single-launch CG of small problems (n, m <= 1024 and
 * min(n, m) >= max(n, m) / 8; dense costs and d = 2 points; d = 3 points use
 * the launches per iteration): each CG solve of NewtonSolve (Alg. 2) runs as
 * one cooperative kernel launch whose workgroups exchange parity-tagged
 * values, instead of four launches per iteration. enable: 1 (the default) or
 * 0 for the launches per iteration; grid: workgroups of that launch (0 ...
 * 128; raised to max(n, m) / 8 when smaller and lowered to min(n, m) when
 * larger, 0 = the minimum). Applies to every later call in this process; the
 * batched solvers do not use it. For tuning and tests. */
eot_status eot_set_cg_persist(int32_t enable, int32_t grid);

/* Opt-in timing of the streaming passes (for benchmarks and profiling). While
 * enabled, every streaming-pass kernel the library launches is bracketed by two
 * HIP events recorded on the stream it is launched on. eot_pass_timing(1)
 * enables and clears the record, eot_pass_timing(0) disables and clears it.
 * eot_pass_timing_read waits for the recorded events and returns how many
 * matching pass launches were recorded and their summed device time in
 * milliseconds; a filter argument of -1 matches anything:
 *   nr, nc  = number of row / column sums of the pass (0..2),
 *   prec    = eot_precision of the pass,
 *   fused_hvp = 1 for the one-pass Hessian-vector product, 0 otherwise.
 * Not meant for production runs: it adds two event records per pass. */
eot_status eot_pass_timing(int32_t enable);
eot_status eot_pass_timing_read(int32_t nr, int32_t nc, int32_t prec, int32_t fused_hvp,
                                int64_t* launches, double* milliseconds);

/* Static text for a status code. */
const char* eot_status_string(int32_t status);

/* Library version string, e.g. "0.1.0 gfx950". */
const char* eot_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EOT_H */
