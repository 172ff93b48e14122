/*
 * FP64 CPU oracle for the truncated-Newton entropic-OT method of
 * Kemertas, Farahmand & Jepson, "A Truncated Newton Method for Optimal
 * Transport" (ICLR 2025).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do. It shares no code or headers with the HIP path.
 *
 * Conventions (the paper's notation, Sec. 2):
 *   beta   = inverse temperature (the paper's gamma);
 *   u, v   = dual potentials in log units;
 *   P_ij   = exp(u_i + v_j - beta*C_ij)            (eq. lagrangian-closed-form)
 *   C      = dense row-major n x m FP64 matrix, leading dimension m.
 * All arithmetic is IEEE double, no fast-math, plain loops.
 *
 * Parity status per function is recorded at each definition in
 * eot_oracle.c ("pinned by ..."); every function below is pinned by at
 * least one test in tests/test_oracle_pins.py.
 */
#ifndef EOT_ORACLE_H
#define EOT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 4 };

typedef struct {
    double gamma_init;     /* initial temperature 1/beta_i                      */
    double gamma_final;    /* final temperature 1/beta_f                        */
    double tol;            /* target L1 marginal error vs the given r, c        */
    double p;              /* tolerance exponent of eps_d (Alg. 1), 1.5      */
    double q1;             /* initial decay factor q^(1), 2                     */
    double w_r;            /* row smoothing weight (Sec. 3.4), w_c = 1/2 - w_r  */
    int32_t adaptive_q;    /* AdjustSchedule on (1) or fixed q (0)              */
    int32_t adaptive_rho0; /* App. B warm discount on (1) or rho0 = 0 (0)       */
    int32_t max_cg;        /* CG iterations per linear solve                    */
    int32_t max_levels;    /* discount levels per NewtonSolve call              */
    int32_t max_backtrack; /* halvings per line search                          */
    int32_t max_newton;    /* Newton steps per projection                       */
    int32_t max_sinkhorn;  /* ChiSinkhorn iterations per call                   */
    int32_t max_mdot;      /* temperature steps                                 */
    int32_t projection;    /* Bregman projection step of Alg. 1: 0 TNP (Alg. 4),
                              1 Sinkhorn (the paper's comparison baseline)      */
} orc_opts;

typedef struct {
    int32_t status;
    int32_t mdot_steps, newton_steps, cg_iters, backtracks, sinkhorn_iters, levels;
    int32_t forcing_misses; /* NewtonSolve exits with the forcing test unmet  */
    int32_t linesearch_unresolved; /* line searches ended at a trial whose Armijo
                              test was below the FP64 resolution of the mass  */
    int64_t passes_newton, passes_linesearch, passes_sinkhorn, passes_projection;
    double final_beta;
    double err_r, err_c;   /* L1 errors vs the unsmoothed marginals at output  */
    double cost;           /* <P, C> at the output potentials                  */
    double dual_value;     /* g(u, v) of eq. opt:sinkhorn-dual, log units      */
    double rho_last;       /* discount returned by the last NewtonSolve        */
    double delta_min_last; /* delta_min of the last projection                 */
} orc_stats;

/* Record of what Alg. 1 (MDOT) and Alg. 4 (TruncatedNewtonProject)
 * decided, step by step: test instrumentation, so that the schedule, the
 * tolerances and the forcing terms can be checked against the paper's rules
 * and compared with another implementation. Arrays are caller-owned with the
 * given capacities (any may be NULL); n_steps / n_newton count every step,
 * also those beyond the capacity, which are not stored. */
typedef struct {
    int32_t cap_steps, cap_newton;   /* in                                          */
    int32_t n_steps, n_newton;       /* out                                         */
    /* per MDOT step t = 1, 2, ... */
    double* beta;        /* inverse temperature of the projection                  */
    double* eps_d;       /* eps_d of Alg. 1 (the projection stops at eps_d / 2)    */
    double* start_err;   /* ||r~ - r(P)||_1 after the projection's first column fix */
    double* delta_min;   /* delta_min of the projection (+inf: no Newton step)     */
    double* q;           /* decay factor after AdjustSchedule at the end of step t */
    int32_t* newton;     /* Newton steps of the projection                         */
    int32_t* sweeps;     /* ChiSinkhorn sweeps of the projection                   */
    double* u_proj;      /* [cap_steps][n]: projected u at step t (log units)      */
    double* v_proj;      /* [cap_steps][m]                                         */
    /* per Newton step k = 1, 2, ... over the whole solve */
    int32_t* step_of;    /* MDOT step it belongs to                                */
    double* gnorm;       /* ||grad g||_1 after ChiSinkhorn                         */
    double* eta;         /* forcing term                                           */
    double* cg_tol;      /* L1 residual tolerance of each CG solve                 */
    double* rho0;        /* discount NewtonSolve starts from                       */
    double* rho_out;     /* discount NewtonSolve returns                           */
    int32_t* cg_iters;   /* CG iterations of the NewtonSolve                       */
    int32_t* levels;     /* discount levels solved                                 */
    double* alpha;       /* accepted line-search step                              */
    double* gnorm_next;  /* ||r~ - r(P)||_1 after the row refresh                  */
} orc_trace;

/* The state Alg. 1 carries from one temperature to the next, so a solve can
 * stop after some temperatures and be resumed: the potentials z^(t) that
 * start projection t (after the extrapolation), the last projected z^(t-1),
 * the inverse temperatures beta^(t), beta^(t-1) (0 before the first
 * projection), the decay factor q and the warm discount rho0 for the next
 * NewtonSolve (App. B). u, u_prev: n, v, v_prev: m, log units, caller-owned. */
typedef struct {
    int32_t t;
    double beta, beta_prev, q, rho0;
    double *u, *v, *u_prev, *v_prev;
} orc_state;

/* ---- plan-level definitions (Sec. 2, eqs. lagrangian-closed-form .. hessian) */
void   orc_log_row_marginal(int64_t n, int64_t m, const double* C, double beta,
                            const double* u, const double* v, double* log_rP);
void   orc_log_col_marginal(int64_t n, int64_t m, const double* C, double beta,
                            const double* u, const double* v, double* log_cP);
double orc_mass(int64_t n, int64_t m, const double* C, double beta,
                const double* u, const double* v);
void   orc_row_square_sum(int64_t n, int64_t m, const double* C, double beta,
                          const double* u, const double* v, const double* c,
                          double* s);
double orc_dual(int64_t n, int64_t m, const double* C, double beta,
                const double* u, const double* v, const double* r, const double* c);
double orc_transport_cost(int64_t n, int64_t m, const double* C, double beta,
                          const double* u, const double* v);
void   orc_hvp(int64_t n, int64_t m, const double* C, double beta,
               const double* u, const double* v, double rho,
               const double* x, const double* y, double* Hx, double* Hy);

/* ---- reduced Newton operator and its solvers (Sec. 3.1, Algs. 2) ---------- */
void orc_fr_apply(int64_t n, int64_t m, const double* C, double beta,
                  const double* u, const double* v, const double* rP,
                  const double* c, double rho, const double* p, double* out);
int  orc_pcg(int64_t n, int64_t m, const double* C, double beta,
             const double* u, const double* v, const double* rP, const double* c,
             const double* s, double rho, const double* b, double tol,
             int32_t max_iter, double* d, int32_t* iters);
int  orc_newton_solve(int64_t n, int64_t m, const double* C, double beta,
                      const double* u, const double* v, const double* r,
                      const double* c, const double* log_rP, double eta,
                      double rho0, int32_t max_cg, int32_t max_levels,
                      double* du, double* dv, double* rho_out,
                      int32_t* cg_iters, int32_t* levels, int64_t* passes,
                      int32_t* forcing_miss);

/* ---- projection and annealing (Algs. 3, 4, 1) ----------------------------- */
int  orc_chi_sinkhorn(int64_t n, int64_t m, const double* C, double beta,
                      double* u, double* v, const double* r, const double* c,
                      double* log_rP, double eps_chi, int32_t max_iter,
                      int32_t* iters);
int  orc_line_search(int64_t n, int64_t m, const double* C, double beta,
                     const double* u, const double* v, const double* grad_u,
                     const double* du, const double* dv, int32_t max_backtrack,
                     double* alpha, double* log_cP_alpha, int32_t* backtracks,
                     int32_t* unresolved);
/* Sinkhorn as the projection: alternate row and column fits until the row
 * marginal is within eps in L1 (the column marginal is exact after each
 * sweep), then the closing row fit of Alg. 4. */
int  orc_sinkhorn_project(int64_t n, int64_t m, const double* C, double beta, double* u,
                          double* v, const double* r, const double* c, double eps,
                          const orc_opts* o, orc_stats* st);
int  orc_tnp(int64_t n, int64_t m, const double* C, double beta, double* u,
             double* v, const double* r, const double* c, double eps,
             const orc_opts* o, double* rho0_io, double* delta_min,
             orc_stats* st);
int  orc_solve(int64_t n, int64_t m, const double* C, const double* r,
               const double* c, const orc_opts* o, double* u, double* v,
               orc_stats* st);
/* orc_solve with options: `warm` (0 or 1) starts from the given u, v at the
 * first temperature instead of (log r~, log c~); `resume` (nullable)
 * continues from a saved state (u, v ignored on input); `state_out`
 * (nullable) receives the state at exit (a solve stopped by max_mdot can be
 * resumed from it); `trace` (nullable) records the steps. */
int  orc_solve_ex(int64_t n, int64_t m, const double* C, const double* r,
                  const double* c, const orc_opts* o, int32_t warm,
                  const orc_state* resume, orc_state* state_out, orc_trace* trace,
                  double* u, double* v, orc_stats* st);

/* ---- Alg. 1's scalar rules, exported so tests can pin them on their own */
/* AdjustSchedule (Sec. 3.3): the decay factor after a projection whose
 * smallest Newton decrease ratio was delta_min. */
double orc_adjust_schedule(double q, double delta_min);
/* Warm-start extrapolation of Alg. 1, in place over k entries:
 * z_next = z + (beta_next - beta) / (beta - beta_prev) (z - z_prev),
 * z_prev <- z. */
void orc_extrapolate(int64_t k, double* z, double* z_prev, double beta_prev,
                     double beta, double beta_next);
/* Forcing term of Alg. 4 at ||grad g||_1 = gnorm and tolerance eps. */
double orc_forcing_eta(double gnorm, double eps);

/* ---- rounding onto U(r, c) (Altschuler et al. 2017, Alg. 2) ---------------- */
void orc_round(int64_t n, int64_t m, const double* C, double beta,
               const double* u, const double* v, const double* r,
               const double* c, double* Pout);

#ifdef __cplusplus
}
#endif
#endif
