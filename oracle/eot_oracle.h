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
    int64_t passes_newton, passes_linesearch, passes_sinkhorn, passes_projection;
    double final_beta;
    double err_r, err_c;   /* L1 errors vs the unsmoothed marginals at output  */
    double cost;           /* <P, C> at the output potentials                  */
    double dual_value;     /* g(u, v) of eq. opt:sinkhorn-dual, log units      */
    double rho_last;       /* discount returned by the last NewtonSolve        */
    double delta_min_last; /* delta_min of the last projection                 */
} orc_stats;

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
                     double* alpha, double* log_cP_alpha, int32_t* backtracks);
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

/* ---- rounding onto U(r, c) (Altschuler et al. 2017, Alg. 2) ---------------- */
void orc_round(int64_t n, int64_t m, const double* C, double beta,
               const double* u, const double* v, const double* r,
               const double* c, double* Pout);

#ifdef __cplusplus
}
#endif
#endif
