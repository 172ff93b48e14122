/*
 * FP64 CPU oracle for the truncated-Newton entropic-OT method
 * (Kemertas, Farahmand & Jepson, ICLR 2025).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product library.
 *
 * Plain, slow, readable: every plan entry is recomputed from its definition
 * (eq. lagrangian-closed-form) whenever it is needed, every reduction is a
 * straight loop in IEEE double, and the algorithms take their steps in the
 * order the paper gives them. OpenMP only splits independent rows (or
 * independent column blocks) between threads; each sum is still accumulated
 * sequentially by one thread, so results do not depend on the thread count.
 *
 * Readings of points the paper leaves open are marked "reading:".
 */
#include "eot_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define COL_BLOCK 64

/* log P_ij = u_i + v_j - beta C_ij  (Sec. 2.1, eq. lagrangian-closed-form) */
static inline double logp(int64_t m, const double* C, double beta,
                          const double* u, const double* v, int64_t i, int64_t j)
{
    return u[i] + v[j] - beta * C[i * m + j];
}

static double* dalloc(int64_t k)
{
    double* p = (double*)calloc((size_t)(k > 0 ? k : 1), sizeof(double));
    return p;
}

static double l1norm(int64_t k, const double* x)
{
    double s = 0.0;
    for (int64_t i = 0; i < k; ++i) s += fabs(x[i]);
    return s;
}

static double dot(int64_t k, const double* x, const double* y)
{
    double s = 0.0;
    for (int64_t i = 0; i < k; ++i) s += x[i] * y[i];
    return s;
}

/* ------------------------------------------------------------------------
 * Marginals. LSE_r and LSE_c are defined in Sec. 2 (Notation):
 *   log r(P)_i = u_i + LSE_j(v_j - beta C_ij),  log c(P)_j = v_j + LSE_i(...).
 * Max-shifted log-sum-exp. Pinned by: long-double brute force, the identity
 * sum r(P) = sum c(P) = sum P, closed 2x2 plan, finite differences of g.
 * ---------------------------------------------------------------------- */
void orc_log_row_marginal(int64_t n, int64_t m, const double* C, double beta,
                          const double* u, const double* v, double* log_rP)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double mx = -INFINITY;
        for (int64_t j = 0; j < m; ++j) {
            double x = logp(m, C, beta, u, v, i, j);
            if (x > mx) mx = x;
        }
        double s = 0.0;
        for (int64_t j = 0; j < m; ++j) s += exp(logp(m, C, beta, u, v, i, j) - mx);
        log_rP[i] = mx + log(s);
    }
}

void orc_log_col_marginal(int64_t n, int64_t m, const double* C, double beta,
                          const double* u, const double* v, double* log_cP)
{
    /* Columns are split into blocks; each block sweeps the rows in order. */
#pragma omp parallel for schedule(static)
    for (int64_t j0 = 0; j0 < m; j0 += COL_BLOCK) {
        int64_t j1 = j0 + COL_BLOCK < m ? j0 + COL_BLOCK : m;
        double mx[COL_BLOCK], s[COL_BLOCK];
        for (int64_t j = j0; j < j1; ++j) { mx[j - j0] = -INFINITY; s[j - j0] = 0.0; }
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = j0; j < j1; ++j) {
                double x = logp(m, C, beta, u, v, i, j);
                if (x > mx[j - j0]) mx[j - j0] = x;
            }
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = j0; j < j1; ++j)
                s[j - j0] += exp(logp(m, C, beta, u, v, i, j) - mx[j - j0]);
        for (int64_t j = j0; j < j1; ++j) log_cP[j] = mx[j - j0] + log(s[j - j0]);
    }
}

/* sum_ij P_ij, accumulated row by row. */
double orc_mass(int64_t n, int64_t m, const double* C, double beta,
                const double* u, const double* v)
{
    double* lr = dalloc(n);
    orc_log_row_marginal(n, m, C, beta, u, v, lr);
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += exp(lr[i]);
    free(lr);
    return s;
}

/* s_i = sum_j P_ij^2 / c_j, so that diag F_r(rho) = r(P) - rho s when
 * c(P) = c (App. A, lemma "condo": M_ii = r(P)_i (1 - rho mu_i) with
 * mu_i = (P_rc)_ii). Pinned by: the dense diagonal of F_r at n <= 64. */
void orc_row_square_sum(int64_t n, int64_t m, const double* C, double beta,
                        const double* u, const double* v, const double* c,
                        double* s)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double p = exp(logp(m, C, beta, u, v, i, j));
            acc += p * p / c[j];
        }
        s[i] = acc;
    }
}

/* g(u, v) = sum P - 1 - <u, r> - <v, c>   (eq. opt:sinkhorn-dual).
 * Pinned by: finite differences (its gradient is the marginal residual),
 * strong duality at the solution. */
double orc_dual(int64_t n, int64_t m, const double* C, double beta,
                const double* u, const double* v, const double* r, const double* c)
{
    return orc_mass(n, m, C, beta, u, v) - 1.0 - dot(n, u, r) - dot(m, v, c);
}

/* <P, C>, row by row. */
double orc_transport_cost(int64_t n, int64_t m, const double* C, double beta,
                          const double* u, const double* v)
{
    double tot = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < m; ++j)
            acc += exp(logp(m, C, beta, u, v, i, j)) * C[i * m + j];
        tot += acc;
    }
    return tot;
}

/* Discounted Hessian-vector product (eq. discounted-hessian; rho = 1 gives
 * eq. hessian):  Hx = r(P) x + sqrt(rho) P y,  Hy = sqrt(rho) P^T x + c(P) y.
 * Pinned by: finite differences of the gradient, H (1, -1) = 0 (footnote of
 * eq. hessian), symmetry, the dense matrix at n <= 64. */
void orc_hvp(int64_t n, int64_t m, const double* C, double beta,
             const double* u, const double* v, double rho,
             const double* x, const double* y, double* Hx, double* Hy)
{
    const double sr = sqrt(rho);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double rp = 0.0, py = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double p = exp(logp(m, C, beta, u, v, i, j));
            rp += p;
            py += p * y[j];
        }
        Hx[i] = rp * x[i] + sr * py;
    }
#pragma omp parallel for schedule(static)
    for (int64_t j0 = 0; j0 < m; j0 += COL_BLOCK) {
        int64_t j1 = j0 + COL_BLOCK < m ? j0 + COL_BLOCK : m;
        double cp[COL_BLOCK], ptx[COL_BLOCK];
        for (int64_t j = j0; j < j1; ++j) { cp[j - j0] = 0.0; ptx[j - j0] = 0.0; }
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = j0; j < j1; ++j) {
                double p = exp(logp(m, C, beta, u, v, i, j));
                cp[j - j0] += p;
                ptx[j - j0] += p * x[i];
            }
        for (int64_t j = j0; j < j1; ++j) Hy[j] = sr * ptx[j - j0] + cp[j - j0] * y[j];
    }
}

/* F_r(rho) p = D(r(P)) p - rho P D(c)^-1 P^T p   (eq. matrix-definitions and
 * the proof of lemma "frprops"). Reading: the column marginal in P_c is the
 * target c, which equals c(P) after the column fixes of Alg. 4.
 * Two explicit passes: w = P^T p, then P (w / c). Pinned by: the dense
 * matrix D(r(P)) - rho P D(c)^-1 P^T at n <= 64, its symmetry, and the
 * Bellman form (I - rho P_rc) d = r/r(P) - 1 (eq. bellman2). */
void orc_fr_apply(int64_t n, int64_t m, const double* C, double beta,
                  const double* u, const double* v, const double* rP,
                  const double* c, double rho, const double* p, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = rP[i] * p[i];
    if (rho == 0.0) return;              /* F_r(0) = D(r(P)) */
    double* w = dalloc(m);
#pragma omp parallel for schedule(static)
    for (int64_t j0 = 0; j0 < m; j0 += COL_BLOCK) {
        int64_t j1 = j0 + COL_BLOCK < m ? j0 + COL_BLOCK : m;
        double acc[COL_BLOCK];
        for (int64_t j = j0; j < j1; ++j) acc[j - j0] = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = j0; j < j1; ++j)
                acc[j - j0] += exp(logp(m, C, beta, u, v, i, j)) * p[i];
        for (int64_t j = j0; j < j1; ++j) w[j] = acc[j - j0] / c[j];
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < m; ++j) acc += exp(logp(m, C, beta, u, v, i, j)) * w[j];
        out[i] -= rho * acc;
    }
    free(w);
}

/* Diagonally preconditioned linear CG on F_r(rho) d = b from d = 0
 * (Sec. 3.1 and lemma "cgconv", which fixes the zero start), with the
 * preconditioner M = diag F_r(rho) = r(P) - rho s (lemma "condo").
 * Stops when the L1 norm of the residual b - F_r d is <= tol (Alg. 2's CG
 * asks for ||F_r d + grad||_1 <= (eta/4)||grad||_1 with b = -grad).
 * Reading: the recursively updated residual is the one tested; M_i is
 * clamped below at (1 - rho) r(P)_i, its exact lower bound when c(P) = c.
 * Standard PCG recurrences (Nocedal & Wright, Alg. 5.3).
 * Pinned by: a dense Cholesky solve at n <= 64. Returns ORC_NOT_CONVERGED
 * when max_iter iterations did not reach tol. */
int orc_pcg(int64_t n, int64_t m, const double* C, double beta,
            const double* u, const double* v, const double* rP, const double* c,
            const double* s, double rho, const double* b, double tol,
            int32_t max_iter, double* d, int32_t* iters)
{
    double* res = dalloc(n);
    double* z = dalloc(n);
    double* p = dalloc(n);
    double* q = dalloc(n);
    double* M = dalloc(n);
    for (int64_t i = 0; i < n; ++i) {
        double mi = rP[i] - rho * s[i];
        double lo = (1.0 - rho) * rP[i];
        M[i] = mi > lo ? mi : lo;
        d[i] = 0.0;
        res[i] = b[i];
        z[i] = res[i] / M[i];
        p[i] = z[i];
    }
    double rz = dot(n, res, z);
    int status = ORC_NOT_CONVERGED;
    int32_t k = 0;
    if (l1norm(n, res) <= tol) status = ORC_OK;
    while (status != ORC_OK && k < max_iter) {
        orc_fr_apply(n, m, C, beta, u, v, rP, c, rho, p, q);
        double alpha = rz / dot(n, p, q);
        for (int64_t i = 0; i < n; ++i) {
            d[i] += alpha * p[i];
            res[i] -= alpha * q[i];
        }
        ++k;
        if (l1norm(n, res) <= tol) { status = ORC_OK; break; }
        for (int64_t i = 0; i < n; ++i) z[i] = res[i] / M[i];
        double rz_new = dot(n, res, z);
        double bet = rz_new / rz;
        rz = rz_new;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + bet * p[i];
    }
    *iters = k;
    free(res); free(z); free(p); free(q); free(M);
    return status;
}

/* NewtonSolve (Alg. 2) with the warm discount of App. B.
 *   rho <- rho0;  d <- -D(r(P))^-1 grad_u g
 *   while ||F_r(1) d + grad_u g||_1 > eta ||grad g||_1:
 *       d <- PCG(F_r(rho), -grad_u g, tol = (eta/4) ||grad g||_1)
 *       rho <- 1 - (1 - rho)/4
 * and d_v = -P_c d_u = -(P^T d_u)/c (as in Alg. 4).
 * Readings: ||grad g||_1 = ||r(P) - r||_1 since c(P) = c (Alg. 4's stopping test);
 * rho_out is the value of rho when the loop exits (one update past the last
 * solve). Alg. 2 has no exit other than the forcing test, which in floating
 * point can be unreachable when P_rc is nearly decomposable (lambda_2 within
 * ~1e-13 of 1, see App. C). So rho is not raised past RHO_MAX = 1 - 2^-30
 * (where kappa(F_r) <= 2/(1 - rho) ~ 2e9), and when the test still fails
 * there, or a CG solve hits max_cg, the last converged CG direction (else
 * the rho = 0 direction) is returned with *forcing_miss = 1; the line
 * search then decides the step.
 * F_r(1) d is evaluated explicitly (two passes) at every test.
 * Pinned by: exit forcing inequality, the Newton-residual structure
 * [F_r(1) d + grad; 0] of the proof of theorem "resid", rho sequence
 * 0, 3/4, 15/16, ..., a dense solve of the undiscounted system. */
#define RHO_MAX (1.0 - 9.313225746154785e-10)
int orc_newton_solve(int64_t n, int64_t m, const double* C, double beta,
                     const double* u, const double* v, const double* r,
                     const double* c, const double* log_rP, double eta,
                     double rho0, int32_t max_cg, int32_t max_levels,
                     double* du, double* dv, double* rho_out,
                     int32_t* cg_iters, int32_t* levels, int64_t* passes,
                     int32_t* forcing_miss)
{
    double* rP = dalloc(n);
    double* grad = dalloc(n);
    double* b = dalloc(n);
    double* s = dalloc(n);
    double* e1 = dalloc(n);
    double* dtry = dalloc(n);
    for (int64_t i = 0; i < n; ++i) {
        rP[i] = exp(log_rP[i]);
        grad[i] = rP[i] - r[i];
        b[i] = -grad[i];
        du[i] = -grad[i] / rP[i];
    }
    orc_row_square_sum(n, m, C, beta, u, v, c, s);
    const double gnorm = l1norm(n, grad);
    double rho = rho0;
    int32_t lev = 0, cgk = 0, miss = 0;
    int64_t np = 0;
    for (;;) {
        orc_fr_apply(n, m, C, beta, u, v, rP, c, 1.0, du, e1);
        np += 2;
        for (int64_t i = 0; i < n; ++i) e1[i] += grad[i];
        if (l1norm(n, e1) <= eta * gnorm) break;
        if (lev >= max_levels || rho > RHO_MAX) { miss = 1; break; }
        int32_t it = 0;
        int st = orc_pcg(n, m, C, beta, u, v, rP, c, s, rho, b, 0.25 * eta * gnorm,
                         max_cg, dtry, &it);
        cgk += it;
        if (rho != 0.0) np += 2 * (int64_t)it;
        if (st != ORC_OK) { miss = 1; break; }
        memcpy(du, dtry, (size_t)n * sizeof(double));
        rho = 1.0 - (1.0 - rho) / 4.0;
        ++lev;
    }
    /* d_v = -(P^T d_u) / c */
#pragma omp parallel for schedule(static)
    for (int64_t j0 = 0; j0 < m; j0 += COL_BLOCK) {
        int64_t j1 = j0 + COL_BLOCK < m ? j0 + COL_BLOCK : m;
        double acc[COL_BLOCK];
        for (int64_t j = j0; j < j1; ++j) acc[j - j0] = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = j0; j < j1; ++j)
                acc[j - j0] += exp(logp(m, C, beta, u, v, i, j)) * du[i];
        for (int64_t j = j0; j < j1; ++j) dv[j] = -acc[j - j0] / c[j];
    }
    np += 1;
    *rho_out = rho;
    *cg_iters = cgk;
    *levels = lev;
    *passes = np;
    *forcing_miss = miss;
    free(rP); free(grad); free(b); free(s); free(e1); free(dtry);
    return ORC_OK;
}

/* chi^2(r | r(P)) in the form sum (r - r(P))^2 / r(P), which equals the
 * paper's <r(P), (r/r(P))^2> - 1 (Sec. 2 Notation) whenever sum r(P) = 1
 * (reading: this form avoids the cancellation of the "- 1"). */
static double chi2(int64_t n, const double* r, const double* log_rP)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double rp = exp(log_rP[i]);
        double d = r[i] - rp;
        s += d * d / rp;
    }
    return s;
}

/* ChiSinkhorn (Alg. 3): while chi^2(r | r(P)) > eps_chi, a u-step, a v-fix
 * and a refresh of log r(P). Pinned by: exit condition, c(P) = c after each
 * sweep, the dual objective never increases. */
int orc_chi_sinkhorn(int64_t n, int64_t m, const double* C, double beta,
                     double* u, double* v, const double* r, const double* c,
                     double* log_rP, double eps_chi, int32_t max_iter,
                     int32_t* iters)
{
    double* lc = dalloc(m);
    int32_t k = 0;
    int status = ORC_OK;
    while (chi2(n, r, log_rP) > eps_chi) {
        if (k >= max_iter) { status = ORC_NOT_CONVERGED; break; }
        for (int64_t i = 0; i < n; ++i) u[i] += log(r[i]) - log_rP[i];
        /* v <- log c - LSE_c(u 1^T - beta C): the column LSE with v = 0 */
        double* zero = dalloc(m);
        orc_log_col_marginal(n, m, C, beta, u, zero, lc);
        free(zero);
        for (int64_t j = 0; j < m; ++j) v[j] = log(c[j]) - lc[j];
        orc_log_row_marginal(n, m, C, beta, u, v, log_rP);
        ++k;
    }
    *iters = k;
    free(lc);
    return status;
}

/* Backtracking line search of Alg. 4: alpha = 1, halve until
 *   ||c(P(alpha))||_1 - 1 <= 0.99 alpha <-grad_u g, d_u>
 * (lemma "suffdecr": this is the Armijo condition with c1 = 0.01 when
 * c(P) = c), where log c(P(alpha)) = v + alpha d_v
 * + LSE_c((u + alpha d_u) 1^T - beta C). Returns the accepted trial's
 * log c(P(alpha)). Pinned by: direct evaluation of the Armijo inequality
 * on g.
 * Resolution (a reading; the paper is silent): the mass is a sum of
 * exponentials whose arguments u_i + v_j - beta C_ij carry rounding errors of
 * a few units in the last place of the potentials' magnitudes (for every
 * entry that is not negligible, |beta C_ij| <= |u_i| + |v_j| + 745), so in
 * FP64 mass - 1 is only known to within
 *   tau = 2^-50 mass (max_i(|u_i| + |du_i|) + max_j(|v_j| + |dv_j|) + 745).
 * When the test fails by at most tau (mass - 1 - 0.99 alpha slope <= tau),
 * the inequality cannot be decided and that trial is accepted; *unresolved
 * (nullable) is set to 1. */
int orc_line_search(int64_t n, int64_t m, const double* C, double beta,
                    const double* u, const double* v, const double* grad_u,
                    const double* du, const double* dv, int32_t max_backtrack,
                    double* alpha, double* log_cP_alpha, int32_t* backtracks,
                    int32_t* unresolved)
{
    double slope = 0.0;                      /* <-grad_u g, d_u> */
    for (int64_t i = 0; i < n; ++i) slope -= grad_u[i] * du[i];
    double* ua = dalloc(n);
    double* va = dalloc(m);
    double a = 1.0;
    int32_t k = 0;
    int status = ORC_OK;
    double span = -1.0;                      /* max|u| + max|v| bound, when needed */
    if (unresolved) *unresolved = 0;
    for (;;) {
        for (int64_t i = 0; i < n; ++i) ua[i] = u[i] + a * du[i];
        for (int64_t j = 0; j < m; ++j) va[j] = v[j] + a * dv[j];
        orc_log_col_marginal(n, m, C, beta, ua, va, log_cP_alpha);
        double mass = 0.0;
        for (int64_t j = 0; j < m; ++j) mass += exp(log_cP_alpha[j]);
        if (mass - 1.0 <= 0.99 * a * slope) break;
        if (isfinite(mass)) {
            if (span < 0.0) {
                double mu = 0.0, mv = 0.0;
                for (int64_t i = 0; i < n; ++i) mu = fmax(mu, fabs(u[i]) + fabs(du[i]));
                for (int64_t j = 0; j < m; ++j) mv = fmax(mv, fabs(v[j]) + fabs(dv[j]));
                span = mu + mv + 745.0;
            }
            if (mass - 1.0 - 0.99 * a * slope <= ldexp(mass * span, -50)) {
                if (unresolved) *unresolved = 1;
                break;
            }
        }
        if (k >= max_backtrack) { status = ORC_NOT_CONVERGED; break; }
        a *= 0.5;
        ++k;
    }
    *alpha = a;
    *backtracks = k;
    free(ua); free(va);
    return status;
}

/* Sinkhorn projection (the baseline the paper compares against, used in
 * place of Alg. 4 inside MDOT): column fit, row marginal; then while
 * ||r - r(P)||_1 > eps: row fit u += log r - log r(P), column fit, row
 * marginal; finally the closing row fit of Alg. 4. Pinned by: reaching the same
 * optimum as the TNP projection, c(P) = c after each sweep, the dual never
 * increasing. */
int orc_sinkhorn_project(int64_t n, int64_t m, const double* C, double beta, double* u,
                         double* v, const double* r, const double* c, double eps,
                         const orc_opts* o, orc_stats* st)
{
    double* lr = dalloc(n);
    double* lc = dalloc(m);
    double* zero = dalloc(m);
    int status = ORC_OK;
    orc_log_col_marginal(n, m, C, beta, u, zero, lc);
    for (int64_t j = 0; j < m; ++j) v[j] = log(c[j]) - lc[j];
    orc_log_row_marginal(n, m, C, beta, u, v, lr);
    st->passes_projection += 2;
    int32_t k = 0;
    for (;;) {
        double gn = 0.0;
        for (int64_t i = 0; i < n; ++i) gn += fabs(r[i] - exp(lr[i]));
        if (gn <= eps) break;
        if (k >= o->max_sinkhorn) { status = ORC_NOT_CONVERGED; break; }
        for (int64_t i = 0; i < n; ++i) u[i] += log(r[i]) - lr[i];
        orc_log_col_marginal(n, m, C, beta, u, zero, lc);
        for (int64_t j = 0; j < m; ++j) v[j] = log(c[j]) - lc[j];
        orc_log_row_marginal(n, m, C, beta, u, v, lr);
        st->passes_sinkhorn += 2;
        ++k;
    }
    st->sinkhorn_iters += k;
    for (int64_t i = 0; i < n; ++i) u[i] += log(r[i]) - lr[i];   /* closing row fit */
    free(lr); free(lc); free(zero);
    return status;
}

/* TruncatedNewtonProject (Alg. 4), with eps_chi = eps^(2/5) and
 * eta = max(||grad||_1, 0.8 eps / ||grad||_1).
 * delta_k (eq. delta_k-ratio) compares the norm used to set eta_k (after
 * ChiSinkhorn) with the norm after the row refresh that follows the step (reading).
 * Returns delta_min over the Newton steps (+inf when none ran). */
/* Forcing term of Alg. 4: eta = max(||grad g||_1, 0.8 eps / ||grad g||_1).
 * Pinned by: hand-worked values of the printed rule (tests/golden). */
double orc_forcing_eta(double gnorm, double eps)
{
    double b = 0.8 * eps / gnorm;
    return gnorm > b ? gnorm : b;
}

static int tnp_impl(int64_t n, int64_t m, const double* C, double beta, double* u,
                    double* v, const double* r, const double* c, double eps,
                    const orc_opts* o, double* rho0_io, double* delta_min,
                    orc_stats* st, orc_trace* tr, int32_t step, double* start_err,
                    int32_t* sweeps_out);

int orc_tnp(int64_t n, int64_t m, const double* C, double beta, double* u,
            double* v, const double* r, const double* c, double eps,
            const orc_opts* o, double* rho0_io, double* delta_min,
            orc_stats* st)
{
    double e0 = 0.0;
    int32_t sw = 0;
    return tnp_impl(n, m, C, beta, u, v, r, c, eps, o, rho0_io, delta_min, st, NULL, 0,
                    &e0, &sw);
}

static int tnp_impl(int64_t n, int64_t m, const double* C, double beta, double* u,
                    double* v, const double* r, const double* c, double eps,
                    const orc_opts* o, double* rho0_io, double* delta_min,
                    orc_stats* st, orc_trace* tr, int32_t step, double* start_err,
                    int32_t* sweeps_out)
{
    double* lr = dalloc(n);
    double* lc = dalloc(m);
    double* grad = dalloc(n);
    double* du = dalloc(n);
    double* dv = dalloc(m);
    double* zero = dalloc(m);
    int status = ORC_OK;

    /* column fix: v <- log c - LSE_c(u 1^T - beta C) */
    orc_log_col_marginal(n, m, C, beta, u, zero, lc);
    for (int64_t j = 0; j < m; ++j) v[j] = log(c[j]) - lc[j];
    /* row marginals: log r(P) <- u + LSE_r(1 v^T - beta C) */
    orc_log_row_marginal(n, m, C, beta, u, v, lr);
    st->passes_projection += 2;

    double dmin = INFINITY;
    int32_t k = 0, sweeps = 0;
    for (;;) {
        double gn = 0.0;
        for (int64_t i = 0; i < n; ++i) gn += fabs(r[i] - exp(lr[i]));
        if (k == 0) *start_err = gn;
        if (gn <= eps) break;                                   /* tolerance met */
        if (k >= o->max_newton) { status = ORC_NOT_CONVERGED; break; }
        int32_t sk = 0;                                         /* ChiSinkhorn */
        int s1 = orc_chi_sinkhorn(n, m, C, beta, u, v, r, c, lr, pow(eps, 0.4),
                                  o->max_sinkhorn, &sk);
        st->sinkhorn_iters += sk;
        st->passes_sinkhorn += 2 * (int64_t)sk;
        sweeps += sk;
        if (s1 != ORC_OK) { status = s1; break; }
        double gk = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            grad[i] = exp(lr[i]) - r[i];
            gk += fabs(grad[i]);
        }
        double eta = orc_forcing_eta(gk, eps);                  /* forcing term */
        double rho_out = 0.0;                                   /* Alg. 2, d_v */
        const double rho_in = *rho0_io;
        int32_t cgk = 0, lev = 0, miss = 0;
        int64_t np = 0;
        int s2 = orc_newton_solve(n, m, C, beta, u, v, r, c, lr, eta, *rho0_io,
                                  o->max_cg, o->max_levels, du, dv, &rho_out,
                                  &cgk, &lev, &np, &miss);
        st->forcing_misses += miss;
        st->cg_iters += cgk;
        st->levels += lev;
        st->passes_newton += np;
        st->rho_last = rho_out;
        *rho0_io = o->adaptive_rho0 ? fmax(0.0, 1.0 - 4.0 * (1.0 - rho_out)) : 0.0;
        if (s2 != ORC_OK) { status = s2; break; }
        double alpha = 1.0;                                     /* line search */
        int32_t bt = 0, unres = 0;
        int s3 = orc_line_search(n, m, C, beta, u, v, grad, du, dv,
                                 o->max_backtrack, &alpha, lc, &bt, &unres);
        st->backtracks += bt;
        st->linesearch_unresolved += unres;
        st->passes_linesearch += 1 + bt;
        if (s3 != ORC_OK) { status = s3; break; }
        for (int64_t i = 0; i < n; ++i) u[i] += alpha * du[i];  /* step */
        for (int64_t j = 0; j < m; ++j) v[j] += alpha * dv[j];
        for (int64_t j = 0; j < m; ++j) v[j] += log(c[j]) - lc[j]; /* column fix */
        orc_log_row_marginal(n, m, C, beta, u, v, lr);          /* row refresh */
        st->passes_projection += 1;
        st->newton_steps += 1;
        double gk1 = 0.0;
        for (int64_t i = 0; i < n; ++i) gk1 += fabs(r[i] - exp(lr[i]));
        double dk = (gk - gk1) / ((1.0 - eta) * gk);
        if (dk < dmin) dmin = dk;
        if (tr) {
            const int32_t e = tr->n_newton;
            if (e < tr->cap_newton) {
                if (tr->step_of) tr->step_of[e] = step;
                if (tr->gnorm) tr->gnorm[e] = gk;
                if (tr->eta) tr->eta[e] = eta;
                if (tr->cg_tol) tr->cg_tol[e] = 0.25 * eta * gk;
                if (tr->rho0) tr->rho0[e] = rho_in;
                if (tr->rho_out) tr->rho_out[e] = rho_out;
                if (tr->cg_iters) tr->cg_iters[e] = cgk;
                if (tr->levels) tr->levels[e] = lev;
                if (tr->alpha) tr->alpha[e] = alpha;
                if (tr->gnorm_next) tr->gnorm_next[e] = gk1;
            }
            tr->n_newton = e + 1;
        }
        ++k;
    }
    /* closing row fit: u <- u + log r - log r(P) */
    for (int64_t i = 0; i < n; ++i) u[i] += log(r[i]) - lr[i];
    *delta_min = dmin;
    *sweeps_out = sweeps;
    free(lr); free(lc); free(grad); free(du); free(dv); free(zero);
    return status;
}

static double entropy(int64_t k, const double* x)
{
    double h = 0.0;
    for (int64_t i = 0; i < k; ++i)
        if (x[i] > 0.0) h -= x[i] * log(x[i]);
    return h;
}

/* AdjustSchedule (Sec. 3.3): a projection whose Newton steps all achieved
 * decrease ratios above 0.95 squares the decay factor (capped at 2), one
 * with a ratio below 0.8 takes its square root, otherwise q is kept.
 * Pinned by: hand-worked sequences (tests/golden/alg1_rules.json) and the
 * set {2^(2^-k)} that every reachable q belongs to. */
double orc_adjust_schedule(double q, double delta_min)
{
    if (delta_min > 0.95) return fmin(2.0, q * q);
    if (delta_min < 0.8) return sqrt(q);
    return q;
}

/* Extrapolation of Alg. 1: z^(t+1) = z^(t) + (beta^(t+1) - beta^(t)) /
 * (beta^(t) - beta^(t-1)) (z^(t) - z^(t-1)); z_prev becomes z^(t).
 * Pinned by: exactness on potentials that are affine in beta, and a
 * separable cost with uniform marginals, whose projected potentials are
 * affine in beta, so every extrapolated start is already projected. */
void orc_extrapolate(int64_t k, double* z, double* z_prev, double beta_prev,
                     double beta, double beta_next)
{
    const double ratio = (beta_next - beta) / (beta - beta_prev);
    for (int64_t i = 0; i < k; ++i) {
        double zn = z[i] + ratio * (z[i] - z_prev[i]);
        z_prev[i] = z[i];
        z[i] = zn;
    }
}

/* MDOT (Alg. 1) with AdjustSchedule (Sec. 3.3), asymmetric smoothing
 * (Sec. 3.4) and TruncatedNewtonProject as the Bregman projection.
 *   eps_d = min(H(r), H(c)) / beta^p;   r~ = (1 - w_r eps_d) r + w_r eps_d / n,
 *   c~ likewise with w_c = 1/2 - w_r (and 1/m);
 *   z^(t) <- TNP(z^(t), beta^(t), r~, c~, eps_d / 2);
 *   q <- AdjustSchedule(q, delta_min);  beta^(t+1) = min(q beta^(t), beta_f);
 *   z^(t+1) by the extrapolation above.
 * Readings: at the final temperature eps_d <- min(eps_d, tol/2) so that the
 * error against the unsmoothed marginals ends below tol; the output is the
 * last projected z of Alg. 1 in log units at beta_f; rounding (its last step) is a
 * separate routine (orc_round). A warm start replaces the initial
 * (log r~, log c~) by the given potentials; a resumed solve takes every
 * carried quantity from the saved state.
 * Pinned by: brute-force assignment as the temperature goes to 0, 2x2
 * closed form, separable costs, strong duality, marginal error <= tol; the
 * trace pins of the schedule (fixed q: beta_i q^k capped at beta_f), the
 * smoothing (projected marginals equal r~ and c~ within eps_d / 2 at
 * intermediate temperatures), eps_d, and the warm discounts. */
int orc_solve_ex(int64_t n, int64_t m, const double* C, const double* r,
                 const double* c, const orc_opts* o, int32_t warm,
                 const orc_state* resume, orc_state* state_out, orc_trace* tr,
                 double* u, double* v, orc_stats* st)
{
    memset(st, 0, sizeof(*st));
    if (tr) { tr->n_steps = 0; tr->n_newton = 0; }
    const double beta_f = 1.0 / o->gamma_final;
    const double beta_i = 1.0 / o->gamma_init;
    const double w_c = 0.5 - o->w_r;
    /* min(H(r), H(c)), floored at tol: a point-mass marginal has entropy 0,
     * which would ask for an exact projection (reading) */
    const double hmin = fmax(fmin(entropy(n, r), entropy(m, c)), o->tol);
    double* rt = dalloc(n);
    double* ct = dalloc(m);
    double* zu_prev = dalloc(n);
    double* zv_prev = dalloc(m);
    double beta_prev = 0.0;
    double beta = beta_i < beta_f ? beta_i : beta_f;
    double q = o->q1;
    double rho0 = 0.0;
    int32_t t = 1;
    int fresh = 1;                                                 /* z^(1) still to set */
    if (resume) {
        t = resume->t;
        beta = resume->beta;
        beta_prev = resume->beta_prev;
        q = resume->q;
        rho0 = resume->rho0;
        memcpy(u, resume->u, (size_t)n * sizeof(double));
        memcpy(v, resume->v, (size_t)m * sizeof(double));
        memcpy(zu_prev, resume->u_prev, (size_t)n * sizeof(double));
        memcpy(zv_prev, resume->v_prev, (size_t)m * sizeof(double));
        fresh = 0;
    } else if (warm) {
        memcpy(zu_prev, u, (size_t)n * sizeof(double));
        memcpy(zv_prev, v, (size_t)m * sizeof(double));
        fresh = 0;
    }
    int status = ORC_OK;
    int done = 0;
    while (!done) {
        if (t > o->max_mdot) { status = ORC_NOT_CONVERGED; break; }
        done = (beta == beta_f);                                   /* last temperature */
        double eps_d = hmin / pow(beta, o->p);                     /* projection tolerance */
        if (done && eps_d > 0.5 * o->tol) eps_d = 0.5 * o->tol;
        for (int64_t i = 0; i < n; ++i)                            /* smoothing */
            rt[i] = (1.0 - o->w_r * eps_d) * r[i] + o->w_r * eps_d / (double)n;
        for (int64_t j = 0; j < m; ++j)
            ct[j] = (1.0 - w_c * eps_d) * c[j] + w_c * eps_d / (double)m;
        if (fresh) {                                               /* initial potentials */
            for (int64_t i = 0; i < n; ++i) u[i] = zu_prev[i] = log(rt[i]);
            for (int64_t j = 0; j < m; ++j) v[j] = zv_prev[j] = log(ct[j]);
            fresh = 0;
        }
        double dmin = INFINITY;                                    /* projection */
        double e0 = 0.0;
        int32_t sweeps = 0;
        const int32_t newton0 = st->newton_steps;
        const int32_t sk0 = st->sinkhorn_iters;
        int s = o->projection == 1
                    ? orc_sinkhorn_project(n, m, C, beta, u, v, rt, ct, 0.5 * eps_d, o, st)
                    : tnp_impl(n, m, C, beta, u, v, rt, ct, 0.5 * eps_d, o, &rho0, &dmin, st,
                               tr, t, &e0, &sweeps);
        st->delta_min_last = dmin;
        st->mdot_steps = t;
        st->final_beta = beta;
        if (s == ORC_OK && !done && o->adaptive_q) q = orc_adjust_schedule(q, dmin);
        if (tr) {
            const int32_t e = tr->n_steps;
            if (e < tr->cap_steps) {
                if (tr->beta) tr->beta[e] = beta;
                if (tr->eps_d) tr->eps_d[e] = eps_d;
                if (tr->start_err) tr->start_err[e] = e0;
                if (tr->delta_min) tr->delta_min[e] = dmin;
                if (tr->q) tr->q[e] = q;
                if (tr->newton) tr->newton[e] = st->newton_steps - newton0;
                if (tr->sweeps) tr->sweeps[e] = st->sinkhorn_iters - sk0;
                if (tr->u_proj) memcpy(tr->u_proj + (size_t)e * n, u, (size_t)n * sizeof(double));
                if (tr->v_proj) memcpy(tr->v_proj + (size_t)e * m, v, (size_t)m * sizeof(double));
            }
            tr->n_steps = e + 1;
        }
        if (s != ORC_OK) { status = s; break; }
        if (done) break;
        double beta_next = fmin(q * beta, beta_f);                 /* next temperature */
        orc_extrapolate(n, u, zu_prev, beta_prev, beta, beta_next);
        orc_extrapolate(m, v, zv_prev, beta_prev, beta, beta_next);
        beta_prev = beta;
        beta = beta_next;
        ++t;
    }
    if (state_out) {
        state_out->t = t;
        state_out->beta = beta;
        state_out->beta_prev = beta_prev;
        state_out->q = q;
        state_out->rho0 = rho0;
        if (state_out->u) memcpy(state_out->u, u, (size_t)n * sizeof(double));
        if (state_out->v) memcpy(state_out->v, v, (size_t)m * sizeof(double));
        if (state_out->u_prev) memcpy(state_out->u_prev, zu_prev, (size_t)n * sizeof(double));
        if (state_out->v_prev) memcpy(state_out->v_prev, zv_prev, (size_t)m * sizeof(double));
    }
    /* Report at the output potentials against the unsmoothed marginals. */
    double* lr = dalloc(n);
    double* lc = dalloc(m);
    orc_log_row_marginal(n, m, C, beta, u, v, lr);
    orc_log_col_marginal(n, m, C, beta, u, v, lc);
    st->err_r = 0.0;
    for (int64_t i = 0; i < n; ++i) st->err_r += fabs(exp(lr[i]) - r[i]);
    st->err_c = 0.0;
    for (int64_t j = 0; j < m; ++j) st->err_c += fabs(exp(lc[j]) - c[j]);
    st->cost = orc_transport_cost(n, m, C, beta, u, v);
    st->dual_value = orc_dual(n, m, C, beta, u, v, r, c);
    st->status = status;
    free(lr); free(lc); free(rt); free(ct); free(zu_prev); free(zv_prev);
    return status;
}

int orc_solve(int64_t n, int64_t m, const double* C, const double* r,
              const double* c, const orc_opts* o, double* u, double* v,
              orc_stats* st)
{
    return orc_solve_ex(n, m, C, r, c, o, 0, NULL, NULL, NULL, u, v, st);
}

/* Rounding onto U(r, c) (Altschuler, Weed & Rigollet 2017, Alg. 2; the last
 * step of Alg. 1): scale rows by min(1, r/r(P)), then columns by min(1, c/c(P')), then
 * add err_r err_c^T / ||err_r||_1. Writes the dense n x m plan. */
void orc_round(int64_t n, int64_t m, const double* C, double beta,
               const double* u, const double* v, const double* r,
               const double* c, double* Pout)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j)
            Pout[i * m + j] = exp(logp(m, C, beta, u, v, i, j));
    for (int64_t i = 0; i < n; ++i) {
        double rs = 0.0;
        for (int64_t j = 0; j < m; ++j) rs += Pout[i * m + j];
        double x = rs > 0.0 ? fmin(1.0, r[i] / rs) : 1.0;
        for (int64_t j = 0; j < m; ++j) Pout[i * m + j] *= x;
    }
    for (int64_t j = 0; j < m; ++j) {
        double cs = 0.0;
        for (int64_t i = 0; i < n; ++i) cs += Pout[i * m + j];
        double y = cs > 0.0 ? fmin(1.0, c[j] / cs) : 1.0;
        for (int64_t i = 0; i < n; ++i) Pout[i * m + j] *= y;
    }
    double* er = dalloc(n);
    double* ec = dalloc(m);
    double nr = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double rs = 0.0;
        for (int64_t j = 0; j < m; ++j) rs += Pout[i * m + j];
        er[i] = r[i] - rs;
        nr += fabs(er[i]);
    }
    for (int64_t j = 0; j < m; ++j) {
        double cs = 0.0;
        for (int64_t i = 0; i < n; ++i) cs += Pout[i * m + j];
        ec[j] = c[j] - cs;
    }
    if (nr > 0.0)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < m; ++j) Pout[i * m + j] += er[i] * ec[j] / nr;
    free(er); free(ec);
}
