/*
 * oracle.c -- plain FP64 CPU reference of restarted reflected-Halpern PDHG.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code with the GPU
 * library, and the GPU library never calls it.
 *
 * It follows the D-PDLP paper (arXiv 2601.07628) step by step, in plain loops,
 * with no blocking or fusion beyond what the method states:
 *
 *   problem        Sec. 2.1, problem (1): min c^T x, l_c <= A x <= u_c,
 *                  l_v <= x <= u_v, with the dual sets Y_i of Sec. 2.1.
 *   PDHG step      Sec. 2.2 (and Algorithm 1, steps 1-2):
 *                    x+ = proj_X(x - tau (c - A^T y))
 *                    y+ = y - sigma A(2x+ - x) - sigma proj_{-S}(y/sigma - A(2x+ - x))
 *                  with tau = eta/omega, sigma = eta*omega.
 *   Halpern        App. A / App. B.1 (reflected Halpern), read affinely:
 *                    z_{k+1} = (k+1)/(k+2) [(1+gamma) T(z_k) - gamma z_k] + z_0/(k+2)
 *   restarts       App. B.2 (sufficient / necessary / artificial decay of the
 *                  fixed-point residual r(z) = ||z - T(z)||_P, P of App. B),
 *                  r^2 expanded as in App. D.2.1.
 *   primal weight  App. B.3 (PID on log(omega ||dx|| / ||dy||)), App. D.2.2.
 *   KKT            App. B.4 (relative primal / dual residuals and gap).
 *   diagonal QP    Sec. 6: objective c^T x + x^T Q x / 2 with Q diagonal; the
 *                  primal step minimises over the box per column (closed
 *                  form), the KKT adds Q x to the dual residual and
 *                  x^T Q x / 2 to the primal and subtracts it from the dual
 *                  objective (the Wolfe dual of the QP).
 *
 * Steps the paper leaves open, and the readings taken here:
 *   - Lagrangian sign: L(x,y) = c^T x - y^T A x - p(-y; l_c, u_c).  This is the
 *     sign under which the primal step above, the dual constraint
 *     c - A^T y = r (App. B.4) and the +A blocks of P agree.
 *   - The dual step is evaluated as  sigma * (w - clamp(w, -u_c, -l_c)),
 *     w = y/sigma - A xbar, which equals the Sec. 2.2 formula and keeps the
 *     result exactly inside Y.
 *   - Halpern index k counts iterations inside the current restart epoch, and
 *     z_0 is the epoch's anchor.  Restarts move to T(z_k) = (xhat, yhat).
 *   - r(z^{n,0}) is measured on the first iteration of each epoch; the
 *     "previous" residual of the necessary-decay test is the one at the
 *     previous check of the same epoch; T in the artificial test is the total
 *     iteration count.
 *   - Rescaling (Ruiz infinity-norm passes, then Pock-Chambolle), the power
 *     iteration for eta and the initial primal weight are not in the paper;
 *     they follow common PDLP-family practice and are parameters.
 *   - KKT is evaluated on the original (unscaled) problem at (xhat, yhat),
 *     with s computed from the scaled primal step and mapped back.
 *   - ||[l_c, u_c]||_2 uses the finite entries only.
 *
 * Parallelism: OpenMP over independent rows / columns only.  Every row or
 * column sum runs sequentially in stored order and every global sum is a
 * sequential loop, so results do not depend on the thread count.
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t m, n;
    const int32_t *row_ptr, *col_idx;
    const double *val;
    const double *c, *con_lo, *con_hi, *var_lo, *var_hi;
} ora_lp;

typedef struct {
    double eps;
    int64_t max_iters;
    int32_t check_period;
    int32_t ruiz_iters;
    double gamma, beta_suf, beta_nec, beta_art;
    double kp, ki, kd;
    double eta, omega0, eta_safety;
    int32_t power_max_iters;
    int32_t use_pc;
    double power_tol, pc_alpha;
} ora_params;

/* Scalars of the iteration state (the vectors live in caller arrays). */
typedef struct {
    double omega;
    double r0, r_prev;
    double pid_int, pid_prev;
    int64_t k, t;
    int32_t pid_started, restarts;
    int32_t status;                 /* 0 running, 1 converged, 2 iteration limit */
    int32_t n_checks;
    double r_primal, r_dual, r_gap, obj_p, obj_d, kkt_r;
} ora_state;

/* One record per check. */
typedef struct {
    int64_t t, k;
    double r, r0, r_primal, r_dual, r_gap, omega;
    int32_t restart;                /* 0 none, 1 sufficient, 2 necessary, 3 artificial */
    int32_t pad;
} ora_log;

typedef struct {
    int32_t m, n;
    int64_t nnz;
    int32_t *rp, *ci;  double *v;    /* scaled A, CSR */
    int32_t *cp, *ri;  double *vt;   /* scaled A, CSC */
    double *c, *clo, *chi, *vlo, *vhi;          /* scaled problem data   */
    double *c0, *clo0, *chi0, *vlo0, *vhi0;     /* original problem data */
    double *dr, *dc;                            /* D_r, D_c              */
    double c_norm, b_norm;          /* original ||c||, ||finite [l_c,u_c]|| */
    double c_norm_s, b_norm_s;      /* the same on the scaled problem       */
    double sigma_max, eta, omega0;
    int32_t power_iters;
    double *q;                      /* scaled diagonal of Q (NULL: an LP)    */
} ora_prob;

static double clampd(double v, double lo, double hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/* ---- A0: CSR -> CSC by counting, prefix sum and a stable scatter ------- */
void ora_csr_to_csc(int32_t m, int32_t n, const int32_t *rp, const int32_t *ci,
                    const double *v, int32_t *cp, int32_t *ri, double *vt)
{
    int64_t nnz = rp[m];
    int64_t *next = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t p = 0; p < nnz; ++p) next[ci[p] + 1]++;
    for (int32_t j = 0; j < n; ++j) next[j + 1] += next[j];
    for (int32_t j = 0; j <= n; ++j) cp[j] = (int32_t)next[j];
    for (int32_t i = 0; i < m; ++i)          /* rows in order: stable */
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
            int64_t q = next[ci[p]]++;
            ri[q] = i;
            vt[q] = v[p];
        }
    free(next);
}

/* ---- plain products ------------------------------------------------------ */
static void spmv_csr(const ora_prob *P, const double *x, double *out)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < P->m; ++i) {
        double s = 0.0;
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) s += P->v[p] * x[P->ci[p]];
        out[i] = s;
    }
}

static void spmv_csc(const ora_prob *P, const double *y, double *out)
{
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < P->n; ++j) {
        double s = 0.0;
        for (int64_t p = P->cp[j]; p < P->cp[j + 1]; ++p) s += P->vt[p] * y[P->ri[p]];
        out[j] = s;
    }
}

static double dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double finite_norm2(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (isfinite(a[i])) s += a[i] * a[i];
        if (isfinite(b[i])) s += b[i] * b[i];
    }
    return sqrt(s);
}

/* ---- A3: rescaling ---------------------------------------------------------
 * Multiply row i by fr[i] and column j by fc[j] in both copies of A, in the
 * order (a * fr[i]) * fc[j], and fold the factors into D_r, D_c.          */
static void apply_scale(ora_prob *P, const double *fr, const double *fc)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < P->m; ++i)
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p)
            P->v[p] = P->v[p] * fr[i] * fc[P->ci[p]];
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < P->n; ++j)
        for (int64_t p = P->cp[j]; p < P->cp[j + 1]; ++p)
            P->vt[p] = P->vt[p] * fr[P->ri[p]] * fc[j];
    for (int32_t i = 0; i < P->m; ++i) P->dr[i] *= fr[i];
    for (int32_t j = 0; j < P->n; ++j) P->dc[j] *= fc[j];
}

/* Ruiz pass: factor 1/sqrt(max |a|) per row and per column (1 if empty). */
static void ruiz_pass(ora_prob *P, double *fr, double *fc)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < P->m; ++i) {
        double mx = 0.0;
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) mx = fmax(mx, fabs(P->v[p]));
        fr[i] = mx > 0.0 ? 1.0 / sqrt(mx) : 1.0;
    }
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < P->n; ++j) {
        double mx = 0.0;
        for (int64_t p = P->cp[j]; p < P->cp[j + 1]; ++p) mx = fmax(mx, fabs(P->vt[p]));
        fc[j] = mx > 0.0 ? 1.0 / sqrt(mx) : 1.0;
    }
    apply_scale(P, fr, fc);
}

/* Pock-Chambolle pass: rows 1/sqrt(sum |a|^(2-alpha)), columns
 * 1/sqrt(sum |a|^alpha) (1 if empty). alpha = 1 uses |a| for both.         */
static void pc_pass(ora_prob *P, double alpha, double *fr, double *fc)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < P->m; ++i) {
        double s = 0.0;
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p)
            s += alpha == 1.0 ? fabs(P->v[p]) : pow(fabs(P->v[p]), 2.0 - alpha);
        fr[i] = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
    }
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < P->n; ++j) {
        double s = 0.0;
        for (int64_t p = P->cp[j]; p < P->cp[j + 1]; ++p)
            s += alpha == 1.0 ? fabs(P->vt[p]) : pow(fabs(P->vt[p]), alpha);
        fc[j] = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
    }
    apply_scale(P, fr, fc);
}

/* ---- A4: power iteration on A^T A (scaled A) -> sigma_max --------------- */
static double power_sigma_max(const ora_prob *P, int32_t max_iters, double tol,
                              int32_t *iters_out)
{
    int32_t m = P->m, n = P->n;
    double *v = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *u = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t j = 0; j < n; ++j) v[j] = 1.0 / sqrt((double)n);
    double sig = 0.0, prev = 0.0;
    int32_t it = 0;
    for (it = 1; it <= max_iters; ++it) {
        spmv_csr(P, v, u);
        spmv_csc(P, u, w);
        double lam = sqrt(dot(w, w, n));       /* ||A^T A v||, ||v|| = 1 */
        sig = sqrt(lam);
        if (lam == 0.0) break;
        for (int32_t j = 0; j < n; ++j) v[j] = w[j] / lam;
        if (it > 1 && fabs(sig - prev) <= tol * sig) break;
        prev = sig;
    }
    if (it > max_iters) it = max_iters;
    free(v); free(u); free(w);
    if (iters_out) *iters_out = it;
    return sig;
}

/* ---- setup: copy, CSC, scaling, eta, omega0 ----------------------------- */
int ora_prepare(const ora_lp *lp, const ora_params *prm, ora_prob **out)
{
    ora_prob *P = (ora_prob *)calloc(1, sizeof(ora_prob));
    int32_t m = lp->m, n = lp->n;
    int64_t nnz = lp->row_ptr[m];
    P->m = m; P->n = n; P->nnz = nnz;
    size_t mz = (size_t)(m > 0 ? m : 1), nz = (size_t)(n > 0 ? n : 1);
    size_t kz = (size_t)(nnz > 0 ? nnz : 1);
    P->rp = (int32_t *)malloc(sizeof(int32_t) * (mz + 1));
    P->ci = (int32_t *)malloc(sizeof(int32_t) * kz);
    P->v = (double *)malloc(sizeof(double) * kz);
    P->cp = (int32_t *)malloc(sizeof(int32_t) * (nz + 1));
    P->ri = (int32_t *)malloc(sizeof(int32_t) * kz);
    P->vt = (double *)malloc(sizeof(double) * kz);
    memcpy(P->rp, lp->row_ptr, sizeof(int32_t) * ((size_t)m + 1));
    memcpy(P->ci, lp->col_idx, sizeof(int32_t) * (size_t)nnz);
    memcpy(P->v, lp->val, sizeof(double) * (size_t)nnz);
    ora_csr_to_csc(m, n, P->rp, P->ci, P->v, P->cp, P->ri, P->vt);

    double **mv[] = {&P->clo, &P->chi, &P->clo0, &P->chi0, &P->dr};
    for (int q = 0; q < 5; ++q) *mv[q] = (double *)malloc(sizeof(double) * mz);
    double **nv[] = {&P->c, &P->vlo, &P->vhi, &P->c0, &P->vlo0, &P->vhi0, &P->dc};
    for (int q = 0; q < 7; ++q) *nv[q] = (double *)malloc(sizeof(double) * nz);
    memcpy(P->c0, lp->c, sizeof(double) * (size_t)n);
    memcpy(P->vlo0, lp->var_lo, sizeof(double) * (size_t)n);
    memcpy(P->vhi0, lp->var_hi, sizeof(double) * (size_t)n);
    memcpy(P->clo0, lp->con_lo, sizeof(double) * (size_t)m);
    memcpy(P->chi0, lp->con_hi, sizeof(double) * (size_t)m);
    for (int32_t i = 0; i < m; ++i) P->dr[i] = 1.0;
    for (int32_t j = 0; j < n; ++j) P->dc[j] = 1.0;

    double *fr = (double *)malloc(sizeof(double) * mz);
    double *fc = (double *)malloc(sizeof(double) * nz);
    for (int32_t it = 0; it < prm->ruiz_iters; ++it) ruiz_pass(P, fr, fc);
    if (prm->use_pc) pc_pass(P, prm->pc_alpha, fr, fc);
    free(fr); free(fc);

    /* scaled data: c~ = D_c c, bounds of A x scale by D_r, bounds of x by 1/D_c */
    for (int32_t j = 0; j < n; ++j) {
        P->c[j] = P->dc[j] * P->c0[j];
        P->vlo[j] = P->vlo0[j] / P->dc[j];
        P->vhi[j] = P->vhi0[j] / P->dc[j];
    }
    for (int32_t i = 0; i < m; ++i) {
        P->clo[i] = P->dr[i] * P->clo0[i];
        P->chi[i] = P->dr[i] * P->chi0[i];
    }
    P->c_norm = sqrt(dot(P->c0, P->c0, n));
    P->b_norm = finite_norm2(P->clo0, P->chi0, m);
    P->c_norm_s = sqrt(dot(P->c, P->c, n));
    P->b_norm_s = finite_norm2(P->clo, P->chi, m);

    if (prm->eta > 0.0) {
        P->eta = prm->eta;
        P->sigma_max = 0.0;
        P->power_iters = 0;
    } else {
        P->sigma_max = power_sigma_max(P, prm->power_max_iters, prm->power_tol,
                                       &P->power_iters);
        P->eta = P->sigma_max > 0.0 ? prm->eta_safety / P->sigma_max : 1.0;
    }
    if (prm->omega0 > 0.0)
        P->omega0 = prm->omega0;
    else if (P->c_norm_s > 1e-10 && P->b_norm_s > 1e-10)
        P->omega0 = P->c_norm_s / P->b_norm_s;
    else
        P->omega0 = 1.0;
    *out = P;
    return 0;
}

void ora_free(ora_prob *P)
{
    if (!P) return;
    void *ptrs[] = {P->rp, P->ci, P->v, P->cp, P->ri, P->vt, P->c, P->clo, P->chi,
                    P->vlo, P->vhi, P->c0, P->clo0, P->chi0, P->vlo0, P->vhi0,
                    P->dr, P->dc, P->q};
    for (size_t q = 0; q < sizeof(ptrs) / sizeof(ptrs[0]); ++q) free(ptrs[q]);
    free(P);
}

/* Accessors for the prepared (scaled) problem. */
void ora_info(const ora_prob *P, double *out6, int32_t *iout2)
{
    out6[0] = P->eta; out6[1] = P->omega0; out6[2] = P->sigma_max;
    out6[3] = P->c_norm; out6[4] = P->b_norm; out6[5] = 0.0;
    iout2[0] = P->power_iters; iout2[1] = 0;
}

void ora_get_scaled(const ora_prob *P, double *v, double *vt, double *dr, double *dc,
                    double *c, double *clo, double *chi, double *vlo, double *vhi)
{
    if (v) memcpy(v, P->v, sizeof(double) * (size_t)P->nnz);
    if (vt) memcpy(vt, P->vt, sizeof(double) * (size_t)P->nnz);
    if (dr) memcpy(dr, P->dr, sizeof(double) * (size_t)P->m);
    if (dc) memcpy(dc, P->dc, sizeof(double) * (size_t)P->n);
    if (c) memcpy(c, P->c, sizeof(double) * (size_t)P->n);
    if (clo) memcpy(clo, P->clo, sizeof(double) * (size_t)P->m);
    if (chi) memcpy(chi, P->chi, sizeof(double) * (size_t)P->m);
    if (vlo) memcpy(vlo, P->vlo, sizeof(double) * (size_t)P->n);
    if (vhi) memcpy(vhi, P->vhi, sizeof(double) * (size_t)P->n);
}

/* Diagonal quadratic objective (Sec. 6): q[n] >= 0 in original columns, or
 * NULL for an LP.  The scaled problem holds D_c Q D_c, so q~_j = dc_j^2 q_j;
 * the step size and primal weight are those of the LP part.               */
int ora_set_qdiag(ora_prob *P, const double *q)
{
    free(P->q);
    P->q = NULL;
    if (!q) return 0;
    P->q = (double *)malloc(sizeof(double) * (size_t)(P->n > 0 ? P->n : 1));
    for (int32_t j = 0; j < P->n; ++j) P->q[j] = P->dc[j] * P->dc[j] * q[j];
    return 0;
}

/* Products with the scaled matrix (for tests). */
void ora_spmv(const ora_prob *P, int32_t transpose, const double *in, double *out)
{
    if (transpose) spmv_csc(P, in, out); else spmv_csr(P, in, out);
}

/* Power iteration on an arbitrary prepared problem (for tests). */
double ora_sigma_max(const ora_prob *P, int32_t max_iters, double tol, int32_t *iters)
{
    return power_sigma_max(P, max_iters, tol, iters);
}

/* ---- the PDHG operator T and one Halpern step (Sec. 2.2, App. B.1) ------
 * In:  x (n), y (m): the current iterate z_k; xa, ya: the epoch anchor.
 * Out: xh, yh = T(z_k); xb = 2 xh - x; xn, yn = z_{k+1} (may alias nothing). */
static void pdhg_halpern(const ora_prob *P, const double *x, const double *y,
                         const double *xa, const double *ya, int64_t k,
                         double tau, double sigma, double gamma,
                         double *xh, double *xb, double *yh, double *xn, double *yn)
{
    int32_t m = P->m, n = P->n;
    double a = (double)(k + 1) / (double)(k + 2);
    double b = 1.0 / (double)(k + 2);
    /* primal: xh = proj_X(x - tau (c - A^T y)), xbar = 2 xh - x.  With a
     * diagonal Q (Sec. 6) xh minimises q x^2 / 2 + (c - A^T y) x
     * + (x - x_k)^2 / (2 tau) over the box, separately per column: the
     * unconstrained minimiser (x_k - tau (c - A^T y)) / (1 + tau q) clamped
     * into [l, u] (a convex one-dimensional quadratic). */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < n; ++j) {
        double aty = 0.0;
        for (int64_t p = P->cp[j]; p < P->cp[j + 1]; ++p) aty += P->vt[p] * y[P->ri[p]];
        double g = P->c[j] - aty;
        double u = x[j] - tau * g;
        if (P->q) u = u / (1.0 + tau * P->q[j]);
        double xhj = clampd(u, P->vlo[j], P->vhi[j]);
        xh[j] = xhj;
        xb[j] = 2.0 * xhj - x[j];
    }
    /* dual: w = y/sigma - A xbar, yh = sigma (w - proj_{-S}(w)) */
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < m; ++i) {
        double q = 0.0;
        for (int64_t p = P->rp[i]; p < P->rp[i + 1]; ++p) q += P->v[p] * xb[P->ci[p]];
        double w = y[i] / sigma - q;
        yh[i] = sigma * (w - clampd(w, -P->chi[i], -P->clo[i]));
    }
    /* reflected Halpern step towards the epoch anchor */
    for (int32_t j = 0; j < n; ++j)
        xn[j] = a * ((1.0 + gamma) * xh[j] - gamma * x[j]) + b * xa[j];
    for (int32_t i = 0; i < m; ++i)
        yn[i] = a * ((1.0 + gamma) * yh[i] - gamma * y[i]) + b * ya[i];
}

/* Exported single step in the scaled space (tests). */
void ora_step(const ora_prob *P, const double *x, const double *y, const double *xa,
              const double *ya, int64_t k, double tau, double sigma, double gamma,
              double *xh, double *xb, double *yh, double *xn, double *yn)
{
    pdhg_halpern(P, x, y, xa, ya, k, tau, sigma, gamma, xh, xb, yh, xn, yn);
}

/* ---- A7: KKT of the original problem at the scaled point (xh, yh) -------
 * out: r_primal, r_dual, r_gap, obj_primal, obj_dual.                     */
static void kkt_eval(const ora_prob *P, const double *xh, const double *yh, double tau,
                     double *out)
{
    int32_t m = P->m, n = P->n;
    double *ax = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *aty = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    spmv_csr(P, xh, ax);
    spmv_csc(P, yh, aty);
    double pres = 0.0, dres = 0.0, cx = 0.0, sx = 0.0, py = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        double axi = ax[i] / P->dr[i];                 /* (A x)_i, original */
        double ri = axi - clampd(axi, P->clo0[i], P->chi0[i]);
        pres += ri * ri;
        double yi = P->dr[i] * yh[i];                  /* original dual     */
        /* -p(-y; l, u) = l^T y+ - u^T y-   (0 * inf = 0) */
        if (yi > 0.0) py += P->clo0[i] * yi;
        else if (yi < 0.0) py += P->chi0[i] * yi;
    }
    for (int32_t j = 0; j < n; ++j) {
        /* scaled c + Q x - A^T y; with D_c Q D_c the scaled Q, its term
         * q~ x~ is D_c (Q x), and q~ x~^2 = x^T Q x per column */
        double qx = P->q ? P->q[j] * xh[j] : 0.0;
        double g = P->c[j] + qx - aty[j];
        double u = xh[j] - tau * g;
        double s = (clampd(u, P->vlo[j], P->vhi[j]) - u) / tau;
        double dres_j = (g - s) / P->dc[j];            /* original c + Qx - A^T y - s */
        dres += dres_j * dres_j;
        double xj = P->dc[j] * xh[j];                  /* original primal   */
        double half_xqx = 0.5 * qx * xh[j];
        cx += P->c0[j] * xj + half_xqx;                /* c^T x + x^T Q x / 2 */
        sx += (s / P->dc[j]) * xj - half_xqx;          /* dual: - x^T Q x / 2 */
    }
    double dobj = py + sx;
    out[0] = sqrt(pres) / (1.0 + P->b_norm);
    out[1] = sqrt(dres) / (1.0 + P->c_norm);
    out[2] = fabs(cx - dobj) / (1.0 + fmax(fabs(cx), fabs(dobj)));
    out[3] = cx;
    out[4] = dobj;
    free(ax); free(aty);
}

/* KKT at an ORIGINAL-space point (x, y) with primal step tau (tests). */
void ora_kkt(const ora_prob *P, const double *x, const double *y, double tau, double *out5)
{
    double *xs = (double *)malloc(sizeof(double) * (size_t)(P->n > 0 ? P->n : 1));
    double *ys = (double *)malloc(sizeof(double) * (size_t)(P->m > 0 ? P->m : 1));
    for (int32_t j = 0; j < P->n; ++j) xs[j] = x[j] / P->dc[j];
    for (int32_t i = 0; i < P->m; ++i) ys[i] = y[i] / P->dr[i];
    kkt_eval(P, xs, ys, tau, out5);
    free(xs); free(ys);
}

/* KKT at a SCALED-space point (tests). */
void ora_kkt_scaled(const ora_prob *P, const double *xh, const double *yh, double tau,
                    double *out5)
{
    kkt_eval(P, xh, yh, tau, out5);
}

/* ---- A9: PID primal-weight update (App. B.3) ---------------------------- */
void ora_pid(double *omega, double *pid_int, double *pid_prev, int32_t *started,
             double dx, double dy, double kp, double ki, double kd)
{
    if (dx < 1e-10 || dy < 1e-10) return;
    double e = log(*omega * dx / dy);
    if (!*started) { *pid_prev = e; *started = 1; }
    *pid_int += e;
    double lw = log(*omega) - (kp * e + ki * *pid_int + kd * (e - *pid_prev));
    *pid_prev = e;
    *omega = exp(lw);
}

/* ---- start point: scaled, clamped into X, projected onto Y --------------- */
void ora_init_state(const ora_prob *P, const double *x0, const double *y0,
                    double *x, double *y, double *xa, double *ya, ora_state *S)
{
    for (int32_t j = 0; j < P->n; ++j) {
        double v = x0 ? x0[j] / P->dc[j] : 0.0;
        x[j] = clampd(v, P->vlo[j], P->vhi[j]);
        xa[j] = x[j];
    }
    for (int32_t i = 0; i < P->m; ++i) {
        double v = y0 ? y0[i] / P->dr[i] : 0.0;
        int lo_f = isfinite(P->clo[i]), hi_f = isfinite(P->chi[i]);
        if (!lo_f && !hi_f) v = 0.0;
        else if (!lo_f) v = fmin(v, 0.0);    /* only an upper bound: y <= 0 */
        else if (!hi_f) v = fmax(v, 0.0);    /* only a lower bound:  y >= 0 */
        y[i] = v;
        ya[i] = v;
    }
    memset(S, 0, sizeof(*S));
    S->omega = P->omega0;
}

/* ---- the restarted Halpern PDHG loop ------------------------------------
 * Runs up to n_iters iterations from the state (x, y, xa, ya, S) in place.
 * xh, yh receive T(z) of the last iteration.  log (may be NULL) receives up
 * to log_cap records.  Returns the number of iterations run.               */
int64_t ora_run(const ora_prob *P, const ora_params *prm, int64_t n_iters,
                double *x, double *y, double *xa, double *ya, double *xh, double *yh,
                ora_state *S, ora_log *log, int32_t log_cap)
{
    int32_t m = P->m, n = P->n;
    size_t mz = (size_t)(m > 0 ? m : 1), nz = (size_t)(n > 0 ? n : 1);
    double *xb = (double *)malloc(sizeof(double) * nz);
    double *xn = (double *)malloc(sizeof(double) * nz);
    double *yn = (double *)malloc(sizeof(double) * mz);
    double *dx = (double *)malloc(sizeof(double) * nz);
    double *dy = (double *)malloc(sizeof(double) * mz);
    double *adx = (double *)malloc(sizeof(double) * mz);
    double eta = P->eta;
    int64_t done = 0;
    int32_t nlog = 0;
    S->status = 0;
    while (done < n_iters) {
        double tau = eta / S->omega, sigma = eta * S->omega;
        int is_check = (S->k == 0) || ((S->t + 1) % prm->check_period == 0);
        pdhg_halpern(P, x, y, xa, ya, S->k, tau, sigma, prm->gamma, xh, xb, yh, xn, yn);
        done++;
        if (!is_check) {
            memcpy(x, xn, sizeof(double) * (size_t)n);
            memcpy(y, yn, sizeof(double) * (size_t)m);
            S->k++; S->t++;
            continue;
        }
        /* KKT at T(z_k) (App. B.4) */
        double kk[5];
        kkt_eval(P, xh, yh, tau, kk);
        S->r_primal = kk[0]; S->r_dual = kk[1]; S->r_gap = kk[2];
        S->obj_p = kk[3]; S->obj_d = kk[4];
        /* fixed-point residual ||z_k - T(z_k)||_P (App. B.2, D.2.1) */
        for (int32_t j = 0; j < n; ++j) dx[j] = x[j] - xh[j];
        for (int32_t i = 0; i < m; ++i) dy[i] = y[i] - yh[i];
        spmv_csr(P, dx, adx);
        double r2 = (S->omega / eta) * dot(dx, dx, n) + dot(dy, dy, m) / (eta * S->omega)
                  + 2.0 * dot(adx, dy, m);
        double r = sqrt(fmax(r2, 0.0));
        S->kkt_r = r;
        int32_t restart = 0;
        double kkt = fmax(kk[0], fmax(kk[1], kk[2]));
        int converged = kkt <= prm->eps;
        if (!converged) {
            if (S->k == 0) {
                S->r0 = r;
            } else if (r <= prm->beta_suf * S->r0) {
                restart = 1;
            } else if (r <= prm->beta_nec * S->r0 && r > S->r_prev) {
                restart = 2;
            } else if ((double)S->k >= prm->beta_art * (double)S->t) {
                restart = 3;
            }
        }
        if (log && nlog < log_cap) {
            ora_log *L = &log[nlog++];
            L->t = S->t; L->k = S->k; L->r = r; L->r0 = S->r0;
            L->r_primal = kk[0]; L->r_dual = kk[1]; L->r_gap = kk[2];
            L->omega = S->omega; L->restart = restart; L->pad = 0;
        }
        S->n_checks++;
        if (converged) {
            S->status = 1;
            S->t++;
            break;
        }
        if (restart) {
            /* PID on the distances to the anchor (App. B.3) */
            double ddx = 0.0, ddy = 0.0;
            for (int32_t j = 0; j < n; ++j) ddx += (xh[j] - xa[j]) * (xh[j] - xa[j]);
            for (int32_t i = 0; i < m; ++i) ddy += (yh[i] - ya[i]) * (yh[i] - ya[i]);
            ora_pid(&S->omega, &S->pid_int, &S->pid_prev, &S->pid_started,
                    sqrt(ddx), sqrt(ddy), prm->kp, prm->ki, prm->kd);
            memcpy(x, xh, sizeof(double) * (size_t)n);
            memcpy(xa, xh, sizeof(double) * (size_t)n);
            memcpy(y, yh, sizeof(double) * (size_t)m);
            memcpy(ya, yh, sizeof(double) * (size_t)m);
            S->k = 0;
            S->restarts++;
        } else {
            S->r_prev = r;
            memcpy(x, xn, sizeof(double) * (size_t)n);
            memcpy(y, yn, sizeof(double) * (size_t)m);
            S->k++;
        }
        S->t++;
    }
    if (S->status == 0 && done >= n_iters) S->status = 2;
    free(xb); free(xn); free(yn); free(dx); free(dy); free(adx);
    return done;
}

/* Unscale a scaled point: x = D_c xh, y = D_r yh. */
void ora_unscale(const ora_prob *P, const double *xh, const double *yh, double *x, double *y)
{
    for (int32_t j = 0; j < P->n; ++j) x[j] = P->dc[j] * xh[j];
    for (int32_t i = 0; i < P->m; ++i) y[i] = P->dr[i] * yh[i];
}

int32_t ora_num_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
