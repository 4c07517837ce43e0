/*
 * Oracle: stencil operators, grid transfers, Galerkin coarsening, dense
 * coarsest solve, smoothers, the V-cycle and the stationary solver.
 * Test infrastructure only (see oracle.h).
 */
#include "oracle.h"
#include <math.h>
#include <string.h>
#include "util.h"
#include <omp.h>

/* ------------------------------------------------------------------ */
/* y = A x.  Section 2, A u = f; a 9-point stencil per node.            */
/* ------------------------------------------------------------------ */
void ora_matvec(int n, const double *A, const double *x, double *y)
{
    const int64_t nn = (int64_t)n * n;
#pragma omp parallel for
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int ii = i + dx, jj = j + dy;
                    if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
                    int c = 3 * (dy + 1) + (dx + 1);
                    acc += A[c * nn + (int64_t)j * n + i] * x[(int64_t)jj * n + ii];
                }
            y[(int64_t)j * n + i] = acc;
        }
}

/* Bilinear interpolation weight of a fine node at offset b from a coarse
 * node (section 6, full coarsening): 1, 1/2, 1/4, zero beyond one cell. */
static double wP(int bx, int by)
{
    if (bx < -1 || bx > 1 || by < -1 || by > 1) return 0.0;
    return (1.0 - 0.5 * abs(bx)) * (1.0 - 0.5 * abs(by));
}

/* Full-weighting weight, (1/16)[1 2 1; 2 4 2; 1 2 1] = wP / 4. */
static double wR(int ax, int ay) { return 0.25 * wP(ax, ay); }

void ora_restrict_fw(int n, const double *r, double *rc)
{
    const int nc = (n - 1) / 2;
#pragma omp parallel for
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I < nc; ++I) {
            double acc = 0.0;
            for (int ay = -1; ay <= 1; ++ay)
                for (int ax = -1; ax <= 1; ++ax)
                    acc += wR(ax, ay) * r[(int64_t)(2 * J + 1 + ay) * n + (2 * I + 1 + ax)];
            rc[(int64_t)J * nc + I] = acc;
        }
}

void ora_prolong_add(int n, const double *ec, double *e)
{
    const int nc = (n - 1) / 2;
#pragma omp parallel for
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            /* coarse nodes whose support reaches fine node (i, j) */
            for (int J = (j - 2) / 2; J <= j / 2; ++J)
                for (int I = (i - 2) / 2; I <= i / 2; ++I) {
                    if (I < 0 || I >= nc || J < 0 || J >= nc) continue;
                    acc += wP(i - (2 * I + 1), j - (2 * J + 1)) * ec[(int64_t)J * nc + I];
                }
            e[(int64_t)j * n + i] += acc;
        }
}

/* Ac = R A P in stencil form.  For coarse node I and coarse offset D:
 *   Ac_I[D] = sum_a wR(a) sum_d A_{2I+1+a}[d] wP(2I+1+a+d - (2(I+D)+1)),
 * zero when I+D lies outside the coarse grid (P has no such column). */
void ora_galerkin(int n, const double *A, double *Ac)
{
    const int nc = (n - 1) / 2;
    const int64_t nn = (int64_t)n * n, ncc = (int64_t)nc * nc;
#pragma omp parallel for
    for (int J = 0; J < nc; ++J)
        for (int I = 0; I < nc; ++I)
            for (int Dy = -1; Dy <= 1; ++Dy)
                for (int Dx = -1; Dx <= 1; ++Dx) {
                    int cD = 3 * (Dy + 1) + (Dx + 1);
                    double acc = 0.0;
                    if (I + Dx >= 0 && I + Dx < nc && J + Dy >= 0 && J + Dy < nc) {
                        for (int ay = -1; ay <= 1; ++ay)
                            for (int ax = -1; ax <= 1; ++ax) {
                                int xi = 2 * I + 1 + ax, xj = 2 * J + 1 + ay;
                                for (int dy = -1; dy <= 1; ++dy)
                                    for (int dx = -1; dx <= 1; ++dx) {
                                        double a = A[(3 * (dy + 1) + (dx + 1)) * nn + (int64_t)xj * n + xi];
                                        acc += wR(ax, ay) * a * wP(ax + dx - 2 * Dx, ay + dy - 2 * Dy);
                                    }
                            }
                    }
                    Ac[cD * ncc + (int64_t)J * nc + I] = acc;
                }
}

/* ------------------------------------------------------------------ */
/* Dense coarsest solve (Algorithm 1: solve A u = r on the last level). */
/* ------------------------------------------------------------------ */
void ora_stencil_to_dense(int n, const double *A, double *M)
{
    const int64_t nn = (int64_t)n * n;
    memset(M, 0, sizeof(double) * nn * nn);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int ii = i + dx, jj = j + dy;
                    if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
                    M[((int64_t)j * n + i) * nn + (int64_t)jj * n + ii] =
                        A[(3 * (dy + 1) + (dx + 1)) * nn + (int64_t)j * n + i];
                }
}

int ora_cholesky(int m, double *M)
{
    for (int k = 0; k < m; ++k) {
        double d = M[(int64_t)k * m + k];
        for (int p = 0; p < k; ++p) d -= M[(int64_t)k * m + p] * M[(int64_t)k * m + p];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        M[(int64_t)k * m + k] = d;
        for (int i = k + 1; i < m; ++i) {
            double s = M[(int64_t)i * m + k];
            for (int p = 0; p < k; ++p) s -= M[(int64_t)i * m + p] * M[(int64_t)k * m + p];
            M[(int64_t)i * m + k] = s / d;
        }
        for (int jj = k + 1; jj < m; ++jj) M[(int64_t)k * m + jj] = 0.0;
    }
    return 0;
}

void ora_cholesky_solve(int m, const double *L, const double *b, double *x)
{
    /* L y = b, then L^T x = y */
    for (int i = 0; i < m; ++i) {
        double s = b[i];
        for (int p = 0; p < i; ++p) s -= L[(int64_t)i * m + p] * x[p];
        x[i] = s / L[(int64_t)i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = x[i];
        for (int p = i + 1; p < m; ++p) s -= L[(int64_t)p * m + i] * x[p];
        x[i] = s / L[(int64_t)i * m + i];
    }
}

/* ------------------------------------------------------------------ */
/* Smoothers: u <- u + M^{-1}(f - A u) (section 2.1), M = D/omega for   */
/* damped Jacobi; the learned smoother is a per-point 5x5 kernel.       */
/* ------------------------------------------------------------------ */
void ora_smooth_jacobi(int n, const double *A, double omega, const double *r, double *e)
{
    const int64_t nn = (int64_t)n * n;
    double *s = (double *)malloc_or_die(sizeof(double) * nn);
    ora_matvec(n, A, e, s);
    for (int64_t p = 0; p < nn; ++p) s[p] = r[p] - s[p];
    for (int64_t p = 0; p < nn; ++p) e[p] += omega * s[p] / A[4 * nn + p];
    free(s);
}

void ora_apply_smoother5(int n, const double *A, const double *W, const double *x, double *y)
{
    const int64_t nn = (int64_t)n * n;
#pragma omp parallel for
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx) {
                    int ii = i + dx, jj = j + dy;
                    if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
                    int k = 5 * (dy + 2) + (dx + 2);
                    acc += W[k * nn + (int64_t)j * n + i] * x[(int64_t)jj * n + ii];
                }
            y[(int64_t)j * n + i] = acc / A[4 * nn + (int64_t)j * n + i];
        }
}

void ora_smooth_stencil5(int n, const double *A, const double *W, const double *r, double *e)
{
    const int64_t nn = (int64_t)n * n;
    double *s = (double *)malloc_or_die(sizeof(double) * nn);
    double *t = (double *)malloc_or_die(sizeof(double) * nn);
    ora_matvec(n, A, e, s);
    for (int64_t p = 0; p < nn; ++p) s[p] = r[p] - s[p];
    ora_apply_smoother5(n, A, W, s, t);
    for (int64_t p = 0; p < nn; ++p) e[p] += t[p];
    free(s);
    free(t);
}

/* ------------------------------------------------------------------ */
/* Hierarchy, V-cycle (Algorithm 1) and solver (section 2, Phi(u0,f,k)) */
/* ------------------------------------------------------------------ */
struct ora_mg {
    int nlev;
    int n[32];
    double *A[32];   /* stencil per level */
    double *W[32];   /* learned smoother per level, NULL = damped Jacobi */
    double *L;       /* Cholesky factor of the coarsest matrix */
};

ora_mg *ora_mg_create(int n, const double *A0, int coarsest_n)
{
    if (n < 1 || coarsest_n < 1) return NULL;
    ora_mg *mg = (ora_mg *)malloc_or_die(sizeof(ora_mg));
    int lv = 0, m = n;
    mg->n[0] = n;
    mg->A[0] = (double *)malloc_or_die(sizeof(double) * 9 * (size_t)n * n);
    memcpy(mg->A[0], A0, sizeof(double) * 9 * (size_t)n * n);
    while (m > coarsest_n) {
        if (m % 2 == 0 || lv >= 30) { ora_mg_destroy(mg); return NULL; }
        int mc = (m - 1) / 2;
        mg->A[lv + 1] = (double *)malloc_or_die(sizeof(double) * 9 * (size_t)mc * mc);
        ora_galerkin(m, mg->A[lv], mg->A[lv + 1]);
        ++lv;
        m = mc;
        mg->n[lv] = m;
    }
    mg->nlev = lv + 1;
    if (m != coarsest_n) { ora_mg_destroy(mg); return NULL; }
    const int mm = m * m;
    mg->L = (double *)malloc_or_die(sizeof(double) * (size_t)mm * mm);
    ora_stencil_to_dense(m, mg->A[lv], mg->L);
    if (ora_cholesky(mm, mg->L) != 0) { ora_mg_destroy(mg); return NULL; }
    return mg;
}

void ora_mg_destroy(ora_mg *mg)
{
    if (!mg) return;
    for (int l = 0; l < 32; ++l) {
        free(mg->A[l]);
        free(mg->W[l]);
    }
    free(mg->L);
    free(mg);
}

int ora_mg_num_levels(const ora_mg *mg) { return mg->nlev; }
int ora_mg_level_n(const ora_mg *mg, int level) { return mg->n[level]; }

void ora_mg_get_stencil(const ora_mg *mg, int level, double *A)
{
    memcpy(A, mg->A[level], sizeof(double) * 9 * (size_t)mg->n[level] * mg->n[level]);
}

int ora_mg_set_smoother(ora_mg *mg, int level, const double *W)
{
    if (level < 0 || level >= mg->nlev - 1) return -1;
    free(mg->W[level]);
    mg->W[level] = NULL;
    if (W) {
        size_t bytes = sizeof(double) * 25 * (size_t)mg->n[level] * mg->n[level];
        mg->W[level] = (double *)malloc_or_die(bytes);
        memcpy(mg->W[level], W, bytes);
    }
    return 0;
}

static void smooth(ora_mg *mg, int l, double omega, const double *r, double *e)
{
    if (mg->W[l])
        ora_smooth_stencil5(mg->n[l], mg->A[l], mg->W[l], r, e);
    else
        ora_smooth_jacobi(mg->n[l], mg->A[l], omega, r, e);
}

/* e = V_l(r): the correction form of Algorithm 1 with zero initial guess. */
void ora_mg_vcycle(ora_mg *mg, int l, int nu1, int nu2, double omega, const double *r, double *e)
{
    const int n = mg->n[l];
    const int64_t nn = (int64_t)n * n;
    if (l == mg->nlev - 1) { /* coarsest level: direct solve */
        ora_cholesky_solve((int)nn, mg->L, r, e);
        return;
    }
    for (int64_t p = 0; p < nn; ++p) e[p] = 0.0;
    for (int s = 0; s < nu1; ++s) smooth(mg, l, omega, r, e);          /* pre-smoothing  */
    const int nc = mg->n[l + 1];
    double *res = (double *)malloc_or_die(sizeof(double) * nn);
    double *rc = (double *)malloc_or_die(sizeof(double) * (size_t)nc * nc);
    double *ec = (double *)malloc_or_die(sizeof(double) * (size_t)nc * nc);
    ora_matvec(n, mg->A[l], e, res);                                      /* residual      */
    for (int64_t p = 0; p < nn; ++p) res[p] = r[p] - res[p];
    ora_restrict_fw(n, res, rc);                                          /* restrict      */
    ora_mg_vcycle(mg, l + 1, nu1, nu2, omega, rc, ec);                    /* coarse solve  */
    ora_prolong_add(n, ec, e);                                            /* correct       */
    for (int s = 0; s < nu2; ++s) smooth(mg, l, omega, r, e);          /* post-smoothing */
    free(res);
    free(rc);
    free(ec);
}

static double norm2(int64_t m, const double *x)
{
    double s = 0.0;
    for (int64_t p = 0; p < m; ++p) s += x[p] * x[p];
    return sqrt(s);
}

int ora_mg_solve(ora_mg *mg, const double *f, double *u, double tol, int maxit, int nu1, int nu2,
                 double omega, double *history, int *converged)
{
    const int n = mg->n[0];
    const int64_t nn = (int64_t)n * n;
    double *r = (double *)malloc_or_die(sizeof(double) * nn);
    double *e = (double *)malloc_or_die(sizeof(double) * nn);
    const double fnorm = norm2(nn, f);
    for (int64_t p = 0; p < nn; ++p) u[p] = 0.0;
    int k = 0;
    *converged = 0;
    for (;;) {
        ora_matvec(n, mg->A[0], u, r);
        for (int64_t p = 0; p < nn; ++p) r[p] = f[p] - r[p];
        double rel = fnorm > 0.0 ? norm2(nn, r) / fnorm : 0.0;
        if (history) history[k] = rel;
        if (rel <= tol) { *converged = 1; break; }
        if (k == maxit) break;
        ora_mg_vcycle(mg, 0, nu1, nu2, omega, r, e);
        for (int64_t p = 0; p < nn; ++p) u[p] += e[p];
        ++k;
    }
    free(r);
    free(e);
    return k;
}

int ora_num_threads(void) { return omp_get_max_threads(); }

void ora_set_threads(int nthreads)
{
    if (nthreads >= 1) omp_set_num_threads(nthreads);
}
