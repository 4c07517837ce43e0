/*
 * Oracle: the stencil-to-smoother CNN (paper section 4.2, convolutional
 * hypernetwork), the high-frequency smoothing loss and its gradient, and
 * Adam.  Test infrastructure only (see oracle.h).
 *
 * The loss follows from section 3.1: the smoother needs to remove only the
 * errors the coarse grid cannot (section 2.2), and for z uniform on a sphere
 * E(n ||X z||^2) = ||X||_F^2, so the norm of (I - H A) applied to random
 * high-frequency unit vectors measures the smoother's error propagator on
 * that subspace.  The gradient is plain reverse-mode differentiation of the
 * forward definition; a ReLU's derivative at exactly 0 is taken as 0.
 */
#include "oracle.h"
#include <math.h>
#include <string.h>
#include "util.h"

int64_t ora_cnn_num_params(int nlayers, const int *ch)
{
    int64_t np = 0;
    for (int l = 0; l < nlayers; ++l) np += (int64_t)ch[l + 1] * ch[l] * 9 + ch[l + 1];
    return np;
}

/* y[co] = b[co] + sum_ci sum_{ky,kx} w[co][ci][ky][kx] x[ci](j+ky-1, i+kx-1),
 * inputs outside the grid taken as zero ("same" padding). */
static void conv3x3(int n, int cin, int cout, const double *w, const double *b,
                    const double *x, double *y)
{
    const int64_t nn = (int64_t)n * n;
#pragma omp parallel for
    for (int co = 0; co < cout; ++co)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double acc = b[co];
                for (int ci = 0; ci < cin; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int jj = j + ky - 1, ii = i + kx - 1;
                            if (jj < 0 || jj >= n || ii < 0 || ii >= n) continue;
                            acc += w[((co * cin + ci) * 3 + ky) * 3 + kx] * x[ci * nn + (int64_t)jj * n + ii];
                        }
                y[co * nn + (int64_t)j * n + i] = acc;
            }
}

/* Forward pass keeping every layer's pre-activation.  pre[l] is
 * [ch[l+1]][n][n]; the activation of layer l is relu(pre[l]) except for the
 * last layer.  x0 receives the network input A / a_C. */
static void cnn_forward_store(int n, const double *A, int nlayers, const int *ch,
                              const double *params, double *x0, double **pre)
{
    const int64_t nn = (int64_t)n * n;
    for (int c = 0; c < 9; ++c)
        for (int64_t p = 0; p < nn; ++p) x0[c * nn + p] = A[c * nn + p] / A[4 * nn + p];
    const double *in = x0;
    double *act = NULL;
    int64_t off = 0;
    for (int l = 0; l < nlayers; ++l) {
        const int cin = ch[l], cout = ch[l + 1];
        const double *w = params + off, *b = params + off + (int64_t)cout * cin * 9;
        off += (int64_t)cout * cin * 9 + cout;
        conv3x3(n, cin, cout, w, b, in, pre[l]);
        if (l + 1 < nlayers) {
            free(act);
            act = (double *)malloc_or_die(sizeof(double) * cout * nn);
            for (int64_t q = 0; q < cout * nn; ++q) act[q] = pre[l][q] > 0.0 ? pre[l][q] : 0.0;
            in = act;
        }
    }
    free(act);
}

void ora_cnn_forward(int n, const double *A, int nlayers, const int *ch, const double *params,
                     double omega, double *W)
{
    const int64_t nn = (int64_t)n * n;
    double *x0 = (double *)malloc_or_die(sizeof(double) * 9 * nn);
    double *pre[16];
    for (int l = 0; l < nlayers; ++l) pre[l] = (double *)malloc_or_die(sizeof(double) * ch[l + 1] * nn);
    cnn_forward_store(n, A, nlayers, ch, params, x0, pre);
    const int cout = ch[nlayers];
    for (int k = 0; k < cout; ++k)
        for (int64_t p = 0; p < nn; ++p) W[k * nn + p] = pre[nlayers - 1][k * nn + p] + (k == 12 ? omega : 0.0);
    /* the off-centre entries of a diffusion row sum to a negative value (to
     * -a_C inside the domain, where rows sum to zero); a row whose off-centre
     * sum is not negative (a Dirichlet node of a masked domain and its
     * Galerkin images on coarser levels, where coarsened Dirichlet rows weigh
     * in) is not a stencil the network was made for: damped Jacobi there */
    for (int64_t p = 0; p < nn; ++p) {
        double off = 0.0;
        for (int c = 0; c < 9; ++c)
            if (c != 4) off += A[c * nn + p];
        if (off >= 0.0)
            for (int k = 0; k < cout; ++k) W[k * nn + p] = k == 12 ? omega : 0.0;
    }
    for (int l = 0; l < nlayers; ++l) free(pre[l]);
    free(x0);
}

/* Gradient of one problem's summed loss contribution with respect to the
 * parameters, given dW = dL/dW (the gradient with respect to the network
 * output).  Accumulates into grad. */
static void cnn_backward(int n, int nlayers, const int *ch, const double *params, const double *x0,
                         double **pre, const double *dW, double *grad)
{
    const int64_t nn = (int64_t)n * n;
    int64_t offs[17];
    offs[0] = 0;
    for (int l = 0; l < nlayers; ++l) offs[l + 1] = offs[l] + (int64_t)ch[l + 1] * ch[l] * 9 + ch[l + 1];
    /* dpre holds the gradient with respect to the current layer's pre-activation */
    double *dpre = (double *)malloc_or_die(sizeof(double) * ch[nlayers] * nn);
    memcpy(dpre, dW, sizeof(double) * ch[nlayers] * nn);
    for (int l = nlayers - 1; l >= 0; --l) {
        const int cin = ch[l], cout = ch[l + 1];
        const double *w = params + offs[l];
        double *gw = grad + offs[l], *gb = grad + offs[l] + (int64_t)cout * cin * 9;
        /* the layer's input: x0 for the first layer, relu(pre[l-1]) otherwise */
        double *xin = (double *)malloc_or_die(sizeof(double) * cin * nn);
        if (l == 0)
            memcpy(xin, x0, sizeof(double) * cin * nn);
        else
            for (int64_t q = 0; q < cin * nn; ++q) xin[q] = pre[l - 1][q] > 0.0 ? pre[l - 1][q] : 0.0;
        /* dL/dw and dL/db */
        for (int co = 0; co < cout; ++co) {
            double sb = 0.0;
            for (int64_t p = 0; p < nn; ++p) sb += dpre[co * nn + p];
            gb[co] += sb;
            for (int ci = 0; ci < cin; ++ci)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        double s = 0.0;
                        for (int j = 0; j < n; ++j)
                            for (int i = 0; i < n; ++i) {
                                int jj = j + ky - 1, ii = i + kx - 1;
                                if (jj < 0 || jj >= n || ii < 0 || ii >= n) continue;
                                s += dpre[co * nn + (int64_t)j * n + i] * xin[ci * nn + (int64_t)jj * n + ii];
                            }
                        gw[((co * cin + ci) * 3 + ky) * 3 + kx] += s;
                    }
        }
        if (l > 0) {
            /* dL/dx of the layer input, then through the previous ReLU */
            double *dx = (double *)malloc_or_die(sizeof(double) * cin * nn);
#pragma omp parallel for
            for (int ci = 0; ci < cin; ++ci)
                for (int jj = 0; jj < n; ++jj)
                    for (int ii = 0; ii < n; ++ii) {
                        double s = 0.0;
                        for (int co = 0; co < cout; ++co)
                            for (int ky = 0; ky < 3; ++ky)
                                for (int kx = 0; kx < 3; ++kx) {
                                    int j = jj - ky + 1, i = ii - kx + 1; /* output that read (ii, jj) */
                                    if (j < 0 || j >= n || i < 0 || i >= n) continue;
                                    s += w[((co * cin + ci) * 3 + ky) * 3 + kx] * dpre[co * nn + (int64_t)j * n + i];
                                }
                        int64_t q = ci * nn + (int64_t)jj * n + ii;
                        dx[q] = pre[l - 1][q] > 0.0 ? s : 0.0;
                    }
            free(dpre);
            dpre = dx;
        }
        free(xin);
    }
    free(dpre);
}

void ora_cnn_vjp(int n, const double *A, int nlayers, const int *ch, const double *params, const double *dW,
                 double *grad)
{
    const int64_t nn = (int64_t)n * n;
    double *x0 = (double *)malloc_or_die(sizeof(double) * 9 * nn);
    double *pre[16];
    for (int l = 0; l < nlayers; ++l) pre[l] = (double *)malloc_or_die(sizeof(double) * ch[l + 1] * nn);
    cnn_forward_store(n, A, nlayers, ch, params, x0, pre);
    cnn_backward(n, nlayers, ch, params, x0, pre, dW, grad);
    for (int l = 0; l < nlayers; ++l) free(pre[l]);
    free(x0);
}

double ora_hf_loss(int B, const int *ns, const double *const *A, const double *const *V, int J,
                   int nlayers, const int *ch, const double *params, double omega, double *grad)
{
    const int64_t np = ora_cnn_num_params(nlayers, ch);
    if (grad) memset(grad, 0, sizeof(double) * np);
    const double scale = 1.0 / ((double)B * J);
    double total = 0.0;
    for (int b = 0; b < B; ++b) {
        const int n = ns[b];
        const int64_t nn = (int64_t)n * n;
        const double *Ab = A[b];
        double *x0 = (double *)malloc_or_die(sizeof(double) * 9 * nn);
        double *pre[16];
        for (int l = 0; l < nlayers; ++l) pre[l] = (double *)malloc_or_die(sizeof(double) * ch[l + 1] * nn);
        cnn_forward_store(n, Ab, nlayers, ch, params, x0, pre);
        double *W = (double *)malloc_or_die(sizeof(double) * 25 * nn);
        for (int k = 0; k < 25; ++k)
            for (int64_t p = 0; p < nn; ++p) W[k * nn + p] = pre[nlayers - 1][k * nn + p] + (k == 12 ? omega : 0.0);
        double *dW = (double *)malloc_or_die(sizeof(double) * 25 * nn);
        double *Av = (double *)malloc_or_die(sizeof(double) * nn);
        double *y = (double *)malloc_or_die(sizeof(double) * nn);
        for (int jv = 0; jv < J; ++jv) {
            const double *v = V[b] + (int64_t)jv * nn;
            ora_matvec(n, Ab, v, Av);
            ora_apply_smoother5(n, Ab, W, Av, y);  /* y = H A v */
            double g2 = 0.0;
            for (int64_t p = 0; p < nn; ++p) g2 += (v[p] - y[p]) * (v[p] - y[p]);
            const double gn = sqrt(g2);
            total += gn;
            if (!grad || gn == 0.0) continue;
            /* d||g||/dW_p[k] = -(g_p/||g||) Av_{p+k} / a_C(p) */
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const int64_t p = (int64_t)j * n + i;
                    const double gp = (v[p] - y[p]) / gn;
                    for (int dy = -2; dy <= 2; ++dy)
                        for (int dx = -2; dx <= 2; ++dx) {
                            int ii = i + dx, jj = j + dy;
                            if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
                            int k = 5 * (dy + 2) + (dx + 2);
                            dW[k * nn + p] -= scale * gp * Av[(int64_t)jj * n + ii] / Ab[4 * nn + p];
                        }
                }
        }
        if (grad) cnn_backward(n, nlayers, ch, params, x0, pre, dW, grad);
        free(W);
        free(dW);
        free(Av);
        free(y);
        for (int l = 0; l < nlayers; ++l) free(pre[l]);
        free(x0);
    }
    return total * scale;
}

void ora_adam_step(int64_t np, double *p, double *m, double *v, const double *g, int t, double lr,
                   double beta1, double beta2, double eps)
{
    const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t q = 0; q < np; ++q) {
        m[q] = beta1 * m[q] + (1.0 - beta1) * g[q];
        v[q] = beta2 * v[q] + (1.0 - beta2) * g[q] * g[q];
        const double mhat = m[q] / c1, vhat = v[q] / c2;
        p[q] -= lr * mhat / (sqrt(vhat) + eps);
    }
}
