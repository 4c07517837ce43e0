/*
 * Oracle: discretisations.  Test infrastructure only (see oracle.h).
 *
 * Q1 stencil: the paper's section 4 gives the bilinear nine-point stencil for
 * a cellwise isotropic coefficient g (corners -g/3, edges -(g_i+g_j)/6,
 * centre (2/3) sum g, all over h^2).  For a symmetric tensor K per cell the
 * same element integrals of the bilinear basis give, for the cell in which
 * the node is local corner (sx, sy) (sx = +1 when the cell lies east of the
 * node, sy = +1 when it lies north):
 *   self                      (k11 + k22)/3 + sx*sy*k12/2
 *   neighbour along x         -k11/3 + k22/6
 *   neighbour along y          k11/6 - k22/3
 *   diagonal neighbour        -(k11 + k22)/6 - sx*sy*k12/2
 * With k11 = k22 = g, k12 = 0 this is exactly the paper's formula.
 */
#include "oracle.h"
#include <math.h>
#include <string.h>
#include "util.h"

static int in_grid(int n, int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; }

void ora_stencil_q1_cells(int n, const double *k11, const double *k12,
                          const double *k22, double *A)
{
    const int64_t nn = (int64_t)n * n;
    const int nc = n + 1; /* cells per side */
#pragma omp parallel for
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            double s[9] = {0};
            /* the four cells around node (i, j): cell (I, J) has lower-left node (I-1, J-1) */
            for (int sy = -1; sy <= 1; sy += 2) {
                for (int sx = -1; sx <= 1; sx += 2) {
                    int I = i + (sx > 0 ? 1 : 0);
                    int J = j + (sy > 0 ? 1 : 0);
                    int64_t cidx = (int64_t)J * nc + I;
                    double a = k11[cidx], b = k12[cidx], c = k22[cidx];
                    double sgn = (double)(sx * sy);
                    /* self */
                    s[4] += (a + c) / 3.0 + sgn * b / 2.0;
                    /* x-neighbour on the cell's side */
                    s[3 * 1 + (sx + 1)] += -a / 3.0 + c / 6.0;
                    /* y-neighbour on the cell's side */
                    s[3 * (sy + 1) + 1] += a / 6.0 - c / 3.0;
                    /* diagonal neighbour */
                    s[3 * (sy + 1) + (sx + 1)] += -(a + c) / 6.0 - sgn * b / 2.0;
                }
            }
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int c = 3 * (dy + 1) + (dx + 1);
                    double v = in_grid(n, i + dx, j + dy) ? s[c] : 0.0;
                    A[c * nn + (int64_t)j * n + i] = v;
                }
        }
    }
}

void ora_stencil_q1_rotated(int n, double theta, double eps, double *A)
{
    /* K = R diag(1, eps) R^T with R the rotation by theta */
    const double c = cos(theta), s = sin(theta);
    const double k11 = c * c + eps * s * s;
    const double k12 = c * s * (1.0 - eps);
    const double k22 = s * s + eps * c * c;
    const int64_t ncell = (int64_t)(n + 1) * (n + 1);
    double *a = (double *)malloc_or_die(3 * ncell * sizeof(double));
    for (int64_t q = 0; q < ncell; ++q) {
        a[q] = k11;
        a[ncell + q] = k12;
        a[2 * ncell + q] = k22;
    }
    ora_stencil_q1_cells(n, a, a + ncell, a + 2 * ncell, A);
    free(a);
}

void ora_stencil_cellavg5(int n, const double *a, double *A)
{
    const int64_t nn = (int64_t)n * n;
    const int nc = n + 1;
#pragma omp parallel for
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            /* cells around node (i, j): SW = (i, j), SE = (i+1, j), NW = (i, j+1), NE = (i+1, j+1) */
            double sw = a[(int64_t)j * nc + i], se = a[(int64_t)j * nc + i + 1];
            double nw = a[(int64_t)(j + 1) * nc + i], ne = a[(int64_t)(j + 1) * nc + i + 1];
            double aE = 0.5 * (se + ne), aW = 0.5 * (sw + nw);
            double aN = 0.5 * (nw + ne), aS = 0.5 * (sw + se);
            double s[9] = {0};
            s[4] = aE + aW + aN + aS;
            s[5] = -aE;
            s[3] = -aW;
            s[7] = -aN;
            s[1] = -aS;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int c = 3 * (dy + 1) + (dx + 1);
                    A[c * nn + (int64_t)j * n + i] = in_grid(n, i + dx, j + dy) ? s[c] : 0.0;
                }
        }
    }
}
