// Red-black coarsening (section 6.1: restriction (1/8)[0 1 0; 1 4 1; 0 1 0]
// and interpolation (1/4)][0 1 0; 1 4 1; 0 1 0][ along the level's mesh axes,
// Galerkin coarse operators) with damped Jacobi or the two-layer convolution
// smoother H = f2(f1) of section 6 on zero-padded irregular grids.  FP64.
//
// Every kernel works on a batch of vectors (blockIdx.z = vector) of one level;
// a per-vector flag array (or null) skips vectors that are done.  Point
// kernels use 64 x 4 threads per block, one node each; stencils are generic
// footprints (RBOffsets) because red-black Galerkin levels grow past 3 x 3.
#include "redblack.hpp"

namespace mg {

namespace {

constexpr int kBX = 64, kBY = 4;
constexpr int kNT = kBX * kBY;

dim3 point_grid(int N, int nvec) { return dim3((N + kBX - 1) / kBX, (N + kBY - 1) / kBY, nvec); }

__device__ inline bool inside(int N, int i, int j) { return i >= 0 && i < N && j >= 0 && j < N; }

// ------------------------------------------------------------------ operator
__global__ void __launch_bounds__(kNT) k_rb_residual(RBGeom g, RBOffsets o, const double *__restrict__ A,
                                                     const double *__restrict__ b, const double *__restrict__ x,
                                                     double *__restrict__ y, double sign, const int *active)
{
    const int v = blockIdx.z;
    if (active && !active[v]) return;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.N || j >= g.N) return;
    const int64_t p = (int64_t)j * g.P + i, off = v * g.vs;
    double acc = 0.0;
    if (rb_has(g.kind, i, j)) {
        const int64_t plane = g.vs;
        for (int c = 0; c < o.K; ++c) {
            const int ii = i + o.dx[c], jj = j + o.dy[c];
            if (inside(g.N, ii, jj)) acc += A[c * plane + p] * x[off + (int64_t)jj * g.P + ii];
        }
        acc = (b ? b[off + p] : 0.0) + sign * acc;
    }
    y[off + p] = acc;
}

// r = f - A u with per-block sums of r^2 (fixed block shape and order: deterministic).
__global__ void __launch_bounds__(kNT) k_rb_outer(RBGeom g, RBOffsets o, const double *__restrict__ A,
                                                  const double *__restrict__ f, const double *__restrict__ u,
                                                  double *__restrict__ r, double *__restrict__ partial, int nb,
                                                  const int *active)
{
    __shared__ double red[kNT / 64];
    const int v = blockIdx.z;
    if (active && !active[v]) return;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    double rr = 0.0;
    if (i < g.N && j < g.N) {
        const int64_t p = (int64_t)j * g.P + i, off = v * g.vs;
        double acc = 0.0;
        if (rb_has(g.kind, i, j)) {
            for (int c = 0; c < o.K; ++c) {
                const int ii = i + o.dx[c], jj = j + o.dy[c];
                if (inside(g.N, ii, jj)) acc += A[c * g.vs + p] * u[off + (int64_t)jj * g.P + ii];
            }
            acc = f[off + p] - acc;
        }
        r[off + p] = acc;
        rr = acc * acc;
    }
    const double s = block_sum<kNT>(rr, red);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[(int64_t)v * nb + blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_rb_sum(const double *__restrict__ partial, int nb, double *__restrict__ out)
{
    __shared__ double red[4];
    const int v = blockIdx.x;
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) acc += partial[(int64_t)v * nb + q];
    const double s = block_sum<256>(acc, red);
    if (threadIdx.x == 0) out[v] = s;
}

// ---------------------------------------------------------------- smoothers
__global__ void __launch_bounds__(kNT) k_rb_jacobi(RBGeom g, const double *__restrict__ Ac, double omega,
                                                   const double *__restrict__ s, double *__restrict__ e, int acc,
                                                   const int *active)
{
    const int v = blockIdx.z;
    if (active && !active[v]) return;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.N || j >= g.N) return;
    const int64_t p = (int64_t)j * g.P + i, off = v * g.vs;
    double d = 0.0;
    if (rb_has(g.kind, i, j)) d = omega * s[off + p] / Ac[p];
    e[off + p] = (acc ? e[off + p] : 0.0) + d;
}

// y (+)= Mout conv3(Min x, w): zero padding on the N x N array.
__global__ void __launch_bounds__(kNT) k_rb_conv(RBGeom g, const double *__restrict__ w, const double *__restrict__ x,
                                                 double *__restrict__ y, int mask_in, int mask_out, int acc,
                                                 const int *active)
{
    const int v = blockIdx.z;
    if (active && !active[v]) return;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.N || j >= g.N) return;
    const int64_t p = (int64_t)j * g.P + i, off = v * g.vs;
    double sum = 0.0;
    if (!mask_out || rb_has(g.kind, i, j)) {
        for (int k = 0; k < 9; ++k) {
            const int ii = i + k % 3 - 1, jj = j + k / 3 - 1;
            if (inside(g.N, ii, jj) && (!mask_in || rb_has(g.kind, ii, jj)))
                sum += w[k] * x[off + (int64_t)jj * g.P + ii];
        }
    }
    y[off + p] = (acc ? y[off + p] : 0.0) + sum;
}

// The tangent sources d(H x)/d w_j for the 18 weights (forward-mode training).
__global__ void __launch_bounds__(kNT) k_rb_dH(RBGeom g, const double *__restrict__ w, const double *__restrict__ x,
                                               int64_t xstride, const double *__restrict__ t, int64_t tstride_t,
                                               double *__restrict__ dy, int64_t ystride, int64_t tstride,
                                               const int *active, int active_stride)
{
    const int b = blockIdx.z;
    if (active && !active[(int64_t)b * active_stride]) return;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.N || j >= g.N || !rb_has(g.kind, i, j)) return;
    const int64_t p = (int64_t)j * g.P + i;
    const double *xb = x + b * xstride, *tb = t + b * tstride_t;
    double *yb = dy + b * ystride;
    for (int k = 0; k < 9; ++k) {
        const int kx = k % 3 - 1, ky = k / 3 - 1;
        // layer 1, tap k: f2(unit_k(M x)) at p
        double s1 = 0.0;
        for (int k2 = 0; k2 < 9; ++k2) {
            const int qi = i + k2 % 3 - 1, qj = j + k2 / 3 - 1;
            if (!inside(g.N, qi, qj)) continue;
            const int si = qi + kx, sj = qj + ky;
            if (inside(g.N, si, sj) && rb_has(g.kind, si, sj)) s1 += w[9 + k2] * xb[(int64_t)sj * g.P + si];
        }
        // layer 2, tap k: unit_k(t) at p
        const int ti = i + kx, tj = j + ky;
        const double s2 = inside(g.N, ti, tj) ? tb[(int64_t)tj * g.P + ti] : 0.0;
        yb[k * tstride + p] += s1;
        yb[(9 + k) * tstride + p] += s2;
    }
}

// ---------------------------------------------------------------- transfers
// From a full fine level to its checkerboard (same array), the mesh axes are the grid axes; from a
// checkerboard to the full grid of both-odd nodes, the diagonals.
__global__ void __launch_bounds__(kNT) k_rb_restrict(RBGeom gf, RBGeom gc, const double *__restrict__ s,
                                                     double *__restrict__ rc, const int *active)
{
    const int v = blockIdx.z;
    if (active && !active[v]) return;
    const int I = blockIdx.x * kBX + threadIdx.x, J = blockIdx.y * kBY + threadIdx.y;
    if (I >= gc.N || J >= gc.N) return;
    const double *sv = s + v * gf.vs;
    double val = 0.0;
    if (rb_has(gc.kind, I, J)) {
        const bool diag = gf.kind == kRBChecker;
        const int fi = diag ? 2 * I + 1 : I, fj = diag ? 2 * J + 1 : J;
        double nb = 0.0;
        for (int q = 0; q < 4; ++q) {
            const int dx = diag ? (q & 1 ? 1 : -1) : (q == 0 ? 1 : q == 1 ? -1 : 0);
            const int dy = diag ? (q & 2 ? 1 : -1) : (q == 2 ? 1 : q == 3 ? -1 : 0);
            const int ii = fi + dx, jj = fj + dy;
            if (inside(gf.N, ii, jj)) nb += sv[(int64_t)jj * gf.P + ii];
        }
        val = 0.5 * sv[(int64_t)fj * gf.P + fi] + 0.125 * nb;
    }
    rc[v * gc.vs + (int64_t)J * gc.P + I] = val;
}

__global__ void __launch_bounds__(kNT) k_rb_prolong(RBGeom gf, RBGeom gc, const double *__restrict__ ec,
                                                    double *__restrict__ e, const int *active)
{
    const int v = blockIdx.z;
    if (active && !active[v]) return;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= gf.N || j >= gf.N || !rb_has(gf.kind, i, j)) return;
    const double *cv = ec + v * gc.vs;
    const int64_t p = v * gf.vs + (int64_t)j * gf.P + i;
    if (gf.kind == kRBFull) {
        if (((i + j) & 1) == 0) {  // a coarse (black) node keeps its value
            e[p] += cv[(int64_t)j * gc.P + i];
            return;
        }
        double acc = 0.0;  // a red node: 1/4 of its black axis neighbours
        if (i + 1 < gf.N) acc += cv[(int64_t)j * gc.P + i + 1];
        if (i > 0) acc += cv[(int64_t)j * gc.P + i - 1];
        if (j + 1 < gf.N) acc += cv[(int64_t)(j + 1) * gc.P + i];
        if (j > 0) acc += cv[(int64_t)(j - 1) * gc.P + i];
        e[p] += 0.25 * acc;
        return;
    }
    if (i & 1) {  // both odd: the coarse node (i-1)/2, (j-1)/2
        e[p] += cv[(int64_t)((j - 1) >> 1) * gc.P + ((i - 1) >> 1)];
        return;
    }
    double acc = 0.0;  // both even: 1/4 of the both-odd diagonal neighbours inside the grid
    for (int q = 0; q < 4; ++q) {
        const int ii = i + (q & 1 ? 1 : -1), jj = j + (q & 2 ? 1 : -1);
        if (inside(gf.N, ii, jj)) acc += cv[(int64_t)((jj - 1) >> 1) * gc.P + ((ii - 1) >> 1)];
    }
    e[p] += 0.25 * acc;
}

// ----------------------------------------------------------------- Galerkin
// One thread per (coarse node, coarse offset d): Ac_d(q) = sum_a R(q, a) sum_c Af_c(a) P(a + off_c, q + d),
// over the restriction's five fine nodes a and the fine footprint c; P(b, q') is 1 at b = q' and 1/4
// where b is a mesh-axis neighbour of q' (coordinates in fine units).
__global__ void __launch_bounds__(kNT) k_rb_galerkin(RBGeom gf, RBOffsets of, const double *__restrict__ Af,
                                                     RBGeom gc, RBOffsets oc, double *__restrict__ Ac)
{
    const int d = blockIdx.z;
    const int I = blockIdx.x * kBX + threadIdx.x, J = blockIdx.y * kBY + threadIdx.y;
    if (I >= gc.N || J >= gc.N) return;
    const int64_t pc = (int64_t)J * gc.P + I;
    double val = 0.0;
    const int I2 = I + oc.dx[d], J2 = J + oc.dy[d];
    if (rb_has(gc.kind, I, J) && inside(gc.N, I2, J2) && rb_has(gc.kind, I2, J2)) {
        const bool diag = gf.kind == kRBChecker;
        const int qi = diag ? 2 * I + 1 : I, qj = diag ? 2 * J + 1 : J;        // q in fine units
        const int ti = diag ? 2 * I2 + 1 : I2, tj = diag ? 2 * J2 + 1 : J2;    // q' in fine units
        for (int a = 0; a < 5; ++a) {
            int ax = 0, ay = 0;
            if (a > 0) {
                const int q = a - 1;
                ax = diag ? (q & 1 ? 1 : -1) : (q == 0 ? 1 : q == 1 ? -1 : 0);
                ay = diag ? (q & 2 ? 1 : -1) : (q == 2 ? 1 : q == 3 ? -1 : 0);
            }
            const int ai = qi + ax, aj = qj + ay;
            if (!inside(gf.N, ai, aj)) continue;
            const double wr = a == 0 ? 0.5 : 0.125;
            const int64_t pa = (int64_t)aj * gf.P + ai;
            double inner = 0.0;
            for (int c = 0; c < of.K; ++c) {
                const int bi = ai + of.dx[c], bj = aj + of.dy[c];
                if (!inside(gf.N, bi, bj)) continue;
                const int dx = bi - ti, dy = bj - tj;
                double wp = 0.0;
                if (dx == 0 && dy == 0)
                    wp = 1.0;
                else if (diag ? (dx == 1 || dx == -1) && (dy == 1 || dy == -1)
                              : (dx == 0 && (dy == 1 || dy == -1)) || (dy == 0 && (dx == 1 || dx == -1)))
                    wp = 0.25;
                if (wp != 0.0) inner += Af[c * gf.vs + pa] * wp;
            }
            val += wr * inner;
        }
    }
    Ac[d * gc.vs + pc] = val;
}

// -------------------------------------------------------------- last level
__global__ void __launch_bounds__(64) k_rb_coarse_factor(RBGeom g, RBOffsets o, const double *__restrict__ A, int m,
                                                         double *__restrict__ Ainv, int *flag)
{
    __shared__ double L[kRBMaxCoarse][kRBMaxCoarse + 1];
    __shared__ double X[kRBMaxCoarse][kRBMaxCoarse + 1];
    __shared__ int idx[kRBMaxCoarse * 2];  // point k -> (i, j)
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t == 0) {
        bad = 0;
        int k = 0;
        for (int j = 0; j < g.N; ++j)
            for (int i = 0; i < g.N; ++i)
                if (rb_has(g.kind, i, j) && k < kRBMaxCoarse) {
                    idx[2 * k] = i;
                    idx[2 * k + 1] = j;
                    ++k;
                }
    }
    for (int q = t; q < m * kRBMaxCoarse; q += 64) L[q / kRBMaxCoarse][q % kRBMaxCoarse] = 0.0;
    __syncthreads();
    for (int r = t; r < m; r += 64) {  // row r: the point's footprint, columns by point index
        const int i = idx[2 * r], j = idx[2 * r + 1];
        for (int c = 0; c < o.K; ++c) {
            const int ii = i + o.dx[c], jj = j + o.dy[c];
            if (!inside(g.N, ii, jj) || !rb_has(g.kind, ii, jj)) continue;
            int col = -1;
            for (int q = 0; q < m; ++q)
                if (idx[2 * q] == ii && idx[2 * q + 1] == jj) col = q;
            if (col >= 0) L[r][col] = A[c * g.vs + (int64_t)j * g.P + i];
        }
    }
    __syncthreads();
    for (int k = 0; k < m; ++k) {
        if (t == 0) {
            double d = L[k][k];
            for (int q = 0; q < k; ++q) d -= L[k][q] * L[k][q];
            if (!(d > 0.0)) {
                bad = 1;
                d = 1.0;
            }
            L[k][k] = sqrt(d);
        }
        __syncthreads();
        for (int i = k + 1 + t; i < m; i += 64) {
            double s = L[i][k];
            for (int q = 0; q < k; ++q) s -= L[i][q] * L[k][q];
            L[i][k] = s / L[k][k];
        }
        __syncthreads();
    }
    for (int c = t; c < m; c += 64) {
        for (int i = 0; i < m; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int q = 0; q < i; ++q) s -= L[i][q] * X[q][c];
            X[i][c] = s / L[i][i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double s = X[i][c];
            for (int q = i + 1; q < m; ++q) s -= L[q][i] * X[q][c];
            X[i][c] = s / L[i][i];
        }
    }
    __syncthreads();
    for (int q = t; q < m * m; q += 64) Ainv[q] = X[q / m][q % m];
    if (t == 0 && bad) atomicOr(flag, 8);
}

// One block per vector: the point values in LDS, one output row per thread.
__global__ void __launch_bounds__(64) k_rb_coarse_apply(RBGeom g, int m, const double *__restrict__ Ainv,
                                                        const double *__restrict__ r, double *__restrict__ e,
                                                        const int *active)
{
    __shared__ double rv[kRBMaxCoarse];
    __shared__ int pos[kRBMaxCoarse];
    const int v = blockIdx.x;
    if (active && !active[v]) return;
    const int t = threadIdx.x;
    if (t == 0) {
        int k = 0;
        for (int j = 0; j < g.N; ++j)
            for (int i = 0; i < g.N; ++i)
                if (rb_has(g.kind, i, j) && k < kRBMaxCoarse) pos[k++] = j * g.P + i;
    }
    __syncthreads();
    const double *rvv = r + v * g.vs;
    for (int q = t; q < m; q += 64) rv[q] = rvv[pos[q]];
    __syncthreads();
    double *ev = e + v * g.vs;
    for (int q = t; q < g.N * g.P; q += 64) ev[q] = 0.0;
    __syncthreads();
    for (int q = t; q < m; q += 64) {
        double s = 0.0;
        for (int c = 0; c < m; ++c) s += Ainv[q * m + c] * rv[c];
        ev[pos[q]] = s;
    }
}

// Checks a level-0 nine-point field: centre positive (flag |= 2), entries coupling off the grid zero
// (flag |= 1).
__global__ void __launch_bounds__(kNT) k_rb_validate(RBGeom g, const double *__restrict__ A, int *flag)
{
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.N || j >= g.N) return;
    const int64_t p = (int64_t)j * g.P + i;
    int bad = 0;
    for (int c = 0; c < 9; ++c) {
        const double a = A[c * g.vs + p];
        if (c == 4) {
            if (!(a > 0.0)) bad |= 2;
        } else if (!inside(g.N, i + c % 3 - 1, j + c / 3 - 1) && a != 0.0) {
            bad |= 1;
        } else if (!isfinite(a)) {
            bad |= 1;
        }
    }
    if (bad) atomicOr(flag, bad);
}

// ------------------------------------------------------------------ vectors
__global__ void __launch_bounds__(kNT) k_rb_copy_in(RBGeom g, const double *__restrict__ src, double *__restrict__ dst,
                                                    int64_t dstride)
{
    const int v = blockIdx.z;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (j >= g.N || i > g.N) return;
    const int64_t p = v * dstride + (int64_t)j * g.P + i;
    dst[p] = (i < g.N && rb_has(g.kind, i, j)) ? src[(int64_t)v * g.N * g.N + (int64_t)j * g.N + i] : 0.0;
}

__global__ void __launch_bounds__(kNT) k_rb_copy_out(RBGeom g, const double *__restrict__ src,
                                                     double *__restrict__ dst)
{
    const int v = blockIdx.z;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.N || j >= g.N) return;
    dst[(int64_t)v * g.N * g.N + (int64_t)j * g.N + i] = src[v * g.vs + (int64_t)j * g.P + i];
}

__global__ void __launch_bounds__(kNT) k_rb_axpy(RBGeom g, const double *__restrict__ x, double *__restrict__ y,
                                                 const int *active)
{
    const int v = blockIdx.z;
    if (active && !active[v]) return;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    if (i >= g.N || j >= g.N) return;
    const int64_t p = v * g.vs + (int64_t)j * g.P + i;
    y[p] += x[p];
}

// Per instance b: block sums of ||u_b - u*_b||^2 and <tangent_j, u_b - u*_b>.
__global__ void __launch_bounds__(kNT) k_rb_alpha_dots(RBGeom g, const double *__restrict__ u, int64_t inst_stride,
                                                       const double *__restrict__ ustar, double *__restrict__ partial,
                                                       int nb, const int *want)
{
    __shared__ double red[kNT / 64];
    const int b = blockIdx.z;
    if (!want[b]) return;
    const int i = blockIdx.x * kBX + threadIdx.x, j = blockIdx.y * kBY + threadIdx.y;
    const bool in = i < g.N && j < g.N;
    const int64_t p = (int64_t)j * g.P + i;
    const double *ub = u + b * inst_stride;
    const double d = in ? ub[p] - ustar[b * g.vs + p] : 0.0;
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    for (int q = 0; q <= kRBWeights; ++q) {
        const double val = q == 0 ? d * d : (in ? ub[q * g.vs + p] * d : 0.0);
        const double s = block_sum<kNT>(val, red);
        if (threadIdx.x == 0 && threadIdx.y == 0) partial[((int64_t)b * (kRBWeights + 1) + q) * nb + blk] = s;
    }
}

__global__ void __launch_bounds__(256) k_rb_check(const double *__restrict__ rr, RBState *state, int *act, double tol,
                                                  int maxit, double *history, int hist_stride, int init, int nvec)
{
    const int v = blockIdx.x * 256 + threadIdx.x;
    if (v >= nvec) return;
    RBState &s = state[v];
    if (init) {  // rr = ||f||^2 (u = 0): set up; the first check comes with the first residual
        s.fnorm = sqrt(rr[v]);
        s.iters = 0;
        s.status = 0;
        s.relres = 1.0;
        s.active = 1;
        act[v] = 1;
        return;
    }
    if (!s.active) {
        act[v] = 0;
        return;
    }
    const double rel = s.fnorm > 0.0 ? sqrt(rr[v]) / s.fnorm : 0.0;
    s.relres = rel;
    if (history) history[(int64_t)v * hist_stride + s.iters] = rel;
    if (rel <= tol) {
        s.active = 0;
    } else if (!isfinite(rel) || rel > 1e3) {
        s.active = 0;
        s.status = -4;
    } else if (s.iters >= maxit) {
        s.active = 0;
        s.status = 1;
    } else {
        s.iters += 1;
    }
    act[v] = s.active;
}

__global__ void k_rb_alpha_final(const double *__restrict__ sums, int B, double *__restrict__ out)
{
    const int q = threadIdx.x;  // 0: the loss and per-instance norms; 1 + j: gradient j
    if (q > kRBWeights) return;
    double acc = 0.0;
    for (int b = 0; b < B; ++b) {
        const double L = sqrt(sums[b * (kRBWeights + 1)]);
        if (q == 0) {
            out[1 + b] = L;
            acc += L;
        } else if (L > 0.0) {
            acc += sums[b * (kRBWeights + 1) + q] / L;
        }
    }
    if (q == 0)
        out[0] = acc / B;
    else
        out[1 + B + q - 1] = acc / B;
}

__global__ void k_rb_adam(int n, double *w, double *m, double *v, const double *g, int t, double lr, double b1,
                          double b2, double eps)
{
    const int i = threadIdx.x;
    if (i >= n) return;
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    const double mh = m[i] / (1.0 - pow(b1, (double)t)), vh = v[i] / (1.0 - pow(b2, (double)t));
    w[i] -= lr * mh / (sqrt(vh) + eps);
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_rb_residual(const RBGeom &g, const RBOffsets &o, const double *A, const double *b, const double *x,
                        double *y, double sign, int nvec, const int *active, hipStream_t st)
{
    k_rb_residual<<<point_grid(g.N, nvec), dim3(kBX, kBY), 0, st>>>(g, o, A, b, x, y, sign, active);
}

int rb_norm_blocks(int N) { return ((N + kBX - 1) / kBX) * ((N + kBY - 1) / kBY); }

void launch_rb_outer(const RBGeom &g, const RBOffsets &o, const double *A, const double *f, const double *u,
                     double *r, double *partial, int nvec, const int *active, hipStream_t st)
{
    k_rb_outer<<<point_grid(g.N, nvec), dim3(kBX, kBY), 0, st>>>(g, o, A, f, u, r, partial, rb_norm_blocks(g.N),
                                                                 active);
}

void launch_rb_sum(const double *partial, int nb, double *out, int nvec, hipStream_t st)
{
    k_rb_sum<<<nvec, 256, 0, st>>>(partial, nb, out);
}

void launch_rb_jacobi(const RBGeom &g, const double *Acentre, double omega, const double *s, double *e,
                      bool accumulate, int nvec, const int *active, hipStream_t st)
{
    k_rb_jacobi<<<point_grid(g.N, nvec), dim3(kBX, kBY), 0, st>>>(g, Acentre, omega, s, e, accumulate ? 1 : 0,
                                                                  active);
}

void launch_rb_conv(const RBGeom &g, const double *w, const double *x, double *y, bool mask_in, bool mask_out,
                    bool accumulate, int nvec, const int *active, hipStream_t st)
{
    k_rb_conv<<<point_grid(g.N, nvec), dim3(kBX, kBY), 0, st>>>(g, w, x, y, mask_in ? 1 : 0, mask_out ? 1 : 0,
                                                                accumulate ? 1 : 0, active);
}

void launch_rb_dH(const RBGeom &g, const double *w, const double *x, int64_t xstride, const double *t,
                  int64_t tstride_t, double *dy, int64_t ystride, int64_t tstride, int ninst, const int *active,
                  int active_stride, hipStream_t st)
{
    k_rb_dH<<<point_grid(g.N, ninst), dim3(kBX, kBY), 0, st>>>(g, w, x, xstride, t, tstride_t, dy, ystride, tstride,
                                                               active, active_stride);
}

void launch_rb_restrict(const RBGeom &gf, const RBGeom &gc, const double *s, double *rc, int nvec,
                        const int *active, hipStream_t st)
{
    k_rb_restrict<<<point_grid(gc.N, nvec), dim3(kBX, kBY), 0, st>>>(gf, gc, s, rc, active);
}

void launch_rb_prolong(const RBGeom &gf, const RBGeom &gc, const double *ec, double *e, int nvec, const int *active,
                       hipStream_t st)
{
    k_rb_prolong<<<point_grid(gf.N, nvec), dim3(kBX, kBY), 0, st>>>(gf, gc, ec, e, active);
}

void launch_rb_galerkin(const RBGeom &gf, const RBOffsets &of, const double *Af, const RBGeom &gc,
                        const RBOffsets &oc, double *Ac, hipStream_t st)
{
    k_rb_galerkin<<<point_grid(gc.N, oc.K), dim3(kBX, kBY), 0, st>>>(gf, of, Af, gc, oc, Ac);
}

void launch_rb_coarse_factor(const RBGeom &g, const RBOffsets &o, const double *A, int m, double *Ainv, int *flag,
                             hipStream_t st)
{
    k_rb_coarse_factor<<<1, 64, 0, st>>>(g, o, A, m, Ainv, flag);
}

void launch_rb_coarse_apply(const RBGeom &g, int m, const double *Ainv, const double *r, double *e, int nvec,
                            const int *active, hipStream_t st)
{
    k_rb_coarse_apply<<<nvec, 64, 0, st>>>(g, m, Ainv, r, e, active);
}

void launch_rb_validate(const RBGeom &g, const double *A, int *flag, hipStream_t st)
{
    k_rb_validate<<<point_grid(g.N, 1), dim3(kBX, kBY), 0, st>>>(g, A, flag);
}

void launch_rb_copy_in(const RBGeom &g, const double *src, double *dst, int64_t dstride, int nvec, hipStream_t st)
{
    k_rb_copy_in<<<point_grid(g.N + 1, nvec), dim3(kBX, kBY), 0, st>>>(g, src, dst, dstride);
}

void launch_rb_copy_out(const RBGeom &g, const double *src, double *dst, int nvec, hipStream_t st)
{
    k_rb_copy_out<<<point_grid(g.N, nvec), dim3(kBX, kBY), 0, st>>>(g, src, dst);
}

void launch_rb_axpy(const RBGeom &g, const double *x, double *y, int nvec, const int *active, hipStream_t st)
{
    k_rb_axpy<<<point_grid(g.N, nvec), dim3(kBX, kBY), 0, st>>>(g, x, y, active);
}

void launch_rb_alpha_dots(const RBGeom &g, const double *u, int64_t inst_stride, const double *ustar,
                          double *partial, int ninst, const int *want, hipStream_t st)
{
    k_rb_alpha_dots<<<point_grid(g.N, ninst), dim3(kBX, kBY), 0, st>>>(g, u, inst_stride, ustar, partial,
                                                                       rb_norm_blocks(g.N), want);
}

void launch_rb_check(const double *rr, RBState *state, int *act, double tol, int maxit, double *history,
                     int hist_stride, int init, int nvec, hipStream_t st)
{
    k_rb_check<<<(nvec + 255) / 256, 256, 0, st>>>(rr, state, act, tol, maxit, history, hist_stride, init, nvec);
}

void launch_rb_alpha_final(const double *sums, int B, double *out, hipStream_t st)
{
    k_rb_alpha_final<<<1, 64, 0, st>>>(sums, B, out);
}

void launch_rb_adam(int n, double *w, double *m, double *v, const double *g, int t, double lr, double b1, double b2,
                    double eps, hipStream_t st)
{
    k_rb_adam<<<1, 64, 0, st>>>(n, w, m, v, g, t, lr, b1, b2, eps);
}

}  // namespace mg
