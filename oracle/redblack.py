"""Red-black coarsening (section 6.1) with the two-layer convolution smoother
H = f2(f1) of section 6 ("Neural networks", red-black coarsening) and its
Algorithm 2 loss, FP64 numpy / scipy.sparse.

TEST INFRASTRUCTURE ONLY (oracle).  Nothing in the product library imports
it; it shares no code with the GPU path.

Grids.  Level 0 is the n x n interior grid (n = 2^k - 1, nodes (i, j),
0 <= i, j < n, zero Dirichlet values).  Coarsening alternates:
  * a full N x N level coarsens to its checkerboard: the nodes with i + j
    even ("black"; the red nodes, i + j odd, are the fine-only points).  The
    paper's figure: a semi-coarsening along the 45-degree direction;
  * a checkerboard level coarsens, on its 45-degree rotated mesh, to the full
    grid of the nodes with i and j both odd: the full level of size
    (N - 1)/2 whose node I sits on fine node 2I + 1 (the grid one full
    coarsening step gives).  Its fine-only points are those with i and j
    both even.
As the paper does for its networks, the irregular (checkerboard) levels are
stored padded: every level's vectors are N x N arrays, zero on the points
the level does not have.  Operators are sparse matrices on the N^2 padded
unknowns (row j*N + i), with zero rows and columns on those points.

Transfers.  The paper's stencils: restriction (1/8)[0 1 0; 1 4 1; 0 1 0]
and interpolation (1/4)][0 1 0; 1 4 1; 0 1 0][, acting along the level's own
mesh axes: the grid axes on a full level, the diagonals on a checkerboard
(the rotated mesh).  A coarse point keeps its value (weight 1) and gives 1/4
to each fine-only neighbour; a fine-only point's interpolated value is 1/4
of the sum over its coarse neighbours that lie inside the domain.  The
restriction takes half of the coarse point's own residual and 1/8 of each
fine-only neighbour's.

Coarse operators: Galerkin, A_{l+1} = R_l A_l P_l (the same coarse
correction as the P^T A P form: R = P^T/2 here).  The last level is solved
directly (dense, on its own points).  The V-cycle is Algorithm 1 in
correction form with nu1 / nu2 sweeps.

Smoothers.  Damped Jacobi (omega / diag on the level's points) or the
two-layer stack H x = M f2(f1(M x)) with f1, f2 single-channel 3x3
cross-correlations on the padded N x N array (zero padding) and M the
level's point mask: the CNN sees the padded grid, its input and output are
the level's vector.  Weights: 18 values [2][3][3] (layer, ky, kx), tap
(ky, kx) multiplying x at (j + ky - 1, i + kx - 1).

The Algorithm 2 loss ||Phi(u0, f, k) - u*||_2 of a trained level uses one
cycle of the next coarser levels as Psi_c, the steps r = f - A u, a = H r,
s = r - A a, t = a + P Psi_c(R s), q = r - A t, u += t + H q, and its gradient
with respect to the 18 weights is taken in forward mode (each state carries
its derivative with respect to every weight).

Pinned in tests/test_oracle_redblack.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

OMEGA = 2.0 / 3.0
NWEIGHTS = 18

FULL, CHECKER = "full", "checker"

_AXES = ((1, 0), (-1, 0), (0, 1), (0, -1))
_DIAGONALS = ((1, 1), (-1, 1), (1, -1), (-1, -1))


def point_mask(N: int, kind: str) -> np.ndarray:
    """The points a level has on its N x N array (bool [N, N], [j, i])."""
    j, i = np.mgrid[0:N, 0:N]
    if kind == FULL:
        return np.ones((N, N), dtype=bool)
    return (i + j) % 2 == 0


def level_shapes(n: int, nlevels: int):
    """[(N, kind)] of levels 0 .. nlevels - 1 from an n x n full grid."""
    out = [(n, FULL)]
    while len(out) < nlevels:
        N, kind = out[-1]
        if kind == FULL:
            if N < 3:
                raise ValueError("grid too small for another red-black level")
            out.append((N, CHECKER))
        else:
            out.append(((N - 1) // 2, FULL))
    return out


def _coarse_points(N: int, kind: str):
    """Coarse points of a fine level as (fine i, fine j, coarse index) and the coarse array size."""
    if kind == FULL:  # to the checkerboard of the same array
        pts = [(i, j, j * N + i) for j in range(N) for i in range(N) if (i + j) % 2 == 0]
        return pts, N, _AXES
    Nc = (N - 1) // 2
    pts = [(2 * I + 1, 2 * J + 1, J * Nc + I) for J in range(Nc) for I in range(Nc)]
    return pts, Nc, _DIAGONALS


def prolongation(N: int, kind: str) -> sp.csr_matrix:
    """P from the coarse level of (N, kind) to it: [N^2, Nc^2]; a coarse point
    gives 1 to itself and 1/4 to each fine-only neighbour along the mesh axes."""
    pts, Nc, nbrs = _coarse_points(N, kind)
    rows, cols, vals = [], [], []
    for fi, fj, q in pts:
        rows.append(fj * N + fi)
        cols.append(q)
        vals.append(1.0)
        for dx, dy in nbrs:
            i, j = fi + dx, fj + dy
            if 0 <= i < N and 0 <= j < N:
                rows.append(j * N + i)
                cols.append(q)
                vals.append(0.25)
    return sp.csr_matrix((vals, (rows, cols)), shape=(N * N, Nc * Nc))


def restriction(N: int, kind: str) -> sp.csr_matrix:
    """R to the coarse level of (N, kind): [Nc^2, N^2], the stencil
    (1/8)[0 1 0; 1 4 1; 0 1 0] along the mesh axes (neighbours off the grid
    carry the zero boundary value)."""
    pts, Nc, nbrs = _coarse_points(N, kind)
    rows, cols, vals = [], [], []
    for fi, fj, q in pts:
        rows.append(q)
        cols.append(fj * N + fi)
        vals.append(4.0 / 8.0)
        for dx, dy in nbrs:
            i, j = fi + dx, fj + dy
            if 0 <= i < N and 0 <= j < N:
                rows.append(q)
                cols.append(j * N + i)
                vals.append(1.0 / 8.0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(Nc * Nc, N * N))


def operator_matrix(A) -> sp.csr_matrix:
    """The sparse matrix of a nine-point stencil field A [9, n, n] (channel
    c = 3(dy+1) + (dx+1) couples node (i, j) to (i + dx, j + dy))."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    rows, cols, vals = [], [], []
    j, i = np.mgrid[0:n, 0:n]
    for c in range(9):
        dy, dx = c // 3 - 1, c % 3 - 1
        ii, jj = i + dx, j + dy
        ok = (ii >= 0) & (ii < n) & (jj >= 0) & (jj < n) & (A[c] != 0.0)
        rows.append((j * n + i)[ok])
        cols.append((jj * n + ii)[ok])
        vals.append(A[c][ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n * n, n * n))


def conv3(x, k) -> np.ndarray:
    """y[.., j, i] = sum_{ky,kx} k[ky, kx] x[.., j + ky - 1, i + kx - 1], zero off the array."""
    x = np.asarray(x, dtype=np.float64)
    n0, n1 = x.shape[-2:]
    xp = np.zeros(x.shape[:-2] + (n0 + 2, n1 + 2))
    xp[..., 1:n0 + 1, 1:n1 + 1] = x
    y = np.zeros_like(x)
    for ky in range(3):
        for kx in range(3):
            y += k[ky, kx] * xp[..., ky:ky + n0, kx:kx + n1]
    return y


def _weights(phi) -> np.ndarray:
    w = np.asarray(phi, dtype=np.float64)
    if w.size != NWEIGHTS:
        raise ValueError("a red-black stack has 2 x 3 x 3 weights")
    return w.reshape(2, 3, 3)


def smoother_apply(phi, x, mask) -> np.ndarray:
    """H x = M f2(f1(M x)) (any leading batch dimensions)."""
    w = _weights(phi)
    return conv3(conv3(np.asarray(x) * mask, w[0]), w[1]) * mask


def smoother_derivative(phi, x, mask, j: int) -> np.ndarray:
    """d(H x)/d weight j: the stack with layer j // 9 replaced by the unit kernel at tap j % 9."""
    w = _weights(phi).copy()
    unit = np.zeros((3, 3))
    unit[(j % 9) // 3, j % 3] = 1.0
    w[j // 9] = unit
    return smoother_apply(w, x, mask)


def jacobi_stack(a_centre: float, omega: float = OMEGA) -> np.ndarray:
    """f1 = (omega / a_C) at the centre tap, f2 = the identity: damped Jacobi
    wherever the level's diagonal equals a_centre."""
    w = np.zeros((2, 3, 3))
    w[0, 1, 1] = omega / a_centre
    w[1, 1, 1] = 1.0
    return w


class RBHierarchy:
    """Red-black Galerkin levels of the nine-point operator A0 ([9, n, n]),
    nlevels in all (the last solved directly), each level above the last
    with damped Jacobi or a two-layer stack."""

    def __init__(self, A0, nlevels: int):
        A0 = np.asarray(A0, dtype=np.float64)
        self.shapes = level_shapes(A0.shape[1], nlevels)
        self.num_levels = nlevels
        self.masks = [point_mask(N, k) for N, k in self.shapes]
        self.P = [prolongation(N, k) for N, k in self.shapes[:-1]]
        self.R = [restriction(N, k) for N, k in self.shapes[:-1]]
        self.A = [operator_matrix(A0)]
        for l in range(nlevels - 1):
            self.A.append((self.R[l] @ self.A[l] @ self.P[l]).tocsr())
        N, _ = self.shapes[-1]
        pts = np.flatnonzero(self.masks[-1].reshape(-1))
        self._coarse_pts = pts
        self._coarse_dense = self.A[-1].toarray()[np.ix_(pts, pts)]
        self.smoothers = [None] * (nlevels - 1)

    def level_n(self, level: int) -> int:
        return self.shapes[level][0]

    def diag(self, level: int) -> np.ndarray:
        N = self.level_n(level)
        return self.A[level].diagonal().reshape(N, N)

    def set_smoother(self, level: int, phi=None) -> None:
        if not 0 <= level < self.num_levels - 1:
            raise ValueError("bad level")
        self.smoothers[level] = None if phi is None else _weights(phi).copy()

    def matvec(self, level: int, x) -> np.ndarray:
        N = self.level_n(level)
        return (self.A[level] @ np.asarray(x, dtype=np.float64).reshape(-1)).reshape(N, N)

    def restrict(self, level: int, x) -> np.ndarray:
        N = self.level_n(level + 1)
        return (self.R[level] @ np.asarray(x).reshape(-1)).reshape(N, N)

    def prolong(self, level: int, xc) -> np.ndarray:
        N = self.level_n(level)
        return (self.P[level] @ np.asarray(xc).reshape(-1)).reshape(N, N)

    def coarse_solve(self, r) -> np.ndarray:
        N = self.level_n(self.num_levels - 1)
        e = np.zeros(N * N)
        e[self._coarse_pts] = np.linalg.solve(self._coarse_dense, np.asarray(r).reshape(-1)[self._coarse_pts])
        return e.reshape(N, N)

    def apply_smoother(self, level: int, x) -> np.ndarray:
        """H x on the level (damped Jacobi where no stack is set)."""
        mask = self.masks[level]
        if self.smoothers[level] is None:
            d = self.diag(level)
            return np.where(mask, OMEGA * np.asarray(x) / np.where(mask, d, 1.0), 0.0)
        return smoother_apply(self.smoothers[level], x, mask)

    def vcycle(self, r, level: int = 0, nu1: int = 1, nu2: int = 1) -> np.ndarray:
        """e = V(r) from level (Algorithm 1, correction form)."""
        r = np.asarray(r, dtype=np.float64)
        if level == self.num_levels - 1:
            return self.coarse_solve(r)
        e = np.zeros_like(r)
        for _ in range(nu1):
            e = e + self.apply_smoother(level, r - self.matvec(level, e))
        s = r - self.matvec(level, e)
        e = e + self.prolong(level, self.vcycle(self.restrict(level, s), level + 1, nu1, nu2))
        for _ in range(nu2):
            e = e + self.apply_smoother(level, r - self.matvec(level, e))
        return e

    def solve(self, f, tol: float, maxit: int, nu1: int = 1, nu2: int = 1, level: int = 0):
        """u = 0; while ||f - A u|| > tol ||f|| and k < maxit: u += V(f - A u).
        Returns (u, iterations, history, converged)."""
        f = np.asarray(f, dtype=np.float64)
        u = np.zeros_like(f)
        nf = np.linalg.norm(f)
        hist = []
        k = 0
        while True:
            r = f - self.matvec(level, u)
            hist.append(np.linalg.norm(r) / nf)
            if hist[-1] <= tol:
                return u, k, np.array(hist), True
            if k == maxit:
                return u, k, np.array(hist), False
            u = u + self.vcycle(r, level, nu1, nu2)
            k += 1

    # ------------------------------------------------------------ Algorithm 2
    def _coarse_cycle(self, level: int, x) -> np.ndarray:
        """P Psi_c(R x): one cycle of the levels below `level` (V(1,1))."""
        return self.prolong(level, self.vcycle(self.restrict(level, x), level + 1, 1, 1))

    def alpha_forward(self, level: int, phi, f, u0, k: int) -> np.ndarray:
        """u_k of Algorithm 2's recursion on `level` with the stack phi there."""
        mask = self.masks[level]
        u = np.array(u0, dtype=np.float64)
        for _ in range(k):
            r = f - self.matvec(level, u)
            a = smoother_apply(phi, r, mask)
            s = r - self.matvec(level, a)
            t = a + self._coarse_cycle(level, s)
            q = r - self.matvec(level, t)
            u = u + t + smoother_apply(phi, q, mask)
        return u

    def alpha_loss_and_grad(self, level: int, phi, f, u0, u_star, k: int):
        """||u_k - u*||_2 and its gradient with respect to the 18 weights (forward mode)."""
        mask = self.masks[level]
        w = _weights(phi)
        N = self.level_n(level)
        u = np.array(u0, dtype=np.float64)
        du = np.zeros((NWEIGHTS, N, N))

        def H_and_tangent(x, dx):
            y = smoother_apply(w, x, mask)
            dy = smoother_apply(w, dx, mask)
            for j in range(NWEIGHTS):
                dy[j] += smoother_derivative(w, x, mask, j)
            return y, dy

        def A_batch(X):
            return np.stack([self.matvec(level, x) for x in X])

        def coarse_batch(X):
            return np.stack([self._coarse_cycle(level, x) for x in X])

        for _ in range(k):
            r = f - self.matvec(level, u)
            dr = -A_batch(du)
            a, da = H_and_tangent(r, dr)
            s = r - self.matvec(level, a)
            ds = dr - A_batch(da)
            t = a + self._coarse_cycle(level, s)
            dt = da + coarse_batch(ds)
            q = r - self.matvec(level, t)
            dq = dr - A_batch(dt)
            hq, dhq = H_and_tangent(q, dq)
            u = u + t + hq
            du = du + dt + dhq
        d = u - np.asarray(u_star, dtype=np.float64)
        L = float(np.linalg.norm(d))
        g = np.einsum("jab,ab->j", du, d) / L if L > 0 else np.zeros(NWEIGHTS)
        return L, g

    def batch_loss_and_grad(self, level: int, phi, f_list, u0_list, ustar_list, ks):
        """Mean loss over a batch of instances of the level's problem and its gradient."""
        B = len(ks)
        total, grad = 0.0, np.zeros(NWEIGHTS)
        for f, u0, us, k in zip(f_list, u0_list, ustar_list, ks):
            L, g = self.alpha_loss_and_grad(level, phi, f, u0, us, k)
            total += L / B
            grad += g / B
        return total, grad
