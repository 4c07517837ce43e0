"""The constant-coefficient alpha-CNN smoother of section 5 (full coarsening)
and its Algorithm 2 loss, FP64 numpy.

TEST INFRASTRUCTURE ONLY (oracle).  On each level the smoother is a stack of
six 3x3 convolutions (section 5, "Neural networks"):

    H x = f5(f4(f3(f2(f1(x))))) + f6(x),

each f_i a single-channel 3x3 cross-correlation with kernel phi_i and zero
("same") padding: the values of every intermediate grid outside the n x n
interior are zero.  Weights are an array [6][3][3] (layer, ky, kx), layer
0..4 = f1..f5 and layer 5 = f6; tap (ky, kx) multiplies x at (j + ky - 1,
i + kx - 1).  The stack is linear, so the multigrid iteration stays linear.

The V(1,1) cycle with these smoothers is written here in numpy on top of the
oracle's stencils, matvec and transfers (Algorithm 1 in correction form, a
dense solve on the coarsest level); a level given None takes damped Jacobi.
A level may post-smooth with a different stack; with H^T after the coarse
correction ("symmetric") the cycle's error propagation is self-adjoint in the
A inner product.

The Algorithm 2 loss ||Phi(u0, f, k) - u*||_2 of the trained level uses the
same forward steps as the per-point form (r = f - A u, a = H r, s = r - A a,
t = a + P Psi_c(R s), q = r - A t, u += t + H q).  Its gradient with respect
to the 54 weights is taken here in forward mode: every state carries its
derivative with respect to each weight alongside (the derivative of H x with
respect to weight (layer L, tap k) is the stack with layer L replaced by the
unit kernel at k).  The library computes the same gradient by the adjoint
pass; the two share nothing but the definition.

Pinned in tests/test_oracle_stack.py.
"""
from __future__ import annotations

import numpy as np

from . import OMEGA, Hierarchy, matvec, prolong_add, restrict_fw, smooth_jacobi, stencil_to_dense

NLAYERS = 6
NWEIGHTS = 54


def _weights(phi) -> np.ndarray:
    w = np.asarray(phi, dtype=np.float64)
    if w.size != NWEIGHTS:
        raise ValueError("a stack has 6 x 3 x 3 weights")
    return w.reshape(NLAYERS, 3, 3)


def conv3(x, k) -> np.ndarray:
    """y[.., j, i] = sum_{ky,kx} k[ky, kx] x[.., j + ky - 1, i + kx - 1], zero off the grid."""
    x = np.asarray(x, dtype=np.float64)
    n0, n1 = x.shape[-2:]
    xp = np.zeros(x.shape[:-2] + (n0 + 2, n1 + 2))
    xp[..., 1:n0 + 1, 1:n1 + 1] = x
    y = np.zeros_like(x)
    for ky in range(3):
        for kx in range(3):
            y += k[ky, kx] * xp[..., ky:ky + n0, kx:kx + n1]
    return y


def stack_apply(phi, x) -> np.ndarray:
    """H x for the stack phi (any leading batch dimensions)."""
    w = _weights(phi)
    z = np.asarray(x, dtype=np.float64)
    for layer in range(5):
        z = conv3(z, w[layer])
    return z + conv3(x, w[5])


def stack_transpose(phi) -> np.ndarray:
    """The stack of H^T: the transpose of a zero-padded correlation is the
    correlation with the kernel turned by 180 degrees, and the composition
    reverses, so H^T = f1^T(f2^T(..f5^T)) + f6^T."""
    w = _weights(phi)
    t = np.empty_like(w)
    for layer in range(5):
        t[layer] = w[4 - layer, ::-1, ::-1]
    t[5] = w[5, ::-1, ::-1]
    return t


def stack_jacobi(a_centre: float, omega: float = OMEGA) -> np.ndarray:
    """The stack equal to damped Jacobi on a constant-coefficient operator:
    f1..f5 zero, f6 = (omega / a_C) at the centre tap."""
    w = np.zeros((NLAYERS, 3, 3))
    w[5, 1, 1] = omega / a_centre
    return w


def stack_derivative(phi, x, layer: int, tap: int) -> np.ndarray:
    """d(H x)/d phi[layer][tap]: the stack with that layer's kernel replaced
    by the unit kernel at the tap (layer 5: the unit kernel alone)."""
    w = _weights(phi)
    unit = np.zeros((3, 3))
    unit[tap // 3, tap % 3] = 1.0
    if layer == 5:
        return conv3(x, unit)
    z = np.asarray(x, dtype=np.float64)
    for q in range(5):
        z = conv3(z, unit if q == layer else w[q])
    return z


class StackHierarchy:
    """Galerkin levels of A0 (from the oracle's hierarchy) with one stack
    smoother per level above the coarsest; V(1,1) cycles in numpy."""

    def __init__(self, A0, coarsest_n: int = 7):
        h = Hierarchy(A0, coarsest_n)
        self.stencils = [h.stencil(l) for l in range(h.num_levels)]
        self.num_levels = len(self.stencils)
        self.smoothers = [None] * (self.num_levels - 1)
        self.post = [None] * (self.num_levels - 1)
        self._coarse = stencil_to_dense(self.stencils[-1])

    def set_stack(self, level: int, phi, post=None) -> None:
        """The level's stack before the coarse correction (phi) and after it
        (post; default phi)."""
        if not 0 <= level < self.num_levels - 1:
            raise ValueError("bad level")
        self.smoothers[level] = None if phi is None else _weights(phi).copy()
        self.post[level] = None if phi is None else _weights(phi if post is None else post).copy()

    def _smooth(self, level: int, r, e, after: bool = False):
        """e + H (r - A e) (damped Jacobi where no stack is set)."""
        A = self.stencils[level]
        if self.smoothers[level] is None:
            return smooth_jacobi(A, r, e)
        w = self.post[level] if after else self.smoothers[level]
        return e + stack_apply(w, r - matvec(A, e))

    def vcycle(self, r, level: int = 0, nu1: int = 1, nu2: int = 1) -> np.ndarray:
        """e = V(r) from level (Algorithm 1, correction form, nu1 sweeps before
        and nu2 after the coarse correction)."""
        r = np.asarray(r, dtype=np.float64)
        if level == self.num_levels - 1:
            m = r.shape[0]
            return np.linalg.solve(self._coarse, r.reshape(-1)).reshape(m, m)
        A = self.stencils[level]
        e = np.zeros_like(r)
        for _ in range(nu1):
            e = self._smooth(level, r, e)
        s = r - matvec(A, e)
        e = prolong_add(self.vcycle(restrict_fw(s), level + 1, nu1, nu2), e)
        for _ in range(nu2):
            e = self._smooth(level, r, e, after=True)
        return e

    def solve(self, f, tol: float, maxit: int):
        """u = 0; while ||f - A u|| > tol ||f|| and k < maxit: u += V(f - A u).
        Returns (u, iterations, history, converged)."""
        f = np.asarray(f, dtype=np.float64)
        A = self.stencils[0]
        u = np.zeros_like(f)
        nf = np.linalg.norm(f)
        hist = []
        k = 0
        while True:
            r = f - matvec(A, u)
            hist.append(np.linalg.norm(r) / nf)
            if hist[-1] <= tol:
                return u, k, np.array(hist), True
            if k == maxit:
                return u, k, np.array(hist), False
            u = u + self.vcycle(r)
            k += 1


def _coarse_cycle(hc: StackHierarchy, x):
    """P Psi_c(R x), Psi_c one cycle of hc, the hierarchy of the next coarser
    level (a hierarchy of the coarsest level alone: its exact solve)."""
    n = x.shape[0]
    return prolong_add(hc.vcycle(restrict_fw(x)), np.zeros((n, n)))


def alpha_forward(A, phi, hc: StackHierarchy, f, u0, k, symmetric: bool = False) -> np.ndarray:
    """u_k of Algorithm 2's forward recursion with the stack smoother on the
    trained level and one cycle of hc (the next coarser level) as Psi_c
    (symmetric: H^T after the coarse correction)."""
    post = stack_transpose(phi) if symmetric else phi
    u = np.array(u0, dtype=np.float64)
    for _ in range(k):
        r = f - matvec(A, u)
        a = stack_apply(phi, r)
        s = r - matvec(A, a)
        t = a + _coarse_cycle(hc, s)
        q = r - matvec(A, t)
        u = u + t + stack_apply(post, q)
    return u


def _transpose_index(j: int) -> int:
    """The index in stack_transpose(w) of weight j of w (a permutation)."""
    L, t = j // 9, j % 9
    return (4 - L if L < 5 else 5) * 9 + 8 - t


def alpha_loss_and_grad(A, phi, hc: StackHierarchy, f, u0, u_star, k, symmetric: bool = False):
    """||u_k - u*||_2 and its gradient with respect to the 54 weights, by
    forward-mode differentiation of the recursion (symmetric: H^T after the
    coarse correction, whose weights are a permutation of phi's)."""
    w = _weights(phi)
    wT = stack_transpose(w)
    n = A.shape[1]
    u = np.array(u0, dtype=np.float64)
    du = np.zeros((NWEIGHTS, n, n))  # du[j] = d u / d weight j

    def H_and_tangent(x, dx):
        """H x and d(H x) = H dx + (dH) x for every weight."""
        y = stack_apply(w, x)
        dy = stack_apply(w, dx)
        for j in range(NWEIGHTS):
            dy[j] += stack_derivative(w, x, j // 9, j % 9)
        return y, dy

    def HT_and_tangent(x, dx):
        """H^T x and its tangent: weight j of phi is weight _transpose_index(j) of H^T's stack."""
        y = stack_apply(wT, x)
        dy = stack_apply(wT, dx)
        for j in range(NWEIGHTS):
            i = _transpose_index(j)
            dy[j] += stack_derivative(wT, x, i // 9, i % 9)
        return y, dy

    def A_batch(X):
        return np.stack([matvec(A, x) for x in X])

    def coarse_batch(X):
        return np.stack([_coarse_cycle(hc, x) for x in X])

    for _ in range(k):
        r = f - matvec(A, u)
        dr = -A_batch(du)
        a, da = H_and_tangent(r, dr)
        s = r - matvec(A, a)
        ds = dr - A_batch(da)
        t = a + _coarse_cycle(hc, s)
        dt = da + coarse_batch(ds)
        q = r - matvec(A, t)
        dq = dr - A_batch(dt)
        hq, dhq = (HT_and_tangent if symmetric else H_and_tangent)(q, dq)
        u = u + t + hq
        du = du + dt + dhq
    d = u - np.asarray(u_star, dtype=np.float64)
    L = float(np.linalg.norm(d))
    g = np.einsum("jab,ab->j", du, d) / L if L > 0 else np.zeros(NWEIGHTS)
    return L, g


def batch_loss_and_grad(A, phi, hc: StackHierarchy, f_list, u0_list, ustar_list, ks, symmetric: bool = False):
    """Mean of the loss over a batch of instances of one problem (the stack's
    weights are shared) and its gradient."""
    B = len(ks)
    total, grad = 0.0, np.zeros(NWEIGHTS)
    for f, u0, us, k in zip(f_list, u0_list, ustar_list, ks):
        L, g = alpha_loss_and_grad(A, phi, hc, f, u0, us, k, symmetric)
        total += L / B
        grad += g / B
    return total, grad
