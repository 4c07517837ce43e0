"""The adaptive training loss of Algorithm 2 and its gradient, FP64 (numpy on
top of the oracle's C routines).

TEST INFRASTRUCTURE ONLY (oracle).  At level l of a hierarchy whose coarser
smoothers are fixed, with H = W / a_C the level's trainable smoother, k cycles
from u_0 (Algorithm 2, forward propagation):

    r_i = f - A u_i
    a   = H r_i,            s = r_i - A a
    t   = a + P Psi_c(R s)  (Psi_c: one V(1,1) cycle from the level below, fixed)
    q   = r_i - A t
    u_{i+1} = u_i + t + H q

and the loss ||u_k - u_*||_2.  R = P^T / 4 (full weighting) with the Galerkin
coarse operators; the coarse correction P A_c^{-1} R is the same as with the
paper's P^T.  The gradient with respect to W (the network's output on this
level) is the adjoint (reverse) pass of the same steps, written out plainly:
every step is linear in the state, A is symmetric, and the adjoint of the
fixed coarse cycle is the same cycle with every smoother transposed (a V-cycle
with the same smoother before and after the coarse correction: B = H +
(I - HA) H + (I - HA) P C R (I - AH), so B^T has the same form in H^T and C^T).

Pinned in tests/test_oracle_alpha.py: the forward against the oracle's C
V-cycle, transposed smoother fields against dense transposes, the adjoint
identity of the coarse cycle, and central differences of the loss.
"""
from __future__ import annotations

import numpy as np

from . import apply_smoother5, matvec, prolong_add, restrict_fw, Hierarchy, cnn_forward, cnn_vjp


def transpose_field(A, W):
    """The gather field WT with apply_smoother5(A, WT, x) = H^T x for H = W / a_C."""
    n = A.shape[1]
    ac = A[4]
    WT = np.zeros_like(W)
    for k in range(25):
        dy, dx = k // 5 - 2, k % 5 - 2
        kf = 24 - k  # the tap pointing the other way
        # WT_p[k] = a_C(p) * H_{p + off(k)}[kf], H_q = W_q / a_C(q), zero where p + off(k) is off the grid
        for j in range(n):
            jj = j + dy
            if jj < 0 or jj >= n:
                continue
            for i in range(n):
                ii = i + dx
                if ii < 0 or ii >= n:
                    continue
                WT[k, j, i] = ac[j, i] * W[kf, jj, ii] / ac[jj, ii]
    return WT


def _outer(A, g, x):
    """d/dW of <g, H x> with H = W / a_C: dW_p[k] = g_p x_{p + off(k)} / a_C(p)."""
    n = A.shape[1]
    dW = np.zeros((25, n, n))
    xp = np.zeros((n + 4, n + 4))
    xp[2:n + 2, 2:n + 2] = x
    for k in range(25):
        dy, dx = k // 5 - 2, k % 5 - 2
        dW[k] = g * xp[2 + dy:2 + dy + n, 2 + dx:2 + dx + n] / A[4]
    return dW


def coarse_cycle(h: Hierarchy, x):
    """P Psi_c(R x): one V(1,1) cycle from level 1 of h on the restricted x, prolonged."""
    n = x.shape[0]
    ec = h.vcycle(restrict_fw(x), 1, 1, level=1)
    return prolong_add(ec, np.zeros((n, n)))


def forward(A, W, h: Hierarchy, f, u0, k):
    """u_k and the states the adjoint pass needs ([(r_i, q_i)])."""
    u = np.array(u0, dtype=np.float64)
    states = []
    for _ in range(k):
        r = f - matvec(A, u)
        a = apply_smoother5(A, W, r)
        s = r - matvec(A, a)
        t = a + coarse_cycle(h, s)
        q = r - matvec(A, t)
        u = u + t + apply_smoother5(A, W, q)
        states.append((r, q))
    return u, states


def loss_and_grad(A, W, h: Hierarchy, hT: Hierarchy, f, u0, u_star, k, scale=1.0):
    """scale * ||u_k - u_*||_2 and its gradient with respect to W.

    h: a hierarchy of A whose levels >= 1 carry the fixed coarser smoothers;
    hT: the same hierarchy with those smoothers transposed (transpose_field)."""
    u, states = forward(A, W, h, f, u0, k)
    d = u - u_star
    L = np.linalg.norm(d)
    lam = scale * d / L if L > 0 else np.zeros_like(d)
    WT = transpose_field(A, W)
    dW = np.zeros_like(W)
    for r, q in reversed(states):
        dq = apply_smoother5(A, WT, lam)            # H^T lambda
        dW += _outer(A, lam, q)                      # post-smoothing H q
        dt = lam - matvec(A, dq)
        ds = coarse_cycle(hT, dt)                    # R^T Psi_c^T P^T dt = P Psi_c^T(R dt)
        da = dt - matvec(A, ds)
        dW += _outer(A, da, r)                       # pre-smoothing H r
        dr = ds + dq + apply_smoother5(A, WT, da)
        lam = lam - matvec(A, dr)
    return scale * L, dW


def batch_loss_and_grad(stencils, params, lower_fields, f_list, u0_list, ustar_list, ks, coarsest_n=3):
    """Mean over a batch of the Algorithm 2 loss at the top level of each
    problem's hierarchy, and its gradient with respect to the network
    parameters.  lower_fields[b]: the fixed smoother fields of levels 1, 2, ...
    (one [25, n_l, n_l] array per level above the coarsest)."""
    B = len(stencils)
    total, grad = 0.0, np.zeros(np.asarray(params).size)
    for A, lower, f, u0, us, k in zip(stencils, lower_fields, f_list, u0_list, ustar_list, ks):
        h, hT = Hierarchy(A, coarsest_n), Hierarchy(A, coarsest_n)
        for l, Wl in enumerate(lower, start=1):
            h.set_smoother(l, Wl)
            hT.set_smoother(l, transpose_field(h.stencil(l), Wl))
        W = cnn_forward(A, params)
        L, dW = loss_and_grad(A, W, h, hT, f, u0, us, k, scale=1.0 / B)
        total += L
        grad += cnn_vjp(A, params, dW)
    return total, grad
