"""Flexible GMRES with a multigrid preconditioner, FP64 (section 6, "Incorporation
with FGMRES": the multigrid cycle, whose smoother comes from a network, is
used as the preconditioner of flexible GMRES).

TEST INFRASTRUCTURE ONLY (oracle): the definition of restarted, right-
preconditioned flexible GMRES written out plainly with numpy.  Step j of a
cycle (restart length m, u = u0 + Z y):

    z_j = M(v_j)                              (one preconditioner application)
    w   = A z_j
    h_ij = <w, v_i>, w -= h_ij v_i            (i = 0..j, modified Gram-Schmidt)
    h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}
    y_j = argmin_y || beta e_1 - H_j y ||      (H_j: the (j+2) x (j+1) Hessenberg)

with v_0 = r_0 / beta, beta = ||r_0||.  The least-squares problem is solved
from scratch with numpy at every step (no Givens rotations); its residual is
the residual norm of u0 + Z_j y_j.  A cycle ends when that norm reaches
tol ||f|| or after m steps; u is then updated, the true residual recomputed,
and a new cycle starts from it.

Pinned in tests/test_oracle_krylov.py against an explicit Krylov-space
minimisation, exact convergence in N steps, monotone residuals, and the
bound by the stationary iteration that a linear preconditioner gives.
"""
from __future__ import annotations

import numpy as np


def fgmres(matvec, precond, f, tol: float, maxit: int, restart: int = 30, u0=None):
    """Solves A u = f.  matvec(x) = A x and precond(r) ~ A^{-1} r on arrays of
    f's shape.  Returns (u, iters, history, converged): iters counts
    preconditioner applications, history[k] is the relative residual after k
    of them (history[0] = 1 for u0 = 0)."""
    f = np.asarray(f, dtype=np.float64)
    shape = f.shape
    fv = f.ravel()
    fnorm = np.linalg.norm(fv)
    u = np.zeros_like(fv) if u0 is None else np.asarray(u0, dtype=np.float64).ravel().copy()
    r = fv - matvec(u.reshape(shape)).ravel()
    beta = np.linalg.norm(r)
    hist = [beta / fnorm if fnorm > 0 else 0.0]
    iters = 0
    if fnorm == 0.0 or beta <= tol * fnorm:
        return u.reshape(shape), 0, np.array(hist), True
    while iters < maxit:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        y = np.zeros(0)
        for j in range(restart):
            Z.append(np.asarray(precond(V[j].reshape(shape)), dtype=np.float64).ravel())
            w = matvec(Z[j].reshape(shape)).ravel()
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            rhs = np.zeros(j + 2)
            rhs[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], rhs, rcond=None)[0]
            res = np.linalg.norm(rhs - H[:j + 2, :j + 1] @ y)
            iters += 1
            hist.append(res / fnorm)
            if res <= tol * fnorm or iters >= maxit or H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
        u = u + np.array(Z).T @ y
        r = fv - matvec(u.reshape(shape)).ravel()
        beta = np.linalg.norm(r)
        if beta <= tol * fnorm:
            return u.reshape(shape), iters, np.array(hist), True
    return u.reshape(shape), iters, np.array(hist), False
