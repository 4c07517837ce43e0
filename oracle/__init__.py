"""FP64 CPU oracle for the learned-smoother multigrid method (arXiv 2102.12071).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never does.  This module wraps
the C routines of ``oracle.h`` with numpy arrays (float64, C order).  Grid
vectors are ``[n, n]`` arrays indexed ``[j, i]`` (row j is the y index),
stencil fields ``[9, n, n]`` and smoother fields ``[25, n, n]``; see
``oracle.h`` for the conventions and for which independent checks pin each
routine.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)

# Channel counts of the network: 9 stencil channels in, three hidden layers of
# 32, 25 output channels (one 5x5 smoother stencil per point).
CNN_CHANNELS = (9, 32, 32, 32, 25)
OMEGA = 2.0 / 3.0


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = C.CDLL(_LIB_PATH)
    sig = {
        "ora_stencil_q1_cells": (None, [C.c_int, _dp, _dp, _dp, _dp]),
        "ora_stencil_q1_rotated": (None, [C.c_int, C.c_double, C.c_double, _dp]),
        "ora_stencil_cellavg5": (None, [C.c_int, _dp, _dp]),
        "ora_matvec": (None, [C.c_int, _dp, _dp, _dp]),
        "ora_restrict_fw": (None, [C.c_int, _dp, _dp]),
        "ora_prolong_add": (None, [C.c_int, _dp, _dp]),
        "ora_galerkin": (None, [C.c_int, _dp, _dp]),
        "ora_stencil_to_dense": (None, [C.c_int, _dp, _dp]),
        "ora_cholesky": (C.c_int, [C.c_int, _dp]),
        "ora_cholesky_solve": (None, [C.c_int, _dp, _dp, _dp]),
        "ora_smooth_jacobi": (None, [C.c_int, _dp, C.c_double, _dp, _dp]),
        "ora_smooth_stencil5": (None, [C.c_int, _dp, _dp, _dp, _dp]),
        "ora_apply_smoother5": (None, [C.c_int, _dp, _dp, _dp, _dp]),
        "ora_cnn_vjp": (None, [C.c_int, _dp, C.c_int, _ip, _dp, _dp, _dp]),
        "ora_mg_create": (C.c_void_p, [C.c_int, _dp, C.c_int]),
        "ora_mg_destroy": (None, [C.c_void_p]),
        "ora_mg_num_levels": (C.c_int, [C.c_void_p]),
        "ora_mg_level_n": (C.c_int, [C.c_void_p, C.c_int]),
        "ora_mg_get_stencil": (None, [C.c_void_p, C.c_int, _dp]),
        "ora_mg_set_smoother": (C.c_int, [C.c_void_p, C.c_int, _dp]),
        "ora_mg_vcycle": (None, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, _dp, _dp]),
        "ora_mg_solve": (C.c_int, [C.c_void_p, _dp, _dp, C.c_double, C.c_int, C.c_int, C.c_int,
                                   C.c_double, _dp, _ip]),
        "ora_cnn_num_params": (C.c_int64, [C.c_int, _ip]),
        "ora_cnn_forward": (None, [C.c_int, _dp, C.c_int, _ip, _dp, C.c_double, _dp]),
        "ora_hf_loss": (C.c_double, [C.c_int, _ip, C.POINTER(_dp), C.POINTER(_dp), C.c_int, C.c_int,
                                     _ip, _dp, C.c_double, _dp]),
        "ora_num_threads": (C.c_int, []),
        "ora_set_threads": (None, [C.c_int]),
        "ora_adam_step": (None, [C.c_int64, _dp, _dp, _dp, _dp, C.c_int, C.c_double, C.c_double,
                                 C.c_double, C.c_double]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _ints(seq) -> np.ndarray:
    return np.ascontiguousarray(seq, dtype=np.int32)


def _ip_of(a: np.ndarray):
    return a.ctypes.data_as(_ip)


# ---------------------------------------------------------------- stencils
def stencil_q1_cells(n: int, k11, k12, k22) -> np.ndarray:
    """Q1 stencil of -div(K grad u), K per cell ([n+1, n+1] arrays)."""
    k11, k12, k22 = _f64(k11), _f64(k12), _f64(k22)
    for k in (k11, k12, k22):
        assert k.shape == (n + 1, n + 1)
    A = np.empty((9, n, n))
    _load().ora_stencil_q1_cells(n, _p(k11), _p(k12), _p(k22), _p(A))
    return A


def stencil_q1_rotated(n: int, theta: float, eps: float) -> np.ndarray:
    A = np.empty((9, n, n))
    _load().ora_stencil_q1_rotated(n, float(theta), float(eps), _p(A))
    return A


def stencil_cellavg5(n: int, a) -> np.ndarray:
    a = _f64(a)
    assert a.shape == (n + 1, n + 1)
    A = np.empty((9, n, n))
    _load().ora_stencil_cellavg5(n, _p(a), _p(A))
    return A


# --------------------------------------------------------------- operators
def matvec(A, x) -> np.ndarray:
    A, x = _f64(A), _f64(x)
    n = A.shape[1]
    y = np.empty((n, n))
    _load().ora_matvec(n, _p(A), _p(x), _p(y))
    return y


def restrict_fw(r) -> np.ndarray:
    r = _f64(r)
    n = r.shape[0]
    nc = (n - 1) // 2
    rc = np.empty((nc, nc))
    _load().ora_restrict_fw(n, _p(r), _p(rc))
    return rc


def prolong_add(ec, e) -> np.ndarray:
    """Returns e + P ec (e is not modified)."""
    ec, out = _f64(ec), _f64(e).copy()
    _load().ora_prolong_add(out.shape[0], _p(ec), _p(out))
    return out


def stencil_mask(A, mask) -> np.ndarray:
    """The operator of a domain inside the square (section 6, other geometries):
    nodes with mask 0 are Dirichlet nodes (value 0) and decouple (their row keeps
    its centre entry only); the rows of the nodes inside drop the couplings to
    them.  Pinned against the principal submatrix of the dense operator."""
    A = _f64(A)
    n = A.shape[1]
    inside = np.asarray(mask) != 0
    out = A.copy()
    for c in range(9):
        if c == 4:
            continue
        dy, dx = c // 3 - 1, c % 3 - 1
        for j in range(n):
            for i in range(n):
                jj, ii = j + dy, i + dx
                nb = 0 <= jj < n and 0 <= ii < n and inside[jj, ii]
                if not (inside[j, i] and nb):
                    out[c, j, i] = 0.0
    return out


def galerkin(A) -> np.ndarray:
    A = _f64(A)
    n = A.shape[1]
    nc = (n - 1) // 2
    Ac = np.empty((9, nc, nc))
    _load().ora_galerkin(n, _p(A), _p(Ac))
    return Ac


def stencil_to_dense(A) -> np.ndarray:
    A = _f64(A)
    n = A.shape[1]
    M = np.empty((n * n, n * n))
    _load().ora_stencil_to_dense(n, _p(A), _p(M))
    return M


def cholesky(M) -> np.ndarray:
    L = _f64(M).copy()
    if _load().ora_cholesky(L.shape[0], _p(L)) != 0:
        raise np.linalg.LinAlgError("matrix is not positive definite")
    return L


def cholesky_solve(L, b) -> np.ndarray:
    L, b = _f64(L), _f64(b)
    x = np.empty_like(b)
    _load().ora_cholesky_solve(L.shape[0], _p(L), _p(b), _p(x))
    return x


def smooth_jacobi(A, r, e, omega: float = OMEGA) -> np.ndarray:
    A, r, out = _f64(A), _f64(r), _f64(e).copy()
    _load().ora_smooth_jacobi(A.shape[1], _p(A), float(omega), _p(r), _p(out))
    return out


def smooth_stencil5(A, W, r, e) -> np.ndarray:
    A, W, r, out = _f64(A), _f64(W), _f64(r), _f64(e).copy()
    _load().ora_smooth_stencil5(A.shape[1], _p(A), _p(W), _p(r), _p(out))
    return out


def apply_smoother5(A, W, x) -> np.ndarray:
    A, W, x = _f64(A), _f64(W), _f64(x)
    y = np.empty_like(x)
    _load().ora_apply_smoother5(A.shape[1], _p(A), _p(W), _p(x), _p(y))
    return y


# --------------------------------------------------------------- hierarchy
class Hierarchy:
    """Multigrid hierarchy with Galerkin levels and a dense coarsest solve."""

    def __init__(self, A0, coarsest_n: int = 7):
        self._A0 = _f64(A0)
        self.n = self._A0.shape[1]
        self._h = _load().ora_mg_create(self.n, _p(self._A0), int(coarsest_n))
        if not self._h:
            raise ValueError("cannot build hierarchy (bad size or non-SPD coarsest matrix)")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().ora_mg_destroy(h)
            self._h = None

    @property
    def num_levels(self) -> int:
        return _load().ora_mg_num_levels(self._h)

    def level_n(self, level: int) -> int:
        return _load().ora_mg_level_n(self._h, level)

    def stencil(self, level: int) -> np.ndarray:
        m = self.level_n(level)
        A = np.empty((9, m, m))
        _load().ora_mg_get_stencil(self._h, level, _p(A))
        return A

    def set_smoother(self, level: int, W=None) -> None:
        if W is None:
            rc = _load().ora_mg_set_smoother(self._h, level, None)
        else:
            W = _f64(W)
            rc = _load().ora_mg_set_smoother(self._h, level, _p(W))
        if rc != 0:
            raise ValueError("bad level")

    def vcycle(self, r, nu1: int = 1, nu2: int = 1, omega: float = OMEGA, level: int = 0) -> np.ndarray:
        r = _f64(r)
        e = np.empty_like(r)
        _load().ora_mg_vcycle(self._h, level, nu1, nu2, float(omega), _p(r), _p(e))
        return e

    def solve(self, f, tol: float, maxit: int, nu1: int = 1, nu2: int = 1, omega: float = OMEGA):
        """Returns (u, iterations, history[0..iterations], converged)."""
        f = _f64(f)
        u = np.empty_like(f)
        hist = np.zeros(maxit + 1)
        conv = C.c_int(0)
        k = _load().ora_mg_solve(self._h, _p(f), _p(u), float(tol), int(maxit), nu1, nu2, float(omega),
                                 _p(hist), C.byref(conv))
        return u, k, hist[: k + 1].copy(), bool(conv.value)


# --------------------------------------------------------------------- CNN
def cnn_num_params(channels=CNN_CHANNELS) -> int:
    ch = _ints(channels)
    return int(_load().ora_cnn_num_params(len(channels) - 1, _ip_of(ch)))


def cnn_forward(A, params, channels=CNN_CHANNELS, omega: float = OMEGA) -> np.ndarray:
    """W = omega*delta_0 + CNN(A / a_C), [25, n, n]."""
    A, prm, ch = _f64(A), _f64(params), _ints(channels)
    assert prm.size == cnn_num_params(channels)
    n = A.shape[1]
    W = np.empty((channels[-1], n, n))
    _load().ora_cnn_forward(n, _p(A), len(channels) - 1, _ip_of(ch), _p(prm), float(omega), _p(W))
    return W


def cnn_vjp(A, params, dW, channels=CNN_CHANNELS) -> np.ndarray:
    """Gradient with respect to the parameters of <dW, W(params)> for one problem."""
    A, prm, dW = _f64(A), _f64(params), _f64(dW)
    ch = _ints(channels)
    g = np.zeros(prm.size)
    _load().ora_cnn_vjp(A.shape[1], _p(A), len(channels) - 1, _ip_of(ch), _p(prm), _p(dW), _p(g))
    return g


def hf_loss(stencils, vectors, params, channels=CNN_CHANNELS, omega: float = OMEGA, grad: bool = True):
    """Mean HF smoothing loss over a batch; returns (loss, grad or None).

    stencils: list of [9, n_b, n_b]; vectors: list of [J, n_b, n_b]."""
    B = len(stencils)
    assert len(vectors) == B and B > 0
    J = vectors[0].shape[0]
    As = [_f64(a) for a in stencils]
    Vs = [_f64(v) for v in vectors]
    for a, v in zip(As, Vs):
        assert v.shape == (J, a.shape[1], a.shape[1])
    ns = _ints([a.shape[1] for a in As])
    Ap = (_dp * B)(*[_p(a) for a in As])
    Vp = (_dp * B)(*[_p(v) for v in Vs])
    prm, ch = _f64(params), _ints(channels)
    g = np.zeros(prm.size) if grad else None
    L = _load().ora_hf_loss(B, _ip_of(ns), Ap, Vp, J, len(channels) - 1, _ip_of(ch), _p(prm), float(omega),
                            _p(g) if grad else None)
    return float(L), g


def adam_step(p, m, v, g, t: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """Returns updated (p, m, v) copies after Adam step number t (t >= 1)."""
    p, m, v, g = _f64(p).copy(), _f64(m).copy(), _f64(v).copy(), _f64(g)
    _load().ora_adam_step(p.size, _p(p), _p(m), _p(v), _p(g), int(t), lr, beta1, beta2, eps)
    return p, m, v


# ------------------------------------------------------------------ timing aids
def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().ora_num_threads())


def set_threads(nthreads: int) -> None:
    """Sets the oracle's OpenMP thread count (results do not depend on it)."""
    _load().ora_set_threads(int(nthreads))
