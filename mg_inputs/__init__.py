"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random numbers and lays them out; it holds none of the
method's arithmetic (no stencils, transfers, smoothers or networks).  Every
generator is deterministic in its seed.

Workloads (the rotated anisotropic operator of the paper's section 6 with the
bilinear finite-element stencil of section 4, and the variable-coefficient
diffusion of section 6.2 with a log-normal random field):

* ``C1``: n = 63, theta = pi/6, eps = 0.01, RHS U(-1, 1) from seed 0.
* ``C2``: n = 1023, theta = pi/3, eps = 1e-3, RHS U(-1, 1) from seed 0.
* ``C3``: training batches of 256 problems, n in {31, 63}, theta ~ U[0, pi),
  log10 eps ~ U[-3, 0], 16 high-frequency vectors per problem.
* ``C4``: n = 4095, a = exp(g) with g a squared-exponential Gaussian random
  field (length 0.1, sigma 1, seed 7), RHS U(-1, 1).
* ``C5``: 512 problems, n uniform in {63, 127, 255, 511, 1023}, theta ~ U[0, pi),
  log10 eps ~ U[-4, 0], RHS U(-1, 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

CNN_CHANNELS = (9, 32, 32, 32, 25)


# ------------------------------------------------------------ right-hand sides
def rhs_uniform(n: int, seed: int = 0) -> np.ndarray:
    """f ~ U(-1, 1) on the n x n interior, drawn in row-major (j, i) order."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n * n).reshape(n, n)


def random_field(shape, seed: int, low: float = -1.0, high: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(low, high, size=shape)


# ------------------------------------------------------ high-frequency vectors
def hf_vectors(n: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """Unit vectors drawn uniformly from the span of the high-frequency
    Dirichlet sine modes sin(pi kx (i+1)/(n+1)) sin(pi ky (j+1)/(n+1)),
    kx, ky in 1..n with max(kx, ky) > n/2.  Gaussian amplitudes on that
    orthogonal basis give a uniformly random direction in the subspace.
    Returns [count, n, n]."""
    k = np.arange(1, n + 1)
    x = np.arange(n)
    S = np.sin(np.pi * np.outer(x + 1, k) / (n + 1))          # S[i, k-1]
    KX, KY = np.meshgrid(k, k)                                   # [ky-1, kx-1]
    mask = (np.maximum(KX, KY) > n / 2.0).astype(np.float64)
    out = np.empty((count, n, n))
    for c in range(count):
        xi = rng.standard_normal((n, n)) * mask                  # amplitudes [ky, kx]
        v = S @ xi @ S.T                                         # v[j, i]
        out[c] = v / np.linalg.norm(v)
    return out


def hf_pool(n: int, count: int, seed: int) -> np.ndarray:
    return hf_vectors(n, count, np.random.default_rng([seed, n]))


# --------------------------------------------------------- Gaussian random field
def gaussian_random_field(m: int, length: float = 0.1, sigma: float = 1.0, seed: int = 7) -> np.ndarray:
    """Stationary Gaussian field on the m x m cell centres ((I+1/2)/m, (J+1/2)/m)
    of the unit square with covariance sigma^2 exp(-r^2 / (2 length^2)), by
    circulant embedding on a 2m-periodic torus (negative eigenvalues of the
    embedding clipped to zero).  Returns [m, m] indexed [J, I]."""
    rng = np.random.default_rng(seed)
    M = 2 * m
    h = 1.0 / m
    d = np.minimum(np.arange(M), M - np.arange(M)) * h
    DX, DY = np.meshgrid(d, d)
    cov = sigma * sigma * np.exp(-(DX * DX + DY * DY) / (2.0 * length * length))
    lam = np.fft.fft2(cov).real
    lam = np.maximum(lam, 0.0)
    z = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    g = np.fft.fft2(np.sqrt(lam / (M * M)) * z)
    return np.ascontiguousarray(g.real[:m, :m])


def lognormal_coefficient(n: int, length: float = 0.1, sigma: float = 1.0, seed: int = 7) -> np.ndarray:
    """a = exp(g) on the (n+1) x (n+1) cells of an n x n interior grid."""
    return np.exp(gaussian_random_field(n + 1, length, sigma, seed))


# ------------------------------------------------------------ network weights
def domain_mask(n: int, kind: str) -> np.ndarray:
    """Node mask (1 inside, 0 on the removed part, uint8 [n, n]) of a domain in
    the unit square, node (i, j) at ((i+1)h, (j+1)h), h = 1/(n+1):
    'square': all nodes; 'lshape': the square without the quadrant x, y >= 1/2
    (its boundary included); 'cylinder': the square without the disk of radius
    1/5 about (1/2, 1/2) (boundary included)."""
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    X, Y = np.meshgrid(x, x)  # X[j, i] = x_i, Y[j, i] = y_j
    if kind == "square":
        out = np.ones((n, n), dtype=bool)
    elif kind == "lshape":
        out = ~((X >= 0.5) & (Y >= 0.5))
    elif kind == "cylinder":
        out = (X - 0.5) ** 2 + (Y - 0.5) ** 2 > 0.2 ** 2
    else:
        raise ValueError(kind)
    return out.astype(np.uint8)


def random_domain_mask(n: int, rng: np.random.Generator) -> np.ndarray:
    """A random domain inside the unit square (uint8 [n, n], 1 inside): with
    equal odds, the square without a disk (centre ~ U(0.25, 0.75)^2, radius ~
    U(0.08, 0.3)) or without one corner rectangle [a, 1] x [b, 1] mirrored to a
    random corner (a, b ~ U(0.3, 0.7)); boundaries of the removed part included."""
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    X, Y = np.meshgrid(x, x)
    if rng.uniform() < 0.5:
        cx, cy = rng.uniform(0.25, 0.75, 2)
        r = rng.uniform(0.08, 0.3)
        out = (X - cx) ** 2 + (Y - cy) ** 2 > r * r
    else:
        a, b = rng.uniform(0.3, 0.7, 2)
        Xc = X if rng.uniform() < 0.5 else 1.0 - X
        Yc = Y if rng.uniform() < 0.5 else 1.0 - Y
        out = ~((Xc >= a) & (Yc >= b))
    return out.astype(np.uint8)


def cnn_param_count(channels=CNN_CHANNELS) -> int:
    return sum(channels[l + 1] * channels[l] * 9 + channels[l + 1] for l in range(len(channels) - 1))


def cnn_init(seed: int, channels=CNN_CHANNELS, zero_last: bool = True) -> np.ndarray:
    """Flat parameter vector, per layer weights [Cout][Cin][3][3] then bias
    [Cout].  Hidden layers: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights
    and biases (the usual default for convolutions); the last layer is zero
    when ``zero_last`` so that the untrained network is damped Jacobi.
    Values are rounded to float32 so that every consumer sees the same
    numbers."""
    rng = np.random.default_rng(seed)
    parts = []
    L = len(channels) - 1
    for l in range(L):
        cin, cout = channels[l], channels[l + 1]
        bound = 1.0 / math.sqrt(cin * 9)
        if l == L - 1 and zero_last:
            w = np.zeros(cout * cin * 9)
            b = np.zeros(cout)
        else:
            w = rng.uniform(-bound, bound, cout * cin * 9)
            b = rng.uniform(-bound, bound, cout)
        parts += [w, b]
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def cnn_random(seed: int, channels=CNN_CHANNELS, scale_last: float = 0.05) -> np.ndarray:
    """Random parameters with a small non-zero last layer (parity tests)."""
    p = cnn_init(seed, channels, zero_last=False)
    L = len(channels) - 1
    n_last = channels[L] * channels[L - 1] * 9 + channels[L]
    p[-n_last:] *= scale_last * math.sqrt(channels[L - 1] * 9)
    return p.astype(np.float32).astype(np.float64)


def stack_init(seed: int) -> np.ndarray:
    """Weights [6][3][3] of a convolution-stack smoother (f1..f5 composed,
    plus f6) for an operator with centre entry 1: f1..f4 U(-1/3, 1/3) (the
    usual default for a 3x3 single-channel kernel), f5 zero, f6 = 2/3 at the
    centre tap, so that the untrained stack is damped Jacobi and every kernel
    receives a gradient after the first step.  Rounded to float32."""
    rng = np.random.default_rng(seed)
    w = np.zeros((6, 3, 3))
    w[:4] = rng.uniform(-1.0 / 3.0, 1.0 / 3.0, (4, 3, 3))
    w[5, 1, 1] = 2.0 / 3.0
    return w.astype(np.float32).astype(np.float64)


def stack_random(seed: int, scale_last: float = 0.05) -> np.ndarray:
    """Stack weights with every kernel non-zero (parity tests): as stack_init,
    f5 U(-scale_last, scale_last) and f6 perturbed by the same amount."""
    rng = np.random.default_rng(seed)
    w = stack_init(seed + 1000)
    w[4] = rng.uniform(-scale_last, scale_last, (3, 3))
    w[5] += rng.uniform(-scale_last, scale_last, (3, 3))
    return w.astype(np.float32).astype(np.float64)


# ----------------------------------------------------------------- workloads
@dataclass
class RotatedProblem:
    n: int
    theta: float
    eps: float
    rhs_seed: int


def config_c1() -> RotatedProblem:
    return RotatedProblem(63, math.pi / 6, 0.01, 0)


def config_c2() -> RotatedProblem:
    return RotatedProblem(1023, math.pi / 3, 1e-3, 0)


def training_draws(batch: int, seed: int, sizes=(31, 63), log_eps=(-3.0, 0.0)):
    """(n, theta, eps) per problem of one training batch."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=batch)
    theta = rng.uniform(0.0, math.pi, batch)
    eps = 10.0 ** rng.uniform(log_eps[0], log_eps[1], batch)
    return ns.astype(np.int32), theta, eps


def c5_draws(count: int = 512, seed: int = 5):
    """(n, theta, eps, rhs seed) per problem of the uneven batch."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array([63, 127, 255, 511, 1023]), size=count)
    theta = rng.uniform(0.0, math.pi, count)
    eps = 10.0 ** rng.uniform(-4.0, 0.0, count)
    seeds = rng.integers(0, 2 ** 31 - 1, size=count)
    return ns.astype(np.int32), theta, eps, seeds
