"""Python binding of the mgcnn C ABI (``include/mgcnn.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libmgcnn.so``.  PyTorch provides device memory (CUDA/HIP tensors) and the
current stream.  There is no CPU fallback: if the library is missing or the
device is not a gfx950, every call raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgcnn.so")

MG_OK, MG_NOT_CONVERGED = 0, 1
MG_ERR_ARG, MG_ERR_SHAPE, MG_ERR_DEVICE, MG_ERR_DIVERGED, MG_ERR_STATE, MG_ERR_OOM = -1, -2, -3, -4, -5, -6
SMOOTHER_JACOBI, SMOOTHER_CNN, SMOOTHER_STACK = 0, 1, 2
STACK_WEIGHTS = 54
PREC_FP64, PREC_MIXED = 0, 1

CNN_CHANNELS = (9, 32, 32, 32, 25)
NUM_TIMED_KERNELS = 11
NUM_TILES = 9
TILE_KERNELS = ("descend", "ascend")

# Every exported symbol of the header, with its ctypes signature.
_c_dp = C.POINTER(C.c_double)
_c_fp = C.POINTER(C.c_float)
_c_ip = C.POINTER(C.c_int32)


class MGError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


_STATUS = {0: "MG_OK", 1: "MG_NOT_CONVERGED", -1: "MG_ERR_ARG", -2: "MG_ERR_SHAPE", -3: "MG_ERR_DEVICE",
           -4: "MG_ERR_DIVERGED", -5: "MG_ERR_STATE", -6: "MG_ERR_OOM"}


class Problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("stencil", C.c_void_p)]


class COptions(C.Structure):
    _fields_ = [("smoother", C.c_int32), ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("omega", C.c_double),
                ("coarsest_n", C.c_int32), ("precision", C.c_int32), ("use_graph", C.c_int32),
                ("check_every", C.c_int32), ("fallback", C.c_int32)]


class NetDesc(C.Structure):
    _fields_ = [("nlayers", C.c_int32), ("channels", _c_ip)]


class TrainBatch(C.Structure):
    _fields_ = [("nprob", C.c_int32), ("n", _c_ip), ("stencil", C.POINTER(C.c_void_p)),
                ("vectors", C.POINTER(C.c_void_p)), ("nvec", C.c_int32)]


class TrainDraw(C.Structure):
    _fields_ = [("nprob", C.c_int32), ("n", C.POINTER(C.c_int32)), ("theta", C.POINTER(C.c_double)),
                ("eps", C.POINTER(C.c_double)), ("npools", C.c_int32), ("pool_n", C.POINTER(C.c_int32)),
                ("pool", C.POINTER(C.c_void_p)), ("pool_size", C.POINTER(C.c_int32)),
                ("index", C.POINTER(C.c_int32)), ("nvec", C.c_int32)]


class TrainOpts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("adam_eps", C.c_float),
                ("omega", C.c_double), ("precision", C.c_int32), ("apply_update", C.c_int32)]


class AlphaBatch(C.Structure):
    _fields_ = [("nprob", C.c_int32), ("k", _c_ip), ("f", C.POINTER(C.c_void_p)), ("u0", C.POINTER(C.c_void_p)),
                ("u_star", C.POINTER(C.c_void_p)), ("dW", C.POINTER(C.c_void_p))]


SIGNATURES = {
    "mg_stencil_q1_rotated": (C.c_int, [C.c_int32, C.c_double, C.c_double, C.c_void_p, C.c_void_p]),
    "mg_stencil_cellavg5": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mg_galerkin": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mg_stencil_mask": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mg_options_default": (None, [C.POINTER(COptions)]),
    "mg_setup": (C.c_int, [C.POINTER(Problem), C.c_int32, C.POINTER(COptions), C.c_void_p, C.POINTER(C.c_void_p)]),
    "mg_destroy": (C.c_int, [C.c_void_p]),
    "mg_num_levels": (C.c_int, [C.c_void_p, C.c_int32, _c_ip]),
    "mg_get_stencil": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "mg_smoother_infer": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mg_smoother_infer_size": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "mg_smoother_infer_levels": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "mg_smoother_transpose": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mg_alpha_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(AlphaBatch),
                                C.POINTER(TrainOpts), _c_dp, _c_dp, _c_fp]),
    "mg_set_smoother": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "mg_set_stack": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _c_dp, C.c_int32, C.c_int32]),
    "mg_set_stack_post": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _c_dp, C.c_int32, C.c_int32]),
    "mg_stack_apply": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "mg_stack_alpha_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_int32, C.c_int32, C.POINTER(AlphaBatch), C.POINTER(TrainOpts), _c_dp,
                                      _c_dp, _c_dp]),
    "mg_get_smoother": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "mg_vcycle": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "mg_solve": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_double, C.c_int32, _c_ip,
                           _c_dp, _c_ip, _c_dp]),
    "mg_solve_fgmres": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_double, C.c_int32,
                                  C.c_int32, _c_ip, _c_dp, _c_ip, _c_dp]),
    "mg_solve_fgmres_noalloc": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_double,
                                          C.c_int32, C.c_int32, _c_ip, _c_dp, _c_ip, _c_dp]),
    "mg_last_solve_ms": (C.c_int, [C.c_void_p, _c_dp]),
    "mg_last_fallbacks": (C.c_int, [C.c_void_p, _c_ip]),
    "mg_restencil": (C.c_int, [C.c_void_p, C.POINTER(Problem)]),
    "mg_time_kernels": (C.c_int, [C.c_void_p, C.c_int32, _c_dp]),
    "mg_kernel_name": (C.c_char_p, [C.c_int32]),
    "mg_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.c_char_p]),
    "mg_get_tile": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _c_ip, _c_dp]),
    "mg_set_tile": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]),
    "mg_tile_name": (C.c_char_p, [C.c_int32, C.c_int32]),
    "mg_net_create": (C.c_int, [C.POINTER(NetDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "mg_net_destroy": (C.c_int, [C.c_void_p]),
    "mg_net_num_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "mg_net_get": (C.c_int, [C.c_void_p, _c_fp, C.c_int64]),
    "mg_net_set": (C.c_int, [C.c_void_p, _c_fp, C.c_int64]),
    "mg_net_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "mg_net_load": (C.c_int, [C.c_void_p, C.c_char_p]),
    "mg_train_opts_default": (None, [C.POINTER(TrainOpts)]),
    "mg_train_step": (C.c_int, [C.c_void_p, C.POINTER(TrainBatch), C.POINTER(TrainOpts), _c_fp, _c_fp]),
    "mg_train_step_draw": (C.c_int, [C.c_void_p, C.POINTER(TrainDraw), C.POINTER(TrainOpts), _c_fp, _c_fp]),
    "mg_rb_create": (C.c_int, [C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "mg_rb_destroy": (C.c_int, [C.c_void_p]),
    "mg_rb_level": (C.c_int, [C.c_void_p, C.c_int32, _c_ip, _c_ip, _c_ip]),
    "mg_rb_get_stencil": (C.c_int, [C.c_void_p, C.c_int32, _c_ip, C.c_void_p]),
    "mg_rb_set_smoother": (C.c_int, [C.c_void_p, C.c_int32, _c_dp, C.c_double]),
    "mg_rb_vcycle": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    "mg_rb_solve": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                              C.c_int32, C.c_int32, _c_ip, _c_dp, _c_ip, _c_dp]),
    "mg_rb_last_solve_ms": (C.c_int, [C.c_void_p, _c_dp]),
    "mg_rb_alpha_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                   _c_ip, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(TrainOpts), _c_dp, _c_dp,
                                   _c_dp]),
    "mg_status_str": (C.c_char_p, [C.c_int]),
    "mg_last_error": (C.c_char_p, []),
    "mg_version": (C.c_char_p, []),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libmgcnn.so (built by ``paper_2102_12071_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2102_12071_amd.build` "
                          f"(there is no fallback path)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, allow=(MG_OK,)) -> int:
    if status in allow:
        return status
    msg = load_library().mg_last_error()
    raise MGError(status, msg.decode() if msg else "")


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t: torch.Tensor, shape=None) -> torch.Tensor:
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("expected a device (cuda) tensor")
    if t.dtype != torch.float64:
        raise TypeError("expected a float64 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.contiguous()


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ discretisation
def stencil_q1_rotated(n: int, theta: float, eps: float, device="cuda") -> torch.Tensor:
    out = torch.empty((9, n, n), dtype=torch.float64, device=device)
    _check(load_library().mg_stencil_q1_rotated(n, float(theta), float(eps), _ptr(out), _stream()))
    return out


def stencil_cellavg5(a: torch.Tensor) -> torch.Tensor:
    a = _dev_f64(a)
    n = a.shape[0] - 1
    out = torch.empty((9, n, n), dtype=torch.float64, device=a.device)
    _check(load_library().mg_stencil_cellavg5(n, _ptr(a), _ptr(out), _stream()))
    return out


def stencil_mask(A: torch.Tensor, mask: torch.Tensor) -> torch.Tensor:
    """The stencil restricted to the nodes where mask is nonzero (zero Dirichlet value outside)."""
    A = _dev_f64(A)
    n = A.shape[1]
    if not (isinstance(mask, torch.Tensor) and mask.is_cuda and tuple(mask.shape) == (n, n)):
        raise ValueError("mask must be a device tensor [n, n]")
    m = (mask != 0).to(torch.uint8).contiguous()
    out = torch.empty_like(A)
    _check(load_library().mg_stencil_mask(n, _ptr(m), _ptr(A), _ptr(out), _stream()))
    return out


def galerkin(A: torch.Tensor) -> torch.Tensor:
    A = _dev_f64(A)
    n = A.shape[1]
    nc = (n - 1) // 2
    out = torch.empty((9, nc, nc), dtype=torch.float64, device=A.device)
    _check(load_library().mg_galerkin(n, _ptr(A), _ptr(out), _stream()))
    return out


# ------------------------------------------------------------------------ solver
@dataclass
class Options:
    smoother: int = SMOOTHER_JACOBI
    nu_pre: int = 1
    nu_post: int = 1
    omega: float = 2.0 / 3.0
    coarsest_n: int = 7
    precision: int = PREC_MIXED
    use_graph: int = 1
    check_every: int = 16
    fallback: int = 0

    def to_c(self) -> COptions:
        return COptions(self.smoother, self.nu_pre, self.nu_post, self.omega, self.coarsest_n, self.precision,
                        self.use_graph, self.check_every, self.fallback)


@dataclass
class SolveResult:
    u: List[torch.Tensor]
    iters: np.ndarray
    relres: np.ndarray
    status: np.ndarray
    history: Optional[np.ndarray] = None
    ms: float = 0.0


class Context:
    """A batch of problems and their multigrid hierarchies (mg_setup)."""

    def __init__(self, stencils: Sequence[torch.Tensor], options: Optional[Options] = None, stream=None):
        lib = load_library()
        self.options = options or Options()
        self._stencils = [_dev_f64(a) for a in stencils]
        for a in self._stencils:
            if a.dim() != 3 or a.shape[0] != 9 or a.shape[1] != a.shape[2]:
                raise ValueError("stencils must be [9, n, n]")
        self.ns = [int(a.shape[1]) for a in self._stencils]
        probs = (Problem * len(self.ns))(*[Problem(n, a.data_ptr()) for n, a in zip(self.ns, self._stencils)])
        h = C.c_void_p()
        opt = self.options.to_c()
        self._stream = stream
        _check(lib.mg_setup(probs, len(self.ns), C.byref(opt), _stream(stream), C.byref(h)))
        self._h = h
        self._stencils = None  # mg_setup copied them

    def restencil(self, stencils: Sequence[torch.Tensor]) -> None:
        """New coefficients, same sizes: rebuilds the hierarchy in place."""
        st = [_dev_f64(a) for a in stencils]
        if [int(a.shape[1]) for a in st] != self.ns:
            raise ValueError("sizes differ from set-up")
        probs = (Problem * len(self.ns))(*[Problem(n, a.data_ptr()) for n, a in zip(self.ns, st)])
        _check(load_library().mg_restencil(self._h, probs))

    def time_kernels(self, reps: int = 20) -> dict:
        """Mean launch duration (ms) of each finest-level kernel of problem 0."""
        lib = load_library()
        ms = np.zeros(NUM_TIMED_KERNELS, dtype=np.float64)
        _check(lib.mg_time_kernels(self._h, int(reps), ms.ctypes.data_as(_c_dp)))
        return {lib.mg_kernel_name(k).decode(): float(ms[k]) for k in range(NUM_TIMED_KERNELS)}

    def autotune(self, reps: int = 10, cache: Optional[str] = None) -> None:
        """Times every workgroup shape of the fused level kernels per level size and keeps the fastest."""
        _check(load_library().mg_autotune(self._h, int(reps), cache.encode() if cache else None))

    def tile(self, kernel: str, n: int) -> dict:
        """Shape in use for 'descend' or 'ascend' on level size n, with the per-shape times of the last tuning."""
        lib = load_library()
        k = TILE_KERNELS.index(kernel)
        t = C.c_int32(0)
        ms = np.zeros(NUM_TILES, dtype=np.float64)
        _check(lib.mg_get_tile(self._h, k, int(n), C.byref(t), ms.ctypes.data_as(_c_dp)))
        return {"tile": int(t.value), "shape": lib.mg_tile_name(k, t.value).decode(),
                "ms": {lib.mg_tile_name(k, q).decode(): float(ms[q]) for q in range(NUM_TILES)}}

    def set_tile(self, kernel: str, n: int, tile: int) -> None:
        """Forces a shape for 'descend' or 'ascend' on level size n (0: all sizes)."""
        _check(load_library().mg_set_tile(self._h, TILE_KERNELS.index(kernel), int(n), int(tile)))

    def close(self):
        if getattr(self, "_h", None):
            load_library().mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nprob(self) -> int:
        return len(self.ns)

    def num_levels(self, prob: int = 0) -> int:
        v = C.c_int32()
        _check(load_library().mg_num_levels(self._h, prob, C.byref(v)))
        return v.value

    def level_n(self, prob: int, level: int) -> int:
        n = self.ns[prob]
        for _ in range(level):
            n = (n - 1) // 2
        return n

    def stencil(self, prob: int, level: int) -> torch.Tensor:
        m = self.level_n(prob, level)
        out = torch.empty((9, m, m), dtype=torch.float64, device="cuda")
        _check(load_library().mg_get_stencil(self._h, prob, level, _ptr(out)))
        return out

    def smoother(self, prob: int, level: int) -> torch.Tensor:
        m = self.level_n(prob, level)
        out = torch.empty((25, m, m), dtype=torch.float64, device="cuda")
        _check(load_library().mg_get_smoother(self._h, prob, level, _ptr(out)))
        return out

    def set_smoother(self, prob: int, level: int, W: torch.Tensor) -> None:
        m = self.level_n(prob, level)
        W = _dev_f64(W, (25, m, m))
        _check(load_library().mg_set_smoother(self._h, prob, level, _ptr(W)))
        torch.cuda.current_stream().synchronize()

    def set_stack(self, prob: int, level: int, phi, transpose: bool = False, symmetric: bool = False,
                  normalised: bool = False) -> None:
        """Installs a level's convolution-stack smoother (54 weights [6][3][3], f1..f5 then f6);
        symmetric: its transpose after the coarse correction; normalised: the weights were made
        for a_C = 1 (the library scales them to the level's operator)."""
        w = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
        if w.size != STACK_WEIGHTS:
            raise ValueError("a stack has 54 weights")
        lib = load_library()
        nz = int(bool(normalised))
        _check(lib.mg_set_stack(self._h, prob, level, w.ctypes.data_as(_c_dp), int(bool(transpose)), nz))
        if symmetric:
            _check(lib.mg_set_stack_post(self._h, prob, level, w.ctypes.data_as(_c_dp), int(not transpose), nz))

    def set_stacks(self, stacks: dict, transpose: bool = False, symmetric: bool = False) -> None:
        """Every level above the coarsest of every problem from {trained size: weights normalised
        to a_C = 1}: a level of size m takes the stack of the nearest trained size on the log2
        scale (levels finer than every trained size: the finest one); the library scales it to the
        level's operator."""
        sizes = sorted(int(k) for k in stacks)
        if not sizes:
            raise ValueError("no stacks given")
        for p in range(self.nprob):
            for l in range(self.num_levels(p) - 1):
                m = self.level_n(p, l)
                best = min(sizes, key=lambda q: abs(math.log2(q + 1) - math.log2(m + 1)))
                self.set_stack(p, l, stacks[best], transpose, symmetric, normalised=True)

    def infer(self, net: "Net", size: Optional[int] = None) -> None:
        """Network inference on every smoothing level, or (size given) on the levels of that size only."""
        if size is None:
            _check(load_library().mg_smoother_infer(self._h, net._h))
        else:
            _check(load_library().mg_smoother_infer_size(self._h, net._h, int(size)))

    def infer_levels(self, nets: dict, one_call: bool = True) -> None:
        """Per-level networks keyed by level size (adaptive training gives one per level): every
        smoothing level takes the network of its size, or of the nearest trained size.  One
        mg_smoother_infer_levels call (one_call), or one mg_smoother_infer_size call per size."""
        if not nets:
            raise ValueError("no networks")
        sizes = sorted(nets)
        have = set()
        for p in range(self.nprob):
            for l in range(self.num_levels(p) - 1):
                have.add(self.level_n(p, l))
        pick = {m: nets[min(sizes, key=lambda s: (abs(math.log2(s + 1) - math.log2(m + 1)), -s))]
                for m in sorted(have)}
        if one_call:
            ms = sorted(pick)
            hs = (C.c_void_p * len(ms))(*[pick[m]._h for m in ms])
            ns = (C.c_int32 * len(ms))(*ms)
            _check(load_library().mg_smoother_infer_levels(self._h, hs, ns, len(ms)))
        else:
            for m, net in pick.items():
                _check(load_library().mg_smoother_infer_size(self._h, net._h, int(m)))

    def _vecs(self, xs, name):
        if len(xs) != self.nprob:
            raise ValueError(f"need {self.nprob} {name} vectors")
        return [_dev_f64(x, (n, n)) for x, n in zip(xs, self.ns)]

    def vcycle(self, f: Sequence[torch.Tensor], u: Sequence[torch.Tensor]) -> None:
        """u <- u + V(f - A u) in place."""
        f = self._vecs(f, "f")
        u = self._vecs(u, "u")
        fp = (C.c_void_p * self.nprob)(*[x.data_ptr() for x in f])
        up = (C.c_void_p * self.nprob)(*[x.data_ptr() for x in u])
        _check(load_library().mg_vcycle(self._h, fp, up))

    def solve(self, f: Sequence[torch.Tensor], rtol: float, maxit: int, history: bool = False,
              u: Optional[Sequence[torch.Tensor]] = None) -> SolveResult:
        f = self._vecs(f, "f")
        if u is None:
            u = [torch.empty((n, n), dtype=torch.float64, device="cuda") for n in self.ns]
        else:
            u = self._vecs(u, "u")
        fp = (C.c_void_p * self.nprob)(*[x.data_ptr() for x in f])
        up = (C.c_void_p * self.nprob)(*[x.data_ptr() for x in u])
        iters = np.zeros(self.nprob, dtype=np.int32)
        relres = np.zeros(self.nprob, dtype=np.float64)
        status = np.zeros(self.nprob, dtype=np.int32)
        hist = np.zeros((self.nprob, maxit + 1), dtype=np.float64) if history else None
        st = load_library().mg_solve(self._h, fp, up, float(rtol), int(maxit),
                                     iters.ctypes.data_as(_c_ip), relres.ctypes.data_as(_c_dp),
                                     status.ctypes.data_as(_c_ip),
                                     hist.ctypes.data_as(_c_dp) if history else None)
        _check(st, allow=(MG_OK, MG_NOT_CONVERGED, MG_ERR_DIVERGED))
        ms = C.c_double()
        _check(load_library().mg_last_solve_ms(self._h, C.byref(ms)))
        return SolveResult(u=list(u), iters=iters, relres=relres, status=status, history=hist, ms=ms.value)

    def fallbacks(self) -> np.ndarray:
        """Per problem: 1 if the last solve switched it to damped Jacobi."""
        out = np.zeros(self.nprob, dtype=np.int32)
        _check(load_library().mg_last_fallbacks(self._h, out.ctypes.data_as(_c_ip)))
        return out

    def solve_fgmres(self, f: Sequence[torch.Tensor], rtol: float, maxit: int, restart: int = 30,
                     history: bool = False, u: Optional[Sequence[torch.Tensor]] = None,
                     noalloc: bool = False) -> SolveResult:
        """Flexible GMRES(restart) preconditioned by one V-cycle per iteration (u_0 = 0).
        noalloc: mg_solve_fgmres_noalloc (the Krylov workspace in the library's fixed device array;
        the caller passes u then, or the binding's own u allocation happens here, before the call)."""
        f = self._vecs(f, "f")
        if u is None:
            u = [torch.empty((n, n), dtype=torch.float64, device="cuda") for n in self.ns]
        else:
            u = self._vecs(u, "u")
        fp = (C.c_void_p * self.nprob)(*[x.data_ptr() for x in f])
        up = (C.c_void_p * self.nprob)(*[x.data_ptr() for x in u])
        iters = np.zeros(self.nprob, dtype=np.int32)
        relres = np.zeros(self.nprob, dtype=np.float64)
        status = np.zeros(self.nprob, dtype=np.int32)
        hist = np.zeros((self.nprob, maxit + 1), dtype=np.float64) if history else None
        fn = load_library().mg_solve_fgmres_noalloc if noalloc else load_library().mg_solve_fgmres
        st = fn(self._h, fp, up, float(rtol), int(maxit), int(restart),
                iters.ctypes.data_as(_c_ip), relres.ctypes.data_as(_c_dp),
                status.ctypes.data_as(_c_ip),
                hist.ctypes.data_as(_c_dp) if history else None)
        _check(st, allow=(MG_OK, MG_NOT_CONVERGED, MG_ERR_DIVERGED))
        ms = C.c_double()
        _check(load_library().mg_last_solve_ms(self._h, C.byref(ms)))
        return SolveResult(u=list(u), iters=iters, relres=relres, status=status, history=hist, ms=ms.value)


# ----------------------------------------------------------------------- network
@dataclass
class TrainOptions:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-8
    omega: float = 2.0 / 3.0
    precision: int = 1
    apply_update: int = 1

    def to_c(self) -> TrainOpts:
        return TrainOpts(self.lr, self.beta1, self.beta2, self.adam_eps, self.omega, self.precision,
                         self.apply_update)


class Net:
    """The stencil-to-smoother network (mg_net_*)."""

    def __init__(self, stream=None):
        lib = load_library()
        ch = (C.c_int32 * 5)(*CNN_CHANNELS)
        d = NetDesc(4, ch)
        h = C.c_void_p()
        _check(lib.mg_net_create(C.byref(d), _stream(stream), C.byref(h)))
        self._h = h
        v = C.c_int64()
        _check(lib.mg_net_num_params(h, C.byref(v)))
        self.num_params = v.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().mg_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get(self) -> np.ndarray:
        out = np.zeros(self.num_params, dtype=np.float32)
        _check(load_library().mg_net_get(self._h, out.ctypes.data_as(_c_fp), self.num_params))
        return out

    def set(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.num_params:
            raise ValueError(f"need {self.num_params} parameters")
        _check(load_library().mg_net_set(self._h, p.ctypes.data_as(_c_fp), self.num_params))

    def save(self, path: str) -> None:
        _check(load_library().mg_net_save(self._h, path.encode()))

    def load(self, path: str) -> None:
        _check(load_library().mg_net_load(self._h, path.encode()))

    def train_step(self, stencils: Sequence[torch.Tensor], vectors: Sequence[torch.Tensor],
                   opts: Optional[TrainOptions] = None, want_loss: bool = True, want_grad: bool = False):
        """One step on the HF smoothing loss.  stencils: [9, n, n] float64;
        vectors: [J, n, n] float32 per problem.  Returns (loss, grad)."""
        opts = opts or TrainOptions()
        B = len(stencils)
        if B == 0 or len(vectors) != B:
            raise ValueError("need one vector set per stencil")
        st = [_dev_f64(a) for a in stencils]
        J = int(vectors[0].shape[0])
        vs = []
        for a, v in zip(st, vectors):
            n = a.shape[1]
            if not (v.is_cuda and v.dtype == torch.float32 and tuple(v.shape) == (J, n, n)):
                raise ValueError("vectors must be float32 device tensors [J, n, n]")
            vs.append(v.contiguous())
        ns = (C.c_int32 * B)(*[int(a.shape[1]) for a in st])
        sp = (C.c_void_p * B)(*[a.data_ptr() for a in st])
        vp = (C.c_void_p * B)(*[v.data_ptr() for v in vs])
        batch = TrainBatch(B, ns, sp, vp, J)
        o = opts.to_c()
        loss = C.c_float()
        grad = np.zeros(self.num_params, dtype=np.float32) if want_grad else None
        self._keep = (st, vs)  # alive until the next step
        _check(load_library().mg_train_step(self._h, C.byref(batch), C.byref(o),
                                            C.byref(loss) if want_loss else None,
                                            grad.ctypes.data_as(_c_fp) if want_grad else None))
        return (loss.value if want_loss else None), grad

    def train_step_draw(self, n: Sequence[int], theta: Sequence[float], eps: Sequence[float], pools: dict,
                        index, opts: Optional[TrainOptions] = None, want_loss: bool = True, want_grad: bool = False):
        """One step on problems the library draws up (mg_train_step_draw): per problem the size n,
        the tensor (theta, eps), and index [B, J] into pools {size: float32 device tensor [count, m, m]}.
        Returns (loss, grad)."""
        opts = opts or TrainOptions()
        B = len(n)
        idx = np.ascontiguousarray(np.asarray(index, dtype=np.int32))
        if idx.ndim != 2 or idx.shape[0] != B or len(theta) != B or len(eps) != B:
            raise ValueError("need n, theta, eps of length B and index [B, J]")
        sizes = sorted(int(k) for k in pools)
        for m in sizes:
            t = pools[m]
            if not (t.is_cuda and t.dtype == torch.float32 and t.dim() == 3 and tuple(t.shape[1:]) == (m, m)
                    and t.is_contiguous()):
                raise ValueError("pools must be contiguous float32 device tensors [count, m, m]")
        ns = np.ascontiguousarray(np.asarray(n, dtype=np.int32))
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        ep = np.ascontiguousarray(np.asarray(eps, dtype=np.float64))
        pn = (C.c_int32 * len(sizes))(*sizes)
        pp = (C.c_void_p * len(sizes))(*[pools[m].data_ptr() for m in sizes])
        ps = (C.c_int32 * len(sizes))(*[int(pools[m].shape[0]) for m in sizes])
        d = TrainDraw(B, ns.ctypes.data_as(_c_ip), th.ctypes.data_as(_c_dp), ep.ctypes.data_as(_c_dp), len(sizes),
                      pn, pp, ps, idx.ctypes.data_as(_c_ip), int(idx.shape[1]))
        o = opts.to_c()
        loss = C.c_float()
        grad = np.zeros(self.num_params, dtype=np.float32) if want_grad else None
        self._keep_pools = pools  # the captured step reads them on later replays
        _check(load_library().mg_train_step_draw(self._h, C.byref(d), C.byref(o),
                                                 C.byref(loss) if want_loss else None,
                                                 grad.ctypes.data_as(_c_fp) if want_grad else None))
        return (loss.value if want_loss else None), grad


# ----------------------------------------------------------- adaptive training
def smoother_transpose(A: torch.Tensor, W: torch.Tensor) -> torch.Tensor:
    """The field WT whose smoother WT / a_C is the transpose of W / a_C."""
    A = _dev_f64(A)
    n = A.shape[1]
    W = _dev_f64(W, (25, n, n))
    out = torch.empty_like(W)
    _check(load_library().mg_smoother_transpose(n, _ptr(A), _ptr(W), _ptr(out), _stream()))
    return out


def stack_apply(phi: torch.Tensor, x: torch.Tensor, y: Optional[torch.Tensor] = None,
                accumulate: bool = False) -> torch.Tensor:
    """y (+)= H x for the stack phi (device [54] FP64) on a batch x [count, n, n] or [n, n]."""
    phi = _dev_f64(phi).reshape(-1)
    if phi.numel() != STACK_WEIGHTS:
        raise ValueError("a stack has 54 weights")
    x = _dev_f64(x)
    xb = x.reshape(-1, x.shape[-2], x.shape[-1])
    n = xb.shape[-1]
    if y is None:
        y = torch.zeros_like(x)
    yb = y.reshape(-1, n, n)
    _check(load_library().mg_stack_apply(n, xb.shape[0], _ptr(phi), _ptr(xb), _ptr(yb), int(bool(accumulate)),
                                         _stream()))
    return y


class StackAdam:
    """The 54 device weights of one level's stack and their Adam state (FP64)."""

    def __init__(self, phi):
        self.phi = torch.tensor(np.asarray(phi, dtype=np.float64).reshape(-1), device="cuda")
        self.m = torch.zeros(STACK_WEIGHTS, dtype=torch.float64, device="cuda")
        self.v = torch.zeros(STACK_WEIGHTS, dtype=torch.float64, device="cuda")
        self.t = 0


def stack_alpha_step(top: Context, coarse: Context, coarse_t: Context, state: StackAdam, k: Sequence[int],
                     f: Sequence[torch.Tensor], u0: Sequence[torch.Tensor], u_star: Sequence[torch.Tensor],
                     opts: Optional["TrainOptions"] = None, symmetric: bool = False) -> "AlphaResult":
    """One Algorithm 2 step of a stack smoother (mg_stack_alpha_step): loss, the 54-weight
    gradient (FP64), and an Adam update of state per opts."""
    opts = opts or TrainOptions(precision=0)
    B = top.nprob
    n = top.ns[0]
    if not (len(k) == len(f) == len(u0) == len(u_star) == B):
        raise ValueError(f"need {B} entries of k, f, u0 and u_star")
    f = [_dev_f64(x, (n, n)) for x in f]
    u0 = [_dev_f64(x, (n, n)) for x in u0]
    us = [_dev_f64(x, (n, n)) for x in u_star]
    arr = lambda xs: (C.c_void_p * B)(*[x.data_ptr() for x in xs])
    kk = (C.c_int32 * B)(*[int(x) for x in k])
    batch = AlphaBatch(B, kk, arr(f), arr(u0), arr(us), None)
    o = opts.to_c()
    t = state.t + 1 if opts.apply_update else max(state.t, 1)
    loss = C.c_double()
    losses = np.zeros(B, dtype=np.float64)
    grad = np.zeros(STACK_WEIGHTS, dtype=np.float64)
    _check(load_library().mg_stack_alpha_step(top._h, coarse._h, coarse_t._h, _ptr(state.phi), _ptr(state.m),
                                              _ptr(state.v), t, int(bool(symmetric)), C.byref(batch), C.byref(o),
                                              C.byref(loss),
                                              losses.ctypes.data_as(_c_dp), grad.ctypes.data_as(_c_dp)))
    if opts.apply_update:
        state.t = t
    return AlphaResult(loss=loss.value, losses=losses, grad=grad)


@dataclass
class AlphaResult:
    loss: float
    losses: np.ndarray
    grad: Optional[np.ndarray] = None
    dW: Optional[List[torch.Tensor]] = None


def alpha_step(top: Context, coarse: Context, coarse_t: Context, net: Net, k: Sequence[int],
               f: Sequence[torch.Tensor], u0: Sequence[torch.Tensor], u_star: Sequence[torch.Tensor],
               opts: Optional[TrainOptions] = None, want_grad: bool = False, want_dW: bool = False) -> AlphaResult:
    """One Algorithm 2 step (mg_alpha_step): loss, optional gradients, Adam update per opts."""
    opts = opts or TrainOptions(precision=0)
    B = top.nprob
    n = top.ns[0]
    if not (len(k) == len(f) == len(u0) == len(u_star) == B):
        raise ValueError(f"need {B} entries of k, f, u0 and u_star")
    f = [_dev_f64(x, (n, n)) for x in f]
    u0 = [_dev_f64(x, (n, n)) for x in u0]
    us = [_dev_f64(x, (n, n)) for x in u_star]
    dW = [torch.empty((25, n, n), dtype=torch.float64, device="cuda") for _ in range(B)] if want_dW else None
    arr = lambda xs: (C.c_void_p * B)(*[x.data_ptr() for x in xs])
    kk = (C.c_int32 * B)(*[int(x) for x in k])
    batch = AlphaBatch(B, kk, arr(f), arr(u0), arr(us), arr(dW) if want_dW else None)
    o = opts.to_c()
    loss = C.c_double()
    losses = np.zeros(B, dtype=np.float64)
    grad = np.zeros(net.num_params, dtype=np.float32) if want_grad else None
    _check(load_library().mg_alpha_step(top._h, coarse._h, coarse_t._h, net._h, C.byref(batch), C.byref(o),
                                        C.byref(loss), losses.ctypes.data_as(_c_dp),
                                        grad.ctypes.data_as(_c_fp) if want_grad else None))
    return AlphaResult(loss=loss.value, losses=losses, grad=grad, dW=dW)


# ------------------------------------------------------------ red-black coarsening
RB_WEIGHTS = 18


class RedBlack:
    """Red-black hierarchy of one operator (mg_rb_*): levels alternate between a full grid and its
    checkerboard, stored padded on N x N arrays; damped Jacobi or the two-layer stack per level."""

    def __init__(self, A: torch.Tensor, nlevels: int, stream=None):
        A = _dev_f64(A)
        n = A.shape[-1]
        if tuple(A.shape) != (9, n, n):
            raise ValueError("stencil must be [9, n, n]")
        h = C.c_void_p()
        _check(load_library().mg_rb_create(n, _ptr(A), int(nlevels), _stream(stream), C.byref(h)))
        self._h = h
        self.n = n
        self.num_levels = int(nlevels)
        self.shapes = []
        for l in range(self.num_levels):
            N, ck, K = C.c_int32(), C.c_int32(), C.c_int32()
            _check(load_library().mg_rb_level(self._h, l, C.byref(N), C.byref(ck), C.byref(K)))
            self.shapes.append((N.value, "checker" if ck.value else "full", K.value))

    def close(self):
        if getattr(self, "_h", None):
            load_library().mg_rb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_n(self, level: int) -> int:
        return self.shapes[level][0]

    def stencil(self, level: int):
        """(offsets [K, 2] as (dx, dy), field [K, N, N] on the device)."""
        N, _, K = self.shapes[level]
        offs = np.zeros(2 * K, dtype=np.int32)
        out = torch.empty((K, N, N), dtype=torch.float64, device="cuda")
        _check(load_library().mg_rb_get_stencil(self._h, level, offs.ctypes.data_as(_c_ip), _ptr(out)))
        return offs.reshape(K, 2), out

    def set_smoother(self, level: int, phi=None, a_ref: float = 0.0) -> None:
        """phi: 18 weights [2][3][3] (f1, f2), or None for damped Jacobi; a_ref > 0: the weights
        were made for an operator of centre entry a_ref (the library rescales f1 to the level's)."""
        if phi is None:
            _check(load_library().mg_rb_set_smoother(self._h, level, None, 0.0))
            return
        w = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
        if w.size != RB_WEIGHTS:
            raise ValueError("a red-black stack has 18 weights")
        _check(load_library().mg_rb_set_smoother(self._h, level, w.ctypes.data_as(_c_dp), float(a_ref)))

    def vcycle(self, r: torch.Tensor, level: int = 0, nu_pre: int = 1, nu_post: int = 1) -> torch.Tensor:
        """e = V(r) from level for a batch r [nvec, N, N] (or [N, N])."""
        N = self.level_n(level)
        r = _dev_f64(r)
        rb = r.reshape(-1, N, N)
        e = torch.empty_like(rb)
        _check(load_library().mg_rb_vcycle(self._h, level, rb.shape[0], _ptr(rb), _ptr(e), nu_pre, nu_post))
        return e.reshape(r.shape)

    def solve(self, f: torch.Tensor, rtol: float, maxit: int, nu_pre: int = 1, nu_post: int = 1,
              history: bool = False, level: int = 0) -> SolveResult:
        """The stationary solve from u = 0 on `level` for f [nvec, N, N] (or [N, N])."""
        f = _dev_f64(f)
        N = self.level_n(level)
        fb = f.reshape(-1, N, N)
        nv = fb.shape[0]
        u = torch.empty_like(fb)
        iters = np.zeros(nv, dtype=np.int32)
        relres = np.zeros(nv, dtype=np.float64)
        status = np.zeros(nv, dtype=np.int32)
        hist = np.zeros((nv, maxit + 1), dtype=np.float64) if history else None
        st = load_library().mg_rb_solve(self._h, level, nv, _ptr(fb), _ptr(u), float(rtol), int(maxit), nu_pre,
                                        nu_post,
                                        iters.ctypes.data_as(_c_ip), relres.ctypes.data_as(_c_dp),
                                        status.ctypes.data_as(_c_ip), hist.ctypes.data_as(_c_dp) if history else None)
        _check(st, allow=(MG_OK, MG_NOT_CONVERGED, MG_ERR_DIVERGED))
        ms = C.c_double()
        _check(load_library().mg_rb_last_solve_ms(self._h, C.byref(ms)))
        return SolveResult(u=list(u), iters=iters, relres=relres, status=status, history=hist, ms=ms.value)


class RBAdam:
    """The 18 device weights of one red-black level's stack and their Adam state (FP64)."""

    def __init__(self, phi):
        self.phi = torch.tensor(np.asarray(phi, dtype=np.float64).reshape(-1), device="cuda")
        self.m = torch.zeros(RB_WEIGHTS, dtype=torch.float64, device="cuda")
        self.v = torch.zeros(RB_WEIGHTS, dtype=torch.float64, device="cuda")
        self.t = 0


def rb_alpha_step(h: RedBlack, level: int, state: RBAdam, k: Sequence[int], f: torch.Tensor, u0: torch.Tensor,
                  u_star: torch.Tensor, opts: Optional["TrainOptions"] = None) -> AlphaResult:
    """One Algorithm 2 step of a red-black level's stack (mg_rb_alpha_step): f, u0, u_star [B, N, N]."""
    opts = opts or TrainOptions(precision=0)
    N = h.level_n(level)
    f, u0, us = (_dev_f64(x).reshape(-1, N, N) for x in (f, u0, u_star))
    B = f.shape[0]
    if not (len(k) == u0.shape[0] == us.shape[0] == B):
        raise ValueError(f"need {B} entries of k, f, u0 and u_star")
    kk = np.ascontiguousarray(np.asarray(k, dtype=np.int32))
    o = opts.to_c()
    t = state.t + 1 if opts.apply_update else max(state.t, 1)
    loss = C.c_double()
    losses = np.zeros(B, dtype=np.float64)
    grad = np.zeros(RB_WEIGHTS, dtype=np.float64)
    _check(load_library().mg_rb_alpha_step(h._h, level, _ptr(state.phi), _ptr(state.m), _ptr(state.v), t, B,
                                           kk.ctypes.data_as(_c_ip), _ptr(f), _ptr(u0), _ptr(us), C.byref(o),
                                           C.byref(loss), losses.ctypes.data_as(_c_dp), grad.ctypes.data_as(_c_dp)))
    if opts.apply_update:
        state.t = t
    return AlphaResult(loss=loss.value, losses=losses, grad=grad)
