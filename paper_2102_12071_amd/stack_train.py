"""Adaptive training (Algorithm 2) of the paper's constant-coefficient
alpha-CNN smoothers, H = f5(f4(f3(f2(f1)))) + f6 per level (section 5, full
coarsening), for one problem, on the GPU with the library's own kernels
(mg_stack_alpha_step), and their evaluation.

As in the paper the smoothers are trained per problem (one rotated
anisotropic operator, theta and eps fixed): stage s trains the stack of grid
size n_s = 2^(s+2) - 1 (7, 15, 31, 63 over a 3 x 3 coarsest grid) on Q
instances {A, f, u0, u*} of that size, with f ~ U(-1, 1) per node, u0 ~ N(0, 1)
and u* the exact solution (FP64 FGMRES to 1e-13); the coarse correction is one
V(1,1) cycle of the stacks of the earlier stages (the exact solve in the first
stage).  Each step draws k_b ~ U{1, ..., b} per instance.  Optional update
rounds add the errors the current hierarchy leaves after 30 cycles on A u = 0
as instances {A, 0, e, 0} (section 3.3).

Weights are saved normalised to an operator with centre entry 1 (f5 and f6
times the stage's a_C); a level takes them divided by its own a_C, so a stack
serves any level of the problem's Galerkin hierarchy (for these operators
every Galerkin level is the same stencil over 4).

Options beyond the paper's procedure: stages above n = 63 (--finest, with
--max-points capping the instances per stage); --symmetric, H^T after the
coarse correction (the cycle's error propagation is then self-adjoint in the
A inner product); --select growth / stable, keeping a stage's weights by the
power-iteration estimate of its hierarchy's growth per cycle rather than by
the monitored loss alone.  Each committed run records its command, e.g.

    python -m paper_2102_12071_amd.stack_train --theta 1.0471975511965976 --eps 1e-3 --finest 1023 \
        --max-points 200000 --steps 3000 --large-n 1023 --bmax 8 --lr 3e-3 --lr-final 1e-4 \
        --update-rounds 2 --update-steps 600 --symmetric --select stable --max-growth 0.98 \
        --out paper_2102_12071_amd/weights/stack_theta1.047_eps0.001_symmetric.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, Optional

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import mg_inputs  # noqa: E402
from paper_2102_12071_amd import mgcnn  # noqa: E402
from paper_2102_12071_amd.alpha_train import stage_sizes  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def _dev(x) -> torch.Tensor:
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def load_stacks(path: str) -> Dict[int, np.ndarray]:
    """{size: normalised weights [6][3][3]} of a saved training run."""
    return load_stack_run(path)[0]


def load_stack_run(path: str):
    """The stacks of a saved training run and whether they post-smooth with H^T."""
    with open(path) as fh:
        d = json.load(fh)
    stacks = {int(k): np.array(v, dtype=np.float64).reshape(6, 3, 3) for k, v in d["stacks"].items()}
    return stacks, bool(d.get("symmetric", False))


class StackStage:
    """The instances of one stage and the three contexts of its step."""

    def __init__(self, n: int, theta: float, eps: float, Q: int, stacks: Dict[int, np.ndarray], seed: int,
                 coarsest: int = 3, inject: Optional[list] = None, symmetric: bool = False):
        self.symmetric = symmetric
        rng = np.random.default_rng([seed, n, 2])
        self.n = n
        A = mgcnn.stencil_q1_rotated(n, theta, eps)
        self.f = [_dev(rng.uniform(-1.0, 1.0, (n, n))) for _ in range(Q)]
        self.u0 = [_dev(rng.normal(size=(n, n))) for _ in range(Q)]
        if inject:
            self.f += [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in inject]
            self.u0 += list(inject)
        self.Q = len(self.f)
        fp64 = mgcnn.Options(precision=mgcnn.PREC_FP64, coarsest_n=coarsest)
        self.top = mgcnn.Context([A] * self.Q, fp64)
        res = self.top.solve_fgmres(self.f, 1e-13, 3000, restart=60)
        if not (res.relres <= 1e-12).all():
            raise RuntimeError("exact solutions of the training set did not converge")
        self.u_star = res.u
        self.a_centre = float(self.top.stencil(0, 0)[4].mean())
        A1 = self.top.stencil(0, 1)
        if not stage_sizes((n - 1) // 2, coarsest):  # the level below is the coarsest: its exact solve
            self.coarse = mgcnn.Context([A1] * self.Q, fp64)
            self.coarse_t = self.coarse
        else:
            opt = mgcnn.Options(precision=mgcnn.PREC_FP64, coarsest_n=coarsest, smoother=mgcnn.SMOOTHER_STACK)
            self.coarse = mgcnn.Context([A1] * self.Q, opt)
            self.coarse.set_stacks(stacks, symmetric=symmetric)
            if symmetric:  # a symmetric cycle is its own transpose
                self.coarse_t = self.coarse
            else:
                self.coarse_t = mgcnn.Context([A1] * self.Q, opt)
                self.coarse_t.set_stacks(stacks, transpose=True)
        self.rng = np.random.default_rng([seed, n, 1])

    def step(self, state: mgcnn.StackAdam, opts: mgcnn.TrainOptions, bmax: int):
        k = self.rng.integers(1, bmax + 1, self.Q)
        return mgcnn.stack_alpha_step(self.top, self.coarse, self.coarse_t, state, k, self.f, self.u0, self.u_star,
                                      opts, self.symmetric)

    def monitor(self, state: mgcnn.StackAdam, k: int) -> float:
        o = mgcnn.TrainOptions(precision=0, apply_update=0)
        return mgcnn.stack_alpha_step(self.top, self.coarse, self.coarse_t, state, [k] * self.Q, self.f, self.u0,
                                      self.u_star, o, self.symmetric).loss

    def close(self):
        for c in {id(x): x for x in (self.top, self.coarse, self.coarse_t)}.values():
            c.close()


def worst_errors(n: int, theta: float, eps: float, Q: int, stacks: Dict[int, np.ndarray], seed: int,
                 cycles: int = 30, coarsest: int = 3, rnd: int = 0, symmetric: bool = False):
    """The errors the current hierarchy of the stage reduces worst: cycles on
    A u = 0 from random u0, scaled to the norm of a N(0, 1) vector; and the
    largest per-cycle growth over the last third (a power-iteration estimate
    of the cycle's spectral radius)."""
    rng = np.random.default_rng([seed, n, 3, rnd])
    A = mgcnn.stencil_q1_rotated(n, theta, eps)
    ctx = mgcnn.Context([A] * Q, mgcnn.Options(precision=mgcnn.PREC_FP64, coarsest_n=coarsest,
                                               smoother=mgcnn.SMOOTHER_STACK))
    ctx.set_stacks(stacks, symmetric=symmetric)
    u = [_dev(rng.normal(size=(n, n))) for _ in range(Q)]
    zero = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(Q)]
    tail = max(cycles // 3, 1)
    for c in range(cycles):
        if c == cycles - tail:
            mid = [float(x.norm()) for x in u]
        ctx.vcycle(zero, u)
    ctx.close()
    growth = max((float(x.norm()) / max(a, 1e-300)) ** (1.0 / tail) for x, a in zip(u, mid))
    return [x * (n / max(float(x.norm()), 1e-300)) for x in u], growth


def _run_stage(stage: StackStage, w0: np.ndarray, steps: int, lr: float, lr_final: float, bmax: int, log,
               growth_of=None, max_growth: Optional[float] = None):
    """Adam from the normalised weights w0.  Keeps the weights of the lowest monitored loss at
    k = bmax; with growth_of (normalised weights -> the stage hierarchy's estimated growth per
    cycle): of the smallest growth (rounded to 0.01; the loss breaks ties), or, with max_growth,
    of the lowest loss among those whose growth is below max_growth (else the smallest growth)."""
    w_level = np.array(w0, dtype=np.float64).reshape(6, 3, 3)
    w_level[4:] /= stage.a_centre  # the trained level's own scale (f5, f6 carry H ~ 1 / a_C)
    state = mgcnn.StackAdam(w_level)

    def normalised(phi):
        w = phi.cpu().numpy().reshape(6, 3, 3).copy()
        w[4:] *= stage.a_centre
        return w

    def score(m, phi):
        if growth_of is None:
            return (m,)
        g = growth_of(normalised(phi))
        if max_growth is not None:
            return (0, m) if g < max_growth else (1, g)
        return (round(g, 2), m)

    m0 = stage.monitor(state, bmax)
    best = (score(m0, state.phi), m0, state.phi.clone())
    start = m0
    every = max(steps // 10, 1)
    for s in range(steps):
        a = s / max(steps - 1, 1)
        o = mgcnn.TrainOptions(precision=0, lr=lr * (lr_final / lr) ** a)
        try:
            stage.step(state, o, bmax)
        except mgcnn.MGError as e:  # a diverging step leaves the weights unchanged: stop the stage
            log(f"  n={stage.n} step {s}: {e}")
            break
        if (s + 1) % every == 0 or s + 1 == steps:
            m = stage.monitor(state, bmax)
            sc = score(m, state.phi)
            if sc < best[0]:
                best = (sc, m, state.phi.clone())
            log(f"  n={stage.n} step {s + 1}: monitor loss (k={bmax}) {m:.4e}, score {sc} (best {best[0]})")
    return normalised(best[2]), start, best[1]


def train(theta: float, eps: float, finest: int = 63, Q: int = 50, steps: int = 400, lr: float = 1e-3,
          lr_final: Optional[float] = None, bmax: int = 4, seed: int = 0, coarsest: int = 3,
          update_rounds: int = 0, update_steps: int = 200, warm: bool = False, max_points: int = 0,
          steps_large: Optional[int] = None, large_n: int = 63, symmetric: bool = False, select: str = "loss",
          max_growth: float = 0.98, log=print):
    """Stages from the coarsest up.  warm: a stage starts from the previous stage's weights (the
    operator is the same up to scale on every level) instead of the damped-Jacobi initialisation;
    max_points: at most that many grid points per stage (Q shrinks on large stages, at least 4);
    stages above large_n take steps_large steps and no update rounds."""
    lr_final = lr if lr_final is None else lr_final
    steps_large = steps if steps_large is None else steps_large
    cap = max_growth if select == "stable" else None
    stacks: Dict[int, np.ndarray] = {}
    records = []
    qn = lambda n: max(4, min(Q, max_points // (n * n))) if max_points else Q
    sizes = stage_sizes(finest, coarsest)

    def growth_fn(n):
        if select == "loss":
            return None
        return lambda w: worst_errors(n, theta, eps, min(4, qn(n)), {**{m: s for m, s in stacks.items() if m < n},
                                                                     n: w}, seed, coarsest=coarsest,
                                      symmetric=symmetric)[1]

    def stage(n, prev):
        t0 = time.time()
        st = StackStage(n, theta, eps, qn(n), stacks, seed, coarsest, symmetric=symmetric)
        w0 = stacks[prev] if (warm and prev is not None) else mg_inputs.stack_init(seed + n)
        w, start, end = _run_stage(st, w0, steps if n <= large_n else steps_large, lr, lr_final, bmax, log,
                                   growth_fn(n), cap)
        st.close()
        stacks[n] = w
        _, growth = worst_errors(n, theta, eps, min(8, qn(n)), stacks, seed, coarsest=coarsest, symmetric=symmetric)
        records.append({"stage_n": n, "instances": st.Q, "loss_start": start, "loss_end": end, "growth": growth,
                        "seconds": round(time.time() - t0, 3)})
        log(json.dumps(records[-1]))

    # the stages up to large_n, then the update rounds on them, then the larger stages
    prev = None
    for n in [m for m in sizes if m <= large_n]:
        stage(n, prev)
        prev = n
    for rnd in range(update_rounds):
        for n in [m for m in sizes if m <= large_n]:
            t0 = time.time()
            inject, before = worst_errors(n, theta, eps, max(2, qn(n) // 2), stacks, seed, coarsest=coarsest,
                                          rnd=rnd + 1, symmetric=symmetric)
            lower = {m: s for m, s in stacks.items() if m < n}
            st = StackStage(n, theta, eps, qn(n), lower, seed + 100 * (rnd + 1), coarsest, inject, symmetric)
            w, start, end = _run_stage(st, stacks[n], update_steps, lr_final, lr_final, bmax, log, growth_fn(n),
                                       cap)
            st.close()
            stacks[n] = w
            _, after = worst_errors(n, theta, eps, min(8, qn(n)), stacks, seed, coarsest=coarsest, symmetric=symmetric)
            records.append({"update_round": rnd, "stage_n": n, "growth_before": before, "growth_after": after,
                            "loss_start": start, "loss_end": end, "seconds": round(time.time() - t0, 3)})
            log(json.dumps(records[-1]))
    for n in [m for m in sizes if m > large_n]:
        stage(n, prev)
        prev = n
    return stacks, records


def evaluate(stacks: Dict[int, np.ndarray], n: int, theta: float, eps: float, tol: float = 1e-8,
             maxit: int = 20000, coarsest: int = 7, seed: int = 0, symmetric: bool = False) -> dict:
    """Iterations and solve time to tol: V(1,1) with the stacks against damped Jacobi (mixed precision)."""
    A = mgcnn.stencil_q1_rotated(n, theta, eps)
    f = _dev(mg_inputs.rhs_uniform(n, seed))
    out = {}
    for name, sm in (("alpha_stack", mgcnn.SMOOTHER_STACK), ("jacobi", mgcnn.SMOOTHER_JACOBI)):
        ctx = mgcnn.Context([A], mgcnn.Options(smoother=sm, coarsest_n=coarsest))
        if sm == mgcnn.SMOOTHER_STACK:
            ctx.set_stacks(stacks, symmetric=symmetric)
        ctx.solve([f], tol, maxit)  # warm-up (graph capture)
        r = ctx.solve([f], tol, maxit)
        out[name] = {"iters": int(r.iters[0]), "status": int(r.status[0]), "ms": round(r.ms, 3)}
        ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--theta", type=float, required=True)
    ap.add_argument("--eps", type=float, required=True)
    ap.add_argument("--finest", type=int, default=63)
    ap.add_argument("--instances", type=int, default=50)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=None)
    ap.add_argument("--bmax", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--update-rounds", type=int, default=0)
    ap.add_argument("--update-steps", type=int, default=200)
    ap.add_argument("--warm", action="store_true", help="start each stage from the previous stage's weights")
    ap.add_argument("--max-points", type=int, default=0, help="grid points per stage (0: Q instances always)")
    ap.add_argument("--steps-large", type=int, default=None, help="steps of the stages above --large-n")
    ap.add_argument("--large-n", type=int, default=63)
    ap.add_argument("--symmetric", action="store_true", help="post-smooth with H^T (the symmetric cycle)")
    ap.add_argument("--select", choices=["loss", "growth", "stable"], default="loss",
                    help="keep a stage's weights of the lowest monitored loss, of the smallest growth estimate, "
                         "or of the lowest loss among those with growth below --max-growth")
    ap.add_argument("--max-growth", type=float, default=0.98)
    ap.add_argument("--eval", type=int, nargs="*", default=[63, 255, 1023])
    ap.add_argument("--out", required=True)
    a = ap.parse_args()

    def log(line):
        print(line, flush=True)

    mgcnn.load_library()
    stacks, records = train(a.theta, a.eps, a.finest, a.instances, a.steps, a.lr, a.lr_final, a.bmax, a.seed,
                            update_rounds=a.update_rounds, update_steps=a.update_steps, warm=a.warm,
                            max_points=a.max_points, steps_large=a.steps_large, large_n=a.large_n,
                            symmetric=a.symmetric, select=a.select, max_growth=a.max_growth, log=log)
    for n in a.eval:
        r = evaluate(stacks, n, a.theta, a.eps, symmetric=a.symmetric)
        records.append({"eval": {"n": n, "theta": a.theta, "eps": a.eps}, **r})
        log(json.dumps(records[-1]))
    cmd = "python -m paper_2102_12071_amd.stack_train " + " ".join(sys.argv[1:])
    with open(a.out, "w") as fh:
        json.dump({"command": cmd, "device": "one MI355X", "problem": {"theta": a.theta, "eps": a.eps},
                   "symmetric": a.symmetric, "select": a.select, "max_growth": a.max_growth,
                   "note": "weights [6][3][3] per trained size, normalised to a_C = 1 (f5 and f6 times a_C); "
                           "eval: V(1,1) to 1e-8 over a 7 x 7 coarsest grid, mixed precision",
                   "stacks": {str(n): w.reshape(-1).tolist() for n, w in stacks.items()},
                   "records": records}, fh, indent=1)


if __name__ == "__main__":
    main()
