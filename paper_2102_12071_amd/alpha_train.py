"""Adaptive training of per-level smoother networks (Algorithm 2) on the GPU,
with the library's own kernels (mg_alpha_step), and their evaluation.

Stages run from the second-coarsest level upwards (section 3.3): with a
coarsest grid of 3 x 3, stage s trains the network of grid size n_s = 2^(s+2)
- 1 (7, 15, 31, 63 for a 5-level hierarchy) on Q problems of that size.  The
coarse correction of a stage is one V(1,1) cycle of the hierarchy below,
whose smoothers are the networks of the earlier stages (fixed), or the exact
coarse solve in the first stage.  Each step takes the whole training set with
a fresh k_b ~ U{1, ..., b} per problem.

Training set of a stage (seeded): rotated anisotropic bilinear stencils with
theta ~ U[0, pi) and log10 eps ~ U[-3, 0]; f ~ U(-1, 1) per node; u* the
exact solution (FP64 FGMRES with the multigrid cycle, to 1e-13); u0 ~ N(0, 1).

    python -m paper_2102_12071_amd.alpha_train --steps 400 --out-dir paper_2102_12071_amd/weights
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

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def weight_path(out_dir: str, n: int) -> str:
    return os.path.join(out_dir, f"alpha_n{n}.bin")


def stage_sizes(finest: int, coarsest: int = 3):
    """Grid sizes of the trained levels, coarse to fine."""
    sizes = []
    m = finest
    while m > coarsest:
        sizes.append(m)
        m = (m - 1) // 2
    return sizes[::-1]


def stage_stencils(n: int, Q: int, seed: int):
    """The Q rotated anisotropic stencils of the stage on size n (seeded)."""
    rng = np.random.default_rng([seed, n])
    theta = rng.uniform(0.0, math.pi, Q)
    eps = 10.0 ** rng.uniform(-3.0, 0.0, Q)
    return [mgcnn.stencil_q1_rotated(n, float(t), float(e)) for t, e in zip(theta, eps)]


class Stage:
    """The training set of one stage and the three contexts of its step.

    inject: errors that the current hierarchy fails to reduce (one per
    stencil, from inject_errors); each adds the instance {A, f = 0, u0 = e,
    u* = 0}, whose loss is the norm of k cycles' error propagation applied to e."""

    def __init__(self, n: int, Q: int, nets: Dict[int, mgcnn.Net], seed: int, coarsest: int = 3,
                 inject: Optional[list] = None):
        rng = np.random.default_rng([seed, n, 2])
        self.n = n
        As = stage_stencils(n, Q, seed)
        fp64 = mgcnn.Options(precision=mgcnn.PREC_FP64, coarsest_n=coarsest)
        self.f = [torch.tensor(rng.uniform(-1.0, 1.0, (n, n)), dtype=torch.float64, device="cuda")
                  for _ in range(Q)]
        self.u0 = [torch.tensor(rng.normal(size=(n, n)), dtype=torch.float64, device="cuda") for _ in range(Q)]
        if inject:
            As = As + As[:len(inject)]
            self.f += [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in inject]
            self.u0 += list(inject)
        self.Q = len(As)
        self.top = mgcnn.Context(As, fp64)
        # exact solutions by FP64 FGMRES with the Jacobi cycle (zero right-hand sides: u* = 0 at once)
        res = self.top.solve_fgmres(self.f, 1e-13, 3000, restart=60)
        if not (res.relres <= 1e-12).all():
            raise RuntimeError("exact solutions of the training set did not converge")
        self.u_star = res.u
        A1 = [self.top.stencil(b, 1) for b in range(self.Q)]
        lower = stage_sizes((n - 1) // 2, coarsest)
        if not lower:  # the coarse problem is the coarsest grid: Psi_c is the exact solve
            self.coarse = mgcnn.Context(A1, fp64)
            self.coarse_t = self.coarse
        else:
            cnn = mgcnn.Options(precision=mgcnn.PREC_FP64, coarsest_n=coarsest, smoother=mgcnn.SMOOTHER_CNN)
            self.coarse = mgcnn.Context(A1, cnn)
            self.coarse.infer_levels(nets)
            self.coarse_t = mgcnn.Context(A1, cnn)
            for b in range(self.Q):
                for l in range(self.coarse.num_levels(b) - 1):
                    W = self.coarse.smoother(b, l)
                    self.coarse_t.set_smoother(b, l, mgcnn.smoother_transpose(self.coarse.stencil(b, l), W))
        self.rng = np.random.default_rng([seed, n, 1])

    def step(self, net: mgcnn.Net, opts: mgcnn.TrainOptions, bmax: int):
        k = self.rng.integers(1, bmax + 1, self.Q)
        return mgcnn.alpha_step(self.top, self.coarse, self.coarse_t, net, k, self.f, self.u0, self.u_star, opts)

    def monitor(self, net: mgcnn.Net, k: int) -> float:
        """The loss with every problem at k cycles, no update (a steady view of the noisy training loss)."""
        o = mgcnn.TrainOptions(precision=0, apply_update=0)
        return mgcnn.alpha_step(self.top, self.coarse, self.coarse_t, net, [k] * self.Q, self.f, self.u0,
                                self.u_star, o).loss

    def close(self):
        for c in (self.top, self.coarse, self.coarse_t):
            c.close()


def inject_errors(n: int, Q: int, nets: Dict[int, mgcnn.Net], seed: int, cycles: int = 30, coarsest: int = 3,
                  rnd: int = 0):
    """The paper's update of trained smoothers (section 3.3): the current
    hierarchy of the stage (its network on top, the earlier ones below)
    applied to A u = 0 from a random u0 for some cycles; what is left, u_k,
    is the error it reduces worst (or amplifies).  Returns the u_k scaled to
    the norm of a N(0, 1) vector, and the largest per-cycle growth over the
    last third of the cycles among the stencils, a power-iteration estimate
    of the cycle's spectral radius."""
    rng = np.random.default_rng([seed, n, 3, rnd])
    As = stage_stencils(n, Q, seed)
    ctx = mgcnn.Context(As, mgcnn.Options(precision=mgcnn.PREC_FP64, coarsest_n=coarsest,
                                          smoother=mgcnn.SMOOTHER_CNN))
    ctx.infer_levels(nets)
    u = [torch.tensor(rng.normal(size=(n, n)), dtype=torch.float64, device="cuda") for _ in range(Q)]
    zero = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for _ in range(Q)]
    tail = max(cycles // 3, 1)
    for c in range(cycles):
        if c == cycles - tail:
            mid = [float(x.norm()) for x in u]
        ctx.vcycle(zero, u)
    ctx.close()
    growth = max((float(x.norm()) / max(a, 1e-300)) ** (1.0 / tail) for x, a in zip(u, mid))
    out = [x * (n / max(float(x.norm()), 1e-300)) for x in u]
    return out, growth


def train(finest: int = 63, Q: int = 50, steps: int = 400, lr: float = 1e-3, bmax: int = 4, seed: int = 0,
          init: Optional[str] = None, coarsest: int = 3, lr_final: Optional[float] = None,
          init_dir: Optional[str] = None, log=print) -> Dict[int, mgcnn.Net]:
    """Runs every stage; returns the trained network of each level size.  The
    learning rate decays geometrically from lr to lr_final over a stage; a
    stage keeps the parameters with the lowest loss at k = b cycles on its
    training set (checked every 100 steps, and at the start)."""
    nets: Dict[int, mgcnn.Net] = {}
    lr_final = lr if lr_final is None else lr_final
    for n in stage_sizes(finest, coarsest):
        t0 = time.perf_counter()
        stage = Stage(n, Q, nets, seed, coarsest)
        net = mgcnn.Net()
        if init_dir:
            net.load(weight_path(init_dir, n))  # continue from this level's network
        elif init:
            net.load(init)
        else:
            net.set(mg_inputs.cnn_init(seed + n).astype(np.float32))  # zero last layer: damped Jacobi
        first = stage.monitor(net, bmax)
        best, best_params = first, net.get()
        for s in range(steps):
            rate = lr * (lr_final / lr) ** (s / max(steps - 1, 1))
            r = stage.step(net, mgcnn.TrainOptions(lr=rate, precision=0), bmax)
            if s % 100 == 99 or s == steps - 1:
                mon = stage.monitor(net, bmax)
                if mon < best:
                    best, best_params = mon, net.get()
                log(json.dumps({"stage_n": n, "step": s, "loss": r.loss, f"loss_k{bmax}": mon,
                                "lr": rate, "elapsed_s": round(time.perf_counter() - t0, 3)}))
        net.set(best_params)  # the parameters with the lowest loss at k = b cycles
        last = stage.monitor(net, bmax)
        stage.close()
        nets[n] = net
        _, growth = inject_errors(n, Q, nets, seed + 1, 30, coarsest)
        log(json.dumps({"stage_n": n, "done": True, f"loss_k{bmax}_start": first, f"loss_k{bmax}_end": last,
                        "growth": growth, "seconds": round(time.perf_counter() - t0, 3)}))
    return nets


def update(nets: Dict[int, mgcnn.Net], Q: int = 50, steps: int = 400, lr: float = 3e-4, bmax: int = 4,
           seed: int = 0, rounds: int = 1, cycles: int = 30, coarsest: int = 3, log=print) -> None:
    """Rounds of the paper's smoother update: per stage, coarse to fine, inject
    the errors the current hierarchy reduces worst and retrain the stage's
    network from its current weights on the augmented set."""
    for rnd in range(rounds):
        for n in sorted(nets):
            t0 = time.perf_counter()
            inj, growth = inject_errors(n, Q, nets, seed, cycles, coarsest, rnd)
            stage = Stage(n, Q, {m: v for m, v in nets.items() if m < n}, seed, coarsest, inject=inj)
            first = stage.monitor(nets[n], bmax)
            best, best_params = first, nets[n].get()
            for s in range(steps):
                stage.step(nets[n], mgcnn.TrainOptions(lr=lr, precision=0), bmax)
                if s % 100 == 99 or s == steps - 1:
                    mon = stage.monitor(nets[n], bmax)
                    if mon < best:
                        best, best_params = mon, nets[n].get()
            nets[n].set(best_params)
            last = stage.monitor(nets[n], bmax)
            stage.close()
            _, after = inject_errors(n, Q, nets, seed + 1, cycles, coarsest, rnd)
            log(json.dumps({"update_round": rnd, "stage_n": n, "growth_before": growth, "growth_after": after,
                            f"loss_k{bmax}_start": first, f"loss_k{bmax}_end": last,
                            "seconds": round(time.perf_counter() - t0, 3)}))


def load_nets(out_dir: str = WEIGHTS, finest: int = 63, coarsest: int = 3) -> Dict[int, mgcnn.Net]:
    nets = {}
    for n in stage_sizes(finest, coarsest):
        net = mgcnn.Net()
        net.load(weight_path(out_dir, n))
        nets[n] = net
    return nets


def evaluate(nets: Dict[int, mgcnn.Net], n: int, theta: float, eps: float, tol: float = 1e-8,
             maxit: int = 20000, coarsest: int = 3, hf: Optional[mgcnn.Net] = None, seed: int = 0,
             domain: str = "square") -> dict:
    """Iterations and solve time to tol of V(1,1) with the per-level alpha-CNN
    smoothers, damped Jacobi, and (hf given) the one network trained on the
    high-frequency loss, on one rotated anisotropic problem (domain: 'square',
    'lshape' or 'cylinder', zero Dirichlet values on the removed nodes)."""
    A = mgcnn.stencil_q1_rotated(n, theta, eps)
    m = mg_inputs.domain_mask(n, domain)
    if domain != "square":
        A = mgcnn.stencil_mask(A, torch.tensor(m, device="cuda"))
    f = torch.tensor(mg_inputs.rhs_uniform(n, seed) * m, dtype=torch.float64, device="cuda")
    out = {}
    for name in ("alpha_cnn", "jacobi") + (("hf_cnn",) if hf is not None else ()):
        sm = mgcnn.SMOOTHER_JACOBI if name == "jacobi" else mgcnn.SMOOTHER_CNN
        ctx = mgcnn.Context([A], mgcnn.Options(smoother=sm, coarsest_n=coarsest))
        if name == "alpha_cnn":
            ctx.infer_levels(nets)
        elif name == "hf_cnn":
            ctx.infer(hf)
        ctx.solve([f], tol, maxit)  # warm-up (graph capture)
        r = ctx.solve([f], tol, maxit)
        out[name] = {"iters": int(r.iters[0]), "status": int(r.status[0]), "ms": round(r.ms, 3)}
        ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--finest", type=int, default=63)
    ap.add_argument("--instances", type=int, default=50)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=None, help="learning rate at the end of a stage (default: lr)")
    ap.add_argument("--bmax", type=int, default=4, help="k ~ U{1..bmax} cycles per loss term")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--init", default=None, help="checkpoint to start every stage from (default: damped Jacobi)")
    ap.add_argument("--init-dir", default=None, help="directory of per-level checkpoints each stage continues from")
    ap.add_argument("--update-rounds", type=int, default=0, help="rounds of error injection and retraining")
    ap.add_argument("--update-steps", type=int, default=400)
    ap.add_argument("--update-lr", type=float, default=3e-4)
    ap.add_argument("--load", default=None, help="directory of trained per-level networks to start from")
    ap.add_argument("--out-dir", default=WEIGHTS)
    ap.add_argument("--log", default=None)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    records = []

    def log(line):
        print(line, flush=True)
        records.append(json.loads(line))

    if args.load:
        nets = load_nets(args.load, args.finest)
    else:
        nets = train(args.finest, args.instances, args.steps, args.lr, args.bmax, args.seed, args.init,
                     lr_final=args.lr_final, init_dir=args.init_dir, log=log)
    if args.update_rounds:
        update(nets, args.instances, args.update_steps, args.update_lr, args.bmax, args.seed, args.update_rounds,
               log=log)
    os.makedirs(args.out_dir, exist_ok=True)
    for n, net in nets.items():
        net.save(weight_path(args.out_dir, n))
    hf = mgcnn.Net()
    hf.load(os.path.join(WEIGHTS, "cnn_hf.bin"))
    for n, theta, eps, dom in ((63, math.pi / 6, 0.01, "square"), (255, math.pi / 3, 1e-3, "square"),
                               (1023, math.pi / 3, 1e-3, "square"), (1023, 0.0, 1e-2, "square"),
                               (1023, math.pi / 4, 0.1, "square"), (1023, 2.0, 1.0, "square"),
                               (1023, math.pi / 4, 0.01, "lshape"), (1023, math.pi / 4, 0.01, "cylinder")):
        log(json.dumps({"eval": {"n": n, "theta": theta, "eps": eps, "domain": dom},
                        **evaluate(nets, n, theta, eps, hf=hf, domain=dom)}))
    if args.log:
        with open(args.log, "w") as fh:
            json.dump(records, fh, indent=1)


if __name__ == "__main__":
    main()
