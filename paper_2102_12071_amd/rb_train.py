"""Adaptive training (Algorithm 2) of the red-black smoothers H = f2(f1), one
per level (section 6: red-black coarsening, two convolution layers), for one
problem, on the GPU with the library's own kernels (mg_rb_alpha_step), and
their evaluation against damped Jacobi with the same coarsening.

Stage s = 1 .. L-1 trains level L-1-s of the training hierarchy (an n x n
rotated anisotropic operator, L red-black levels down to a full 7 x 7 grid
solved directly) on Q instances of that level's operator: f ~ U(-1, 1) and
u0 ~ N(0, 1) on the level's points, u* the exact solution (the hierarchy's own
FP64 solve from that level to 1e-13).  The coarse correction is one V(1,1)
cycle of the levels below, which carry the earlier stages' weights; each
step draws k_b ~ U{1, ..., b} per instance; a stage keeps the weights with
the lowest monitored loss at k = b.  Initialisation (the paper starts H as
Jacobi; with f2(f1) alone a zero start gets no gradient): f1 = omega / a_C at
the centre, f2 the identity - damped Jacobi at the level's middle node.

A larger problem's hierarchy takes level l's weights where the training
hierarchy has a smoothing level at the same depth (the interior stencils of
equal depth are equal: the Galerkin products act locally); deeper levels take
the deepest trained level of their kind (full or checkerboard), with f1
rescaled to their own centre entry (mg_rb_set_smoother's a_ref).  A run is
saved as JSON with its command, e.g.

    python -m paper_2102_12071_amd.rb_train --theta 1.0471975511965976 --eps 1e-3 \\
        --out paper_2102_12071_amd/weights/rb_theta1.047_eps0.001.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Dict, Tuple

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import mg_inputs  # noqa: E402
from paper_2102_12071_amd import mgcnn  # noqa: E402

OMEGA = 2.0 / 3.0


def _dev(x) -> torch.Tensor:
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def levels_for(n: int, coarsest: int = 7) -> int:
    """Red-black levels of an n x n grid down to a full coarsest x coarsest grid."""
    L, N = 1, n
    while N > coarsest:
        L += 2
        N = (N - 1) // 2
    if N != coarsest:
        raise ValueError(f"n = {n} does not coarsen to {coarsest}")
    return L


def point_mask(N: int, kind: str) -> np.ndarray:
    j, i = np.mgrid[0:N, 0:N]
    return np.ones((N, N)) if kind == "full" else ((i + j) % 2 == 0).astype(np.float64)


def middle_centre(h: mgcnn.RedBlack, level: int) -> float:
    """The level's centre entry at its middle node (read back from the library)."""
    offs, field = h.stencil(level)
    kc = int(np.flatnonzero((offs[:, 0] == 0) & (offs[:, 1] == 0))[0])
    N = h.level_n(level)
    return float(field[kc, N // 2, N // 2].item())


def jacobi_weights(a_centre: float) -> np.ndarray:
    w = np.zeros((2, 3, 3))
    w[0, 1, 1] = OMEGA / a_centre
    w[1, 1, 1] = 1.0
    return w


def growth(h: mgcnn.RedBlack, level: int, state: mgcnn.RBAdam, mask: np.ndarray, seed: int, k0: int = 20,
           k1: int = 30, count: int = 4) -> float:
    """The stage hierarchy's error growth per cycle on A u = 0 (the cycle's spectral radius, by power
    iteration): (||E^k1 u0|| / ||E^k0 u0||)^(1 / (k1 - k0)), E the error propagation of one cycle of
    level `level` with the weights of state, u0 ~ N(0, 1), the largest over count starts (the loss of
    Algorithm 2 with f = 0 and u* = 0 is ||E^k u0||)."""
    N = h.level_n(level)
    rng = np.random.default_rng([seed, level, 99])
    u0 = _dev(rng.normal(size=(count, N, N)) * mask)
    zero = torch.zeros_like(u0)
    mon = mgcnn.TrainOptions(precision=0, apply_update=0)
    a = mgcnn.rb_alpha_step(h, level, state, [k0] * count, zero, u0, zero, mon).losses
    b = mgcnn.rb_alpha_step(h, level, state, [k1] * count, zero, u0, zero, mon).losses
    g = [(y / max(x, 1e-300)) ** (1.0 / (k1 - k0)) for x, y in zip(a, b)]
    return float(max(g))


def train(theta: float, eps: float, n: int, Q: int, steps: int, bmax: int, lr: float, lr_final: float, seed: int,
          log=print, max_growth: float = 0.0) -> Tuple[Dict[int, np.ndarray], Dict[int, float], list]:
    L = levels_for(n)
    A = mgcnn.stencil_q1_rotated(n, theta, eps)
    h = mgcnn.RedBlack(A, L)
    weights, centres, records = {}, {}, []
    for s in range(1, L):
        lvl = L - 1 - s
        N, kind, K = h.shapes[lvl]
        rng = np.random.default_rng([seed, lvl])
        mask = point_mask(N, kind)
        f = _dev(rng.uniform(-1.0, 1.0, (Q, N, N)) * mask)
        u0 = _dev(rng.normal(size=(Q, N, N)) * mask)
        ex = h.solve(f, 1e-13, 20000, level=lvl)
        if not (ex.status == 0).all():
            raise RuntimeError(f"level {lvl}: the exact solutions did not converge")
        u_star = torch.stack(ex.u)
        a_mid = middle_centre(h, lvl)
        state = mgcnn.RBAdam(jacobi_weights(a_mid))
        mon = mgcnn.TrainOptions(precision=0, apply_update=0)
        kb = [bmax] * Q

        def monitor() -> float:
            return mgcnn.rb_alpha_step(h, lvl, state, kb, f, u0, u_star, mon).loss

        def score(m):
            # max_growth > 0: the lowest loss among checkpoints whose hierarchy's growth per cycle
            # stays below max_growth, else the smallest growth
            if max_growth <= 0.0:
                return (m,), None
            g = growth(h, lvl, state, mask, seed)
            return ((0, m) if g < max_growth else (1, g)), g

        m0 = monitor()
        (best_key, g0), best_loss, best = score(m0), m0, state.phi.cpu().numpy().copy()
        best_growth = g0
        jacobi_loss = m0
        t0 = time.time()
        for it in range(steps):
            lr_it = lr * (lr_final / lr) ** (it / max(steps - 1, 1))
            k = rng.integers(1, bmax + 1, Q)
            out = mgcnn.rb_alpha_step(h, lvl, state, k, f, u0, u_star,
                                      mgcnn.TrainOptions(lr=lr_it, precision=0, apply_update=1))
            if (it + 1) % 25 == 0 or it == steps - 1:
                m = monitor()
                key, g = score(m)
                if key < best_key:
                    best_key, best_loss, best, best_growth = key, m, state.phi.cpu().numpy().copy(), g
        h.set_smoother(lvl, best)
        weights[lvl] = best.reshape(2, 3, 3)
        centres[lvl] = a_mid
        rec = {"level": lvl, "N": N, "kind": kind, "footprint": K, "a_centre": a_mid, "instances": Q,
               "loss_jacobi_k_b": jacobi_loss, "loss_best_k_b": best_loss, "growth_jacobi": g0,
               "growth_kept": best_growth, "seconds": time.time() - t0}
        records.append(rec)
        gtxt = "" if best_growth is None else f", growth per cycle {g0:.3f} (Jacobi) -> {best_growth:.3f}"
        log(f"stage {s}: level {lvl} ({kind} {N}x{N}, {K}-point operator): loss at k = {bmax} "
            f"{jacobi_loss:.4e} (Jacobi) -> {best_loss:.4e}{gtxt} in {time.time() - t0:.1f} s")
    return weights, centres, records


def install(h: mgcnn.RedBlack, weights: Dict[int, np.ndarray], centres: Dict[int, float], kinds: Dict[int, str]):
    """Every smoothing level of h: the trained level of equal depth, else the deepest trained level of
    the same kind with f1 rescaled to the level's centre entry."""
    deepest = {}
    for l in sorted(weights):
        deepest[kinds[l]] = l
    for l in range(h.num_levels - 1):
        if l in weights:
            h.set_smoother(l, weights[l])
        else:
            src = deepest[h.shapes[l][1]]
            h.set_smoother(l, weights[src], a_ref=centres[src])


def evaluate(weights, centres, kinds, n: int, theta: float, eps: float, tol: float = 1e-8, maxit: int = 20000,
             seed: int = 0) -> dict:
    """Cycles and solve time to tol on the n x n problem: the trained smoothers V(1,1), damped Jacobi
    V(1,1) and V(2,2) (two sweeps per smoothing step: the cost of the two convolutions)."""
    A = mgcnn.stencil_q1_rotated(n, theta, eps)
    f = _dev(mg_inputs.rhs_uniform(n, seed))
    out = {"n": n}
    h = mgcnn.RedBlack(A, levels_for(n))
    for name, nu, learned in (("alpha_cnn", 1, True), ("jacobi", 1, False), ("jacobi_v22", 2, False)):
        for l in range(h.num_levels - 1):
            h.set_smoother(l, None)
        if learned:
            install(h, weights, centres, kinds)
        h.solve(f, tol, 5, nu, nu)  # warm-up
        res = h.solve(f, tol, maxit, nu, nu)
        out[name] = {"iters": int(res.iters[0]), "status": int(res.status[0]), "relres": float(res.relres[0]),
                     "solve_ms": res.ms}
    return out


def load_run(path: str):
    with open(path) as fh:
        d = json.load(fh)
    weights = {int(k): np.array(v, dtype=np.float64).reshape(2, 3, 3) for k, v in d["weights"].items()}
    centres = {int(k): float(v) for k, v in d["a_centre"].items()}
    kinds = {int(k): v for k, v in d["kinds"].items()}
    return weights, centres, kinds, d


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--theta", type=float, default=math.pi / 3)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--n", type=int, default=63, help="training grid (levels down to a 7 x 7 grid)")
    ap.add_argument("--Q", type=int, default=50, help="instances per stage (the paper: 50)")
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--bmax", type=int, default=8)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--max-growth", type=float, default=0.0,
                    help="> 0: keep the lowest-loss checkpoint whose stage hierarchy's growth per cycle (power "
                         "iteration) stays below this, else the smallest growth; 0: the lowest loss")
    ap.add_argument("--eval", type=int, nargs="*", default=[63, 255, 1023])
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    mgcnn.load_library()
    weights, centres, records = train(args.theta, args.eps, args.n, args.Q, args.steps, args.bmax, args.lr,
                                      args.lr_final, args.seed, log=lambda m: print(m, flush=True),
                                      max_growth=args.max_growth)
    kinds = {r["level"]: r["kind"] for r in records}
    evals = []
    for n in args.eval:
        ev = evaluate(weights, centres, kinds, n, args.theta, args.eps)
        print(json.dumps(ev), flush=True)
        evals.append(ev)
    rel = os.path.relpath(os.path.abspath(args.out), ROOT)
    cmd = ("python -m paper_2102_12071_amd.rb_train --theta %r --eps %r --n %d --Q %d --steps %d --bmax %d "
           "--lr %r --lr-final %r --seed %d --max-growth %r --eval %s --out %s"
           % (args.theta, args.eps, args.n, args.Q, args.steps, args.bmax, args.lr, args.lr_final, args.seed,
              args.max_growth, " ".join(str(x) for x in args.eval), rel))
    doc = {"problem": {"theta": args.theta, "eps": args.eps}, "train_n": args.n, "command": cmd,
           "weights": {str(k): v.reshape(-1).tolist() for k, v in weights.items()},
           "a_centre": {str(k): v for k, v in centres.items()}, "kinds": {str(k): v for k, v in kinds.items()},
           "records": records, "evaluations": evals}
    with open(args.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
