"""Trains the stencil-to-smoother network on the GPU with the library's own
training kernels (mg_train_step) and writes a checkpoint.

Batches (seeded): each problem draws n in {31, 63}, theta ~ U[0, pi),
log10 eps ~ U[-3, 0]; half of the problems are the rotated anisotropic
bilinear stencil, the other half variable-coefficient five-point stencils of
a = exp(g) (g a Gaussian random field) built on a grid 1, 2 or 4 times finer
and Galerkin-coarsened to n, so that the network sees the coarse-level
stencils it is applied to.  Each problem gets J = 16 unit vectors drawn from
a pool of high-frequency vectors for its size.  With --mask-frac, that
fraction of the problems is cut to a random non-square domain (a disk or a
corner rectangle removed, Dirichlet values there).  The stencils are
generated, masked and coarsened on the device by the library.

    python -m paper_2102_12071_amd.train --steps 3000 --out paper_2102_12071_amd/weights/cnn_hf.bin
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import mg_inputs  # noqa: E402
from paper_2102_12071_amd import mgcnn  # noqa: E402

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "cnn_hf.bin")


class BatchMaker:
    def __init__(self, batch: int, nvec: int, sizes=(31, 63), pool: int = 2048, fields: int = 96,
                 var_frac: float = 0.5, seed: int = 0, mask_frac: float = 0.0):
        self.batch, self.nvec, self.sizes, self.var_frac, self.seed = batch, nvec, sizes, var_frac, seed
        self.mask_frac = mask_frac
        self.pools = {n: torch.tensor(mg_inputs.hf_pool(n, pool, seed + 1000 + n), dtype=torch.float32,
                                      device="cuda") for n in sizes}
        # log-normal coefficient fields on the (n_f + 1)^2 cells of grids n_f = n, 2n+1, 4n+3
        rng = np.random.default_rng(seed + 7)
        self.fields = {}
        for n in sizes:
            for level in range(3):
                nf = n
                for _ in range(level):
                    nf = 2 * nf + 1
                fs = []
                for q in range(fields):
                    length = 10.0 ** rng.uniform(math.log10(0.05), math.log10(0.5))
                    a = mg_inputs.lognormal_coefficient(nf, length, 1.0, int(rng.integers(2 ** 31 - 1)))
                    fs.append(torch.tensor(a, dtype=torch.float64, device="cuda"))
                self.fields[(n, level)] = fs

    def make(self, step: int):
        ns, theta, eps = mg_inputs.training_draws(self.batch, self.seed * 1000003 + step, self.sizes)
        rng = np.random.default_rng([self.seed, step, 17])
        stencils, vectors = [], []
        for q in range(self.batch):
            n = int(ns[q])
            masked = self.mask_frac > 0 and rng.uniform() < self.mask_frac
            if rng.uniform() < self.var_frac:
                level = int(rng.integers(0, 3))
                a = self.fields[(n, level)][int(rng.integers(len(self.fields[(n, level)])))]
                A = mgcnn.stencil_cellavg5(a)
            else:
                # a masked rotated problem is built 1, 2 or 4 times finer and coarsened too
                level = int(rng.integers(0, 3)) if masked else 0
                nf = n
                for _ in range(level):
                    nf = 2 * nf + 1
                A = mgcnn.stencil_q1_rotated(nf, float(theta[q]), float(eps[q]))
            if masked:
                # a non-square domain: Dirichlet rows cut into the stencil field along curved and
                # corner boundaries, and (after coarsening) their Galerkin images, rows the
                # square's outer boundary never shows
                m = torch.tensor(mg_inputs.random_domain_mask(A.shape[1], rng), device="cuda")
                A = mgcnn.stencil_mask(A, m)
            for _ in range(level):
                A = mgcnn.galerkin(A)
            idx = torch.tensor(rng.integers(0, self.pools[n].shape[0], self.nvec), device="cuda")
            stencils.append(A)
            vectors.append(self.pools[n].index_select(0, idx).contiguous())
        return stencils, vectors


def evaluate(net, n=255, theta=math.pi / 3, eps=1e-3, tol=1e-8, maxit=20000):
    """Iterations to tol of the CNN and Jacobi V(1,1) on one rotated problem."""
    A = mgcnn.stencil_q1_rotated(n, theta, eps)
    f = torch.tensor(mg_inputs.rhs_uniform(n, 0), dtype=torch.float64, device="cuda")
    out = {}
    for name, sm in (("cnn", mgcnn.SMOOTHER_CNN), ("jacobi", mgcnn.SMOOTHER_JACOBI)):
        ctx = mgcnn.Context([A], mgcnn.Options(smoother=sm))
        if sm == mgcnn.SMOOTHER_CNN:
            ctx.infer(net)
        r = ctx.solve([f], tol, maxit)
        out[name] = {"iters": int(r.iters[0]), "status": int(r.status[0]), "ms": r.ms}
        ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--nvec", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", type=int, default=1, help="1: BF16 on MFMA (default); 0: FP32")
    ap.add_argument("--var-frac", type=float, default=0.5)
    ap.add_argument("--mask-frac", type=float, default=0.0,
                    help="fraction of problems on a random non-square domain (masked stencils)")
    ap.add_argument("--eval-every", type=int, default=500)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--log", default=None)
    ap.add_argument("--resume", default=None)
    args = ap.parse_args()

    torch.cuda.set_device(0)
    net = mgcnn.Net()
    if args.resume:
        net.load(args.resume)
    else:
        net.set(mg_inputs.cnn_init(args.seed).astype(np.float32))
    maker = BatchMaker(args.batch, args.nvec, var_frac=args.var_frac, seed=args.seed, mask_frac=args.mask_frac)
    held = maker.make(10 ** 6)
    opts = mgcnn.TrainOptions(lr=args.lr, precision=args.precision)
    no_update = mgcnn.TrainOptions(lr=args.lr, precision=args.precision, apply_update=0)
    log = []
    t0 = time.perf_counter()
    for step in range(args.steps + 1):
        if step % args.eval_every == 0 or step == args.steps:
            hl, _ = net.train_step(*held, opts=no_update)
            rec = {"step": step, "heldout_loss": hl, "elapsed_s": time.perf_counter() - t0}
            if step % (2 * args.eval_every) == 0 or step == args.steps:
                rec["eval_n255"] = evaluate(net)
            log.append(rec)
            print(json.dumps(rec), flush=True)
        if step == args.steps:
            break
        st, vs = maker.make(step)
        loss, _ = net.train_step(st, vs, opts=opts, want_loss=(step % 50 == 0))
        if step % 50 == 0:
            print(json.dumps({"step": step, "loss": loss, "elapsed_s": time.perf_counter() - t0}), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    net.save(args.out)
    if args.log:
        with open(args.log, "w") as fh:
            json.dump(log, fh, indent=1)
    print(f"saved {args.out}", flush=True)


if __name__ == "__main__":
    main()
