"""Benchmark: time to 1e-8 relative residual and unknowns/s of the learned-
smoother multigrid solver against the damped-Jacobi one, on one MI355X.

Workload (one "step" = the whole hot path on one problem): the rotated
anisotropic operator of the paper's section 6 (bilinear nine-point stencil,
theta = pi/3, eps = 1e-3) on a 1023 x 1023 interior grid, RHS U(-1, 1) from
seed 0: stencil generation, Galerkin hierarchy and coarsest inverse,
smoother inference (CNN, BF16 MFMA), and the V(1,1) solve with FP64 outer
refinement to ||f - A u|| / ||f|| <= 1e-8.  The same solve with the damped-
Jacobi smoother is timed beside it.  Inputs are resident in device memory when
a step starts.

Prints one JSON line (see the repository's measurement notes).
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 residual & unknowns/s: CNN-smoother MG vs Jacobi MG, 1 GPU"
WEIGHTS = os.path.join(ROOT, "paper_2102_12071_amd", "weights", "cnn_hf.bin")
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16
# Useful FLOP of the 9 -> 32 -> 32 -> 32 -> 25 network of 3x3 convolutions per grid node
CNN_FLOP_PER_NODE = 2 * 9 * (9 * 32 + 32 * 32 + 32 * 32 + 32 * 25)

# Algorithmic bytes per finest-level node of each timed kernel (mixed
# precision: FP64 stencil and FP64 u/f in the outer residual, FP32 stencil and
# FP32 vectors in the cycle, BF16 5x5 smoother 50 B; the coarse vector of the
# restriction/prolongation counts 1/4 of 4 B).
# The V(1,1) solve runs outer_residual, check, descend, ascend (per level) and
# bottom; the other kernels serve other sweep counts.  descend reads r, the
# smoother (CNN) and the stencil and writes e and r_c; ascend (finest level)
# reads e, e_c, r, the stencil and the smoother and updates u in place.  A
# symmetric stencil (every workload here) is read as five of its nine planes,
# the other four entries being the neighbours' mirrored ones: 40 B in FP64,
# 20 B in FP32 (72 and 36 B for a stencil that is not symmetric).  The step
# kernels of other sweep counts read all nine FP32 planes.
A64_SYM, A32_SYM, A32 = 40, 20, 36
BYTES_PER_NODE = {
    "cnn": {"outer_residual": A64_SYM + 8 + 8 + 4, "descend": 4 + 50 + A32_SYM + 4 + 1,
            "ascend": 4 + 1 + A32_SYM + 4 + 50 + 16,
            "smooth_first": 50 + 4 + 4, "residual_restrict": A32_SYM + 4 + 4 + 1,
            "prolong": 4 + 4 + 1, "residual": A32 + 4 + 4 + 4, "smooth_apply": 50 + 4 + 4 + 4,
            "update_u": 8 + 4 + 8},
    "jacobi": {"outer_residual": A64_SYM + 8 + 8 + 4, "descend": 4 + A32_SYM + 4 + 1,
               "ascend": 4 + 1 + A32_SYM + 4 + 16,
               "smooth_first": 4 + 4 + 4, "residual_restrict": A32_SYM + 4 + 4 + 1,
               "prolong": 4 + 4 + 1, "residual": A32 + 4 + 4 + 4, "smooth_apply": 4 + 4 + 4 + 4,
               "update_u": 8 + 4 + 8},
}
SOLVE_KERNELS = ("outer_residual", "descend", "ascend")  # per-node kernels of the V(1,1) solve

# Measured HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled by
# what the counter reads for a plain copy of known size) of every tile shape of the
# finest-level kernels, with the hash of the kernel sources they were taken with.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_hbm_traffic.txt")
KERNEL_SOURCES = ("paper_2102_12071_amd/csrc/fused.hip", "paper_2102_12071_amd/csrc/cycle.hip",
                  "paper_2102_12071_amd/csrc/common.hpp")


def measured_traffic(kernel: str, tile: str):
    """HBM bytes per launch of the CNN-smoother kernel at this tile shape, from the
    committed counter summary; None when it is missing or the sources changed since."""
    import hashlib
    import re
    try:
        line = next(l for l in open(TRAFFIC_FILE) if l.startswith("data: "))
        data = json.loads(line[len("data: "):])
    except (OSError, StopIteration, ValueError):
        return None
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != data.get("source_sha256"):
        return None
    if kernel == "outer_residual":
        names = ["k_outer_residual<float>"]
    elif tile.startswith("split:"):
        m = re.match(r"split: (\d+)x(\d+) fine nodes, (\d+) threads; (\d+)x(\d+) coarse nodes, (\d+) threads", tile)
        if not m:
            return None
        a = m.groups()
        names = [f"k_presmooth<float, true, {a[0]}, {a[1]}, {a[2]}>", f"k_resrestrict<float, {a[3]}, {a[4]}, {a[5]}>"]
    else:
        m = re.match(r"(\d+)x(\d+) (?:coarse|fine) nodes, (\d+) threads", tile)
        if not m:
            return None
        names = [f"k_{kernel}<float, true, {m.group(1)}, {m.group(2)}, {m.group(3)}>"]
    k = data["kernels"]
    if not all(n in k for n in names):
        return None
    return {"bytes": sum(k[n]["fetch"] + k[n]["write"] for n in names),
            "fetch": sum(k[n]["fetch"] for n in names), "write": sum(k[n]["write"] for n in names),
            "kernels": names, "source": os.path.relpath(TRAFFIC_FILE, ROOT),
            "fetch_factor": data["fetch_factor"], "write_factor": data["write_factor"]}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1023)
    ap.add_argument("--theta", type=float, default=math.pi / 3)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=20000)
    ap.add_argument("--weights", default=WEIGHTS, help="the single network's checkpoint (high-frequency loss)")
    ap.add_argument("--smoother", choices=["auto", "alpha", "hf"], default="auto",
                    help="headline smoother: the per-level networks of the adaptive training (alpha: "
                         "weights/alpha_n*.bin), or the single network (hf); auto: alpha when its checkpoints exist")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--tune-reps", type=int, default=10, help="launches per tile shape in the autotuner")
    ap.add_argument("--sweeps", type=int, nargs="*", default=[2, 3],
                    help="damped-Jacobi V(nu,nu) cycles timed beside the CNN's V(1,1) (none: skip)")
    ap.add_argument("--geometries", type=int, default=1,
                    help="1: also solve the L-shaped and cylinder domains (theta = pi/4, eps = 0.01), CNN and "
                         "Jacobi, beside the headline; 0: skip")
    ap.add_argument("--train-steps", type=int, default=10,
                    help="timed BF16 training steps of the 256-problem batch reported beside the headline (0: skip)")
    ap.add_argument("--redblack", type=int, default=1,
                    help="1: also solve the headline problem with red-black coarsening (committed two-layer "
                         "alpha-CNN smoothers, damped Jacobi V(1,1) and V(2,2)); 0: skip")
    ap.add_argument("--restart", type=int, default=30,
                    help="restart length of the FGMRES comparison reported beside the headline (0: skip it)")
    ap.add_argument("--only", choices=["both", "cnn", "jacobi"], default="both",
                    help="profiling aid: run one smoother only (the JSON line then lacks the comparison)")
    ap.add_argument("--workload", choices=["c2", "c4", "c5"], default="c2",
                    help="c2: the headline problem (default); c4: variable-coefficient 4095^2 with FP64 "
                         "refinement to 1e-10; c5: 512 uneven problems batched in one context")
    ap.add_argument("--batch", type=int, default=512, help="c5: number of problems")
    ap.add_argument("--infer-only", type=int, default=0, metavar="REPS",
                    help="profiling aid: only run mg_smoother_infer on the headline problem REPS times and exit")
    ap.add_argument("--train-only", action="store_true",
                    help="profiling aid: only run the timed training steps and print their JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="profiling aid: only run a plain device copy of MIB MiB five times (the known-size "
                         "kernel that scales the HBM byte counters) and exit")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no multi-GPU path "
              f"(independent problems would shard by size-balanced bin packing, one large grid by 2-D "
              f"blocks with halo exchanges)", file=sys.stderr)
        sys.exit(2)
    if os.environ.get("WORLD_SIZE", "1") not in ("1", ""):
        print("bench.py runs on one GPU only (WORLD_SIZE > 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import mg_inputs
    from paper_2102_12071_amd import mgcnn

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    # Python's cyclic collector stays off: once the earlier blocks have left many objects behind, a
    # collection triggered inside a timed loop paused the interpreter for ~45 ms (seen in the drawn
    # training step: one step of ten took 45 ms, the rest 0.85).  Each block collects before it times.
    gc.disable()
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "launches": 5}), flush=True)
        return
    if args.infer_only:
        net = mgcnn.Net()
        net.load(args.weights)
        ctx = mgcnn.Context([mgcnn.stencil_q1_rotated(args.n, args.theta, args.eps)],
                            mgcnn.Options(smoother=mgcnn.SMOOTHER_CNN))
        for _ in range(args.infer_only):
            ctx.infer(net)
        torch.cuda.synchronize()
        print(json.dumps({"inference_calls": args.infer_only, "n": args.n}), flush=True)
        return
    if args.train_only:
        print(json.dumps(training_block(args)), flush=True)
        return
    if args.workload == "c4":
        return workload_c4(args)
    if args.workload == "c5":
        return workload_c5(args)
    n, theta, eps, tol = args.n, args.theta, args.eps, args.tol
    f = torch.tensor(mg_inputs.rhs_uniform(n, 0), dtype=torch.float64, device="cuda")

    net = mgcnn.Net()
    trained = os.path.exists(args.weights)
    if trained:
        net.load(args.weights)
    else:
        net.set(mg_inputs.cnn_init(0).astype(np.float32))
    alpha_nets = load_alpha_nets(args)
    use_alpha = args.smoother == "alpha" or (args.smoother == "auto" and alpha_nets is not None)
    if use_alpha and alpha_nets is None:
        raise SystemExit("--smoother alpha needs the per-level checkpoints weights/alpha_n*.bin")
    # 7 x 7 coarsest grid for both smoothers (the per-level networks were trained over 3 x 3; with the
    # exact solve at 7 x 7 they take the same 444 cycles at C2 and each cycle costs 3 % less)
    coarsest = 7

    def infer(ctx):
        if use_alpha:
            ctx.infer_levels(alpha_nets)
        else:
            ctx.infer(net)

    A = mgcnn.stencil_q1_rotated(n, theta, eps)
    ctx_cnn = mgcnn.Context([A], mgcnn.Options(smoother=mgcnn.SMOOTHER_CNN, precision=mgcnn.PREC_MIXED,
                                               coarsest_n=coarsest))
    ctx_jac = mgcnn.Context([A], mgcnn.Options(smoother=mgcnn.SMOOTHER_JACOBI, precision=mgcnn.PREC_MIXED,
                                               coarsest_n=coarsest))
    for ctx in (ctx_cnn, ctx_jac):  # set-up, outside the timed steps
        ctx.autotune(args.tune_reps)

    def step(ctx, cnn: bool):
        """One pass of the hot path; returns (iters, relres, phase times in ms)."""
        t0 = time.perf_counter()
        As = mgcnn.stencil_q1_rotated(n, theta, eps)          # a1
        ctx.restencil([As])                                   # a2, a3 (synchronises)
        t1 = time.perf_counter()
        if cnn:
            infer(ctx)                                        # a4
            torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = ctx.solve([f], tol, args.maxit)                 # a5 - a10 (synchronises)
        t3 = time.perf_counter()
        return res, (t1 - t0) * 1e3, (t2 - t1) * 1e3, (t3 - t2) * 1e3

    def run(ctx, cnn):
        name = "cnn" if cnn else "jacobi"
        for w in range(args.warmup):
            r = step(ctx, cnn)
            log(f"{name} warmup {w}: {int(r[0].iters[0])} iterations, relres {r[0].relres[0]:.2e}, "
                f"solve {r[3]:.1f} ms")
        gc.collect()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = []
        for k in range(args.steps):
            out.append(step(ctx, cnn))
            log(f"{name} step {k}: {int(out[-1][0].iters[0])} iterations, solve {out[-1][3]:.1f} ms")
        torch.cuda.synchronize()
        total = (time.perf_counter() - t0) * 1e3
        return out, total / args.steps

    if args.only == "jacobi":
        jac_runs, jac_ms = run(ctx_jac, False)
        print(json.dumps({"jacobi_iters": int(jac_runs[-1][0].iters[0]), "ms_per_step": jac_ms}), flush=True)
        return
    cnn_runs, cnn_ms = run(ctx_cnn, True)
    if args.only == "cnn":
        print(json.dumps({"cnn_iters": int(cnn_runs[-1][0].iters[0]), "ms_per_step": cnn_ms}), flush=True)
        return
    jac_runs, jac_ms = run(ctx_jac, False)
    res_c, res_j = cnn_runs[-1][0], jac_runs[-1][0]
    N = n * n

    def summary(runs, ms_step):
        res = runs[-1][0]
        return {"iters": int(res.iters[0]), "relres": float(res.relres[0]), "status": int(res.status[0]),
                "ms_per_step": ms_step,
                "setup_ms": float(np.mean([r[1] for r in runs])), "infer_ms": float(np.mean([r[2] for r in runs])),
                "solve_ms": float(np.mean([r[3] for r in runs])),
                "solve_device_ms": float(res.ms),
                "ms_per_iteration": float(res.ms) / max(int(res.iters[0]), 1),
                "unknowns_per_s": N / (ms_step * 1e-3)}

    cnn_s, jac_s = summary(cnn_runs, cnn_ms), summary(jac_runs, jac_ms)

    # roofline of the dominant finest-level kernel, timed live with HIP events on the library stream
    kt = ctx_cnn.time_kernels(args.kernel_reps)
    dom = max(SOLVE_KERNELS, key=kt.get)
    nbytes = BYTES_PER_NODE["cnn"][dom] * N
    achieved = nbytes / (kt[dom] * 1e-3) / 1e9
    tiles = {k: ctx_cnn.tile(k, n)["shape"] for k in mgcnn.TILE_KERNELS}
    traffic = measured_traffic(dom, tiles.get(dom, ""))
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic["bytes"] if traffic else None,
                "traffic_detail": traffic,
                "bytes_per_launch": nbytes, "avg_launch_ms": kt[dom],
                "kernels_ms": kt,
                "tiles": tiles,
                "tile_ms": {k: ctx_cnn.tile(k, n)["ms"] for k in mgcnn.TILE_KERNELS},
                "kernels_gbs": {k: BYTES_PER_NODE["cnn"][k] * N / (v * 1e-3) / 1e9 for k, v in kt.items()
                                if k in BYTES_PER_NODE["cnn"]}}
    # the kernel timing leaves the context's vectors undefined; the next solve resets them

    out = {
        "metric": METRIC,
        "value": cnn_s["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": cnn_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"rotated anisotropic Q1, n={n}, theta={theta:.6f}, eps={eps:g}, "
                               f"V(1,1) to {tol:g}, CNN smoother vs damped Jacobi",
                   "n": n, "unknowns": N, "tol": tol, "precision": "bf16 CNN/smoother, fp32 cycle, fp64 refinement",
                   "coarsest_n": coarsest,
                   "weights": ("per-level networks of the adaptive training (Algorithm 2), level sizes "
                               f"{sorted(alpha_nets)}; finer levels take the n = {max(alpha_nets)} network"
                               if use_alpha else "one network, trained on the high-frequency loss" if trained
                               else "untrained (zero last layer = damped Jacobi)")},
        "cnn": cnn_s,
        "jacobi": jac_s,
        "speedup_vs_jacobi": {"iterations": jac_s["iters"] / max(cnn_s["iters"], 1),
                              "time_per_step": jac_ms / cnn_ms},
        "roofline": roofline,
    }

    # the fused MFMA inference kernel's rate: one call of the single network over every level
    # (the per-level networks make one call per level size; their time is in cnn.infer_ms), on a
    # context of its own so that the headline context keeps its smoothers for the blocks below
    ctx_inf = mgcnn.Context([A], mgcnn.Options(smoother=mgcnn.SMOOTHER_CNN, coarsest_n=coarsest))
    out["inference"] = inference_block(ctx_inf, lambda c: c.infer(net), n, coarsest)
    ctx_inf.close()
    if args.restart > 0:
        out["fgmres"] = fgmres_block(args, ctx_cnn, ctx_jac, f, n)
    if args.sweeps:
        out["jacobi_sweeps"] = sweeps_block(args, A, f, n, cnn_s, coarsest)
    if args.geometries:
        out["geometries"] = geometry_block(args, net, alpha_nets if use_alpha else None, n)
    stack = stack_block(args, A, f, n, theta, eps, coarsest)
    if stack is not None:
        out["alpha_stack"] = stack
    if args.redblack:
        rbb = redblack_block(args, n, theta, eps)
        if rbb is not None:
            out["redblack"] = rbb
    if args.train_steps > 0:
        out["training"] = training_block(args)
    out["roofline"]["copy_gbs"] = copy_bandwidth()
    if use_alpha:
        out["hf_cnn"] = hf_block(args, net, f, n, theta, eps)
    if not args.no_cpu_baseline:
        if use_alpha:
            params = {m: v.get().astype(np.float64) for m, v in alpha_nets.items()}
        else:
            params = {0: net.get().astype(np.float64)}
        out["cpu_baseline"] = cpu_baseline(n, theta, eps, params, coarsest, tol, args.maxit, cnn_s["iters"])
    print(json.dumps(out), flush=True)


def inference_block(ctx, infer, n, coarsest, reps=10):
    """Smoother inference (the network on every level but the coarsest, BF16
    MFMA) timed on its own: useful FLOP per second against the dense BF16 peak."""
    gc.collect()
    import torch
    nodes, m = 0, n
    while m > coarsest:
        nodes += m * m
        m = (m - 1) // 2
    infer(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        infer(ctx)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    flop = CNN_FLOP_PER_NODE * nodes
    tflops = flop / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "ms_per_call": ms, "nodes": nodes, "flop": flop, "achieved": tflops,
            "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / BF16_MFMA_PEAK_TFLOPS,
            "note": "useful FLOP (halo recomputation not counted); wall time of the call, all levels"}


def sweeps_block(args, A, f, n, cnn_s, coarsest):
    """Damped Jacobi with more sweeps per cycle, V(nu, nu), against the CNN's
    V(1,1): a smoother that costs more per application should be compared at
    equal cost (the paper matches its convolution layers with as many Jacobi
    steps); here the comparison is simply time to the same tolerance."""
    gc.collect()
    import torch

    from paper_2102_12071_amd import mgcnn
    out = {"cnn_v11_solve_ms": cnn_s["solve_ms"], "cnn_v11_iters": cnn_s["iters"]}
    for nu in args.sweeps:
        ctx = mgcnn.Context([A], mgcnn.Options(smoother=mgcnn.SMOOTHER_JACOBI, nu_pre=nu, nu_post=nu,
                                               coarsest_n=coarsest))
        ctx.solve([f], args.tol, args.maxit)  # warm-up
        times = []
        for _ in range(max(args.steps, 1)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.solve([f], args.tol, args.maxit)
            times.append((time.perf_counter() - t0) * 1e3)
        ms = sum(times) / len(times)
        out[f"v{nu}{nu}"] = {"iters": int(res.iters[0]), "status": int(res.status[0]), "solve_ms": ms,
                             "ms_per_iteration": float(res.ms) / max(int(res.iters[0]), 1)}
        log(f"jacobi V({nu},{nu}): {int(res.iters[0])} iterations, {ms:.1f} ms")
        ctx.close()
    return out


def stack_block(args, A, f, n, theta, eps, coarsest):
    """The paper's constant-coefficient alpha-CNN (H = f5(..f1) + f6 per level,
    trained per problem by Algorithm 2; weights/stack_*.json) on this problem,
    for every committed training run that matches it (Algorithm 2's cycle, or
    the symmetric one with H^T after the coarse correction): iterations and
    time to the tolerance, and the rates of the fused stack level kernels on the
    finest level (FP32 algorithmic traffic per fine node: descend reads r and the
    five stencil planes of a symmetric stencil and writes e and a quarter node of
    r_c, 29 B; the finest ascend reads a quarter node of e_c, e, r, the stencil
    and reads and writes u in FP64, 45 B)."""
    gc.collect()
    import glob

    import torch

    from paper_2102_12071_amd import mgcnn
    from paper_2102_12071_amd.stack_train import load_stack_run
    runs = []
    for p in sorted(glob.glob(os.path.join(os.path.dirname(WEIGHTS), "stack_*.json"))):
        with open(p) as fh:
            prob = json.load(fh).get("problem", {})
        if abs(prob.get("theta", -1) - theta) < 1e-9 and abs(prob.get("eps", -1) - eps) < 1e-12 * max(eps, 1):
            runs.append(p)
    if not runs:
        return None
    out = []
    for path in runs:
        stacks, symmetric = load_stack_run(path)
        ctx = mgcnn.Context([A], mgcnn.Options(smoother=mgcnn.SMOOTHER_STACK, coarsest_n=coarsest))
        ctx.set_stacks(stacks, symmetric=symmetric)
        ctx.solve([f], args.tol, args.maxit)  # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.solve([f], args.tol, args.maxit)
        ms = (time.perf_counter() - t0) * 1e3
        k = ctx.time_kernels(args.kernel_reps)
        fg = None
        if args.restart > 0 and int(res.status[0]) == 0:  # the cycle as a preconditioner of FGMRES
            ctx.solve_fgmres([f], args.tol, args.maxit, restart=args.restart)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.solve_fgmres([f], args.tol, args.maxit, restart=args.restart)
            fg = {"iters": int(r.iters[0]), "status": int(r.status[0]), "relres": float(r.relres[0]),
                  "solve_ms": (time.perf_counter() - t0) * 1e3, "restart": args.restart}
        ctx.close()
        nn = float(n) * n
        kern = {name: {"ms": k[name], "algorithmic_bytes": per * nn,
                       "achieved_gbs": per * nn / (k[name] * 1e-3) / 1e9}
                for name, per in (("descend", 4.0 + A32_SYM + 4 + 1), ("ascend", 1.0 + 4 + 4 + A32_SYM + 16))}
        out.append({"weights": os.path.relpath(path, os.path.dirname(os.path.abspath(__file__))),
                    "symmetric": symmetric, "trained_sizes": sorted(stacks), "iters": int(res.iters[0]),
                    "status": int(res.status[0]), "relres": float(res.relres[0]), "solve_ms": ms,
                    "ms_per_iteration": float(res.ms) / max(int(res.iters[0]), 1), "fgmres": fg,
                    "kernels": kern})
        log(f"alpha-CNN stack ({os.path.basename(path)}): {out[-1]['iters']} iterations, "
            f"status {out[-1]['status']}, {ms:.1f} ms, {out[-1]['ms_per_iteration'] * 1e3:.1f} us per cycle; "
            f"fused stack descend {k['descend'] * 1e3:.1f} us, ascend {k['ascend'] * 1e3:.1f} us"
            + (f"; FGMRES {fg['iters']} iterations, {fg['solve_ms']:.1f} ms" if fg else ""))
    return out


def redblack_block(args, n, theta, eps):
    """Red-black coarsening (section 6.1) on the headline problem, FP64: the committed two-layer
    alpha-CNN smoothers (trained by Algorithm 2 at n = 63 for this theta and eps; deeper levels take
    the deepest trained level of their kind, rescaled to their centre entry) in V(1,1), against
    damped Jacobi V(1,1) and the cost-matched V(2,2) (two Jacobi sweeps per smoothing step, as the
    smoother has two convolutions), all with the same red-black hierarchy."""
    gc.collect()
    from paper_2102_12071_amd import rb_train
    path = os.path.join(os.path.dirname(args.weights), f"rb_theta{theta:.3f}_eps{eps:g}.json")
    if not os.path.exists(path):
        log(f"red-black: no trained smoothers at {path}")
        return None
    weights, centres, kinds, _ = rb_train.load_run(path)
    ev = rb_train.evaluate(weights, centres, kinds, n, theta, eps, tol=args.tol)
    ev["weights"] = os.path.basename(path)
    ev["precision"] = "fp64 (generic-footprint kernels, step by step)"
    log(f"red-black: alpha-CNN {ev['alpha_cnn']['iters']} cycles {ev['alpha_cnn']['solve_ms']:.0f} ms; Jacobi "
        f"V(1,1) {ev['jacobi']['iters']} / {ev['jacobi']['solve_ms']:.0f} ms; V(2,2) {ev['jacobi_v22']['iters']} / "
        f"{ev['jacobi_v22']['solve_ms']:.0f} ms")
    return ev


def copy_bandwidth(mib=1024, reps=10):
    """A plain device copy of 1 GiB timed with events: the bandwidth this box
    reaches on the simplest stream (context for the datasheet peak)."""
    import torch
    src = torch.ones((mib << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def training_block(args):
    """Training steps of the stencil-to-smoother network on the high-frequency
    loss, BF16 on the matrix cores with FP32 master weights and Adam: 256
    problems with n in {31, 63} (the size of each problem drawn once, so that
    every step has the same structure), and per step new draws of theta ~
    U[0, pi), log10 eps ~ U[-3, 0] and 16 high-frequency unit vectors per
    problem from pools of 512 per size.  The timed step is the whole of it
    (host draws, the library's stencils and vector gather, forward, loss,
    backward, Adam), replayed from one captured HIP graph
    (mg_train_step_draw); beside it the eager step on one fixed batch of
    caller-made stencils and vectors (mg_train_step).  Useful FLOP: forward and
    the two backward convolutions (data and weight gradients), 3 x 56,448 per
    point."""
    gc.collect()
    import numpy as np
    import torch

    import mg_inputs
    from paper_2102_12071_amd import mgcnn
    B, J, POOL = 256, 16, 512
    ns, theta, eps = mg_inputs.training_draws(B, 12345, (31, 63))
    ns = [int(m) for m in ns]
    pools = {m: torch.tensor(mg_inputs.hf_pool(m, POOL, 1000 + m), dtype=torch.float32, device="cuda")
             for m in (31, 63)}
    rng = np.random.default_rng(7)
    opts = mgcnn.TrainOptions(precision=1, lr=1e-3)

    def draw():
        th = rng.uniform(0.0, np.pi, B)
        ep = 10.0 ** rng.uniform(-3.0, 0.0, B)
        return th, ep, rng.integers(0, POOL, (B, J))

    net = mgcnn.Net()
    net.set(mg_inputs.cnn_init(0).astype(np.float32))
    for _ in range(2):
        th, ep, ix = draw()
        net.train_step_draw(ns, th, ep, pools, ix, opts, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.train_steps):
        th, ep, ix = draw()
        net.train_step_draw(ns, th, ep, pools, ix, opts, want_loss=False)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.train_steps
    th, ep, ix = draw()
    loss, _ = net.train_step_draw(ns, th, ep, pools, ix, mgcnn.TrainOptions(precision=1, apply_update=0))
    # the eager step on one fixed batch, for comparison
    stencils = [mgcnn.stencil_q1_rotated(m, float(t), float(e)) for m, t, e in zip(ns, theta, eps)]
    vectors = [pools[m][torch.tensor(rng.integers(0, POOL, J), device="cuda")].contiguous() for m in ns]
    eager = mgcnn.Net()
    eager.set(mg_inputs.cnn_init(0).astype(np.float32))
    for _ in range(2):
        eager.train_step(stencils, vectors, opts, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.train_steps):
        eager.train_step(stencils, vectors, opts, want_loss=False)
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / args.train_steps
    points = int(sum(m ** 2 for m in ns))
    tflops = 3 * CNN_FLOP_PER_NODE * points / (ms * 1e-3) / 1e12
    log(f"training: {ms:.2f} ms per drawn, graph-replayed step ({tflops:.0f} TFLOP/s useful); eager fixed batch "
        f"{ms_eager:.2f} ms")
    return {"problems": B, "vectors_per_problem": J, "points": points, "ms_per_step": ms,
            "useful_tflops": tflops, "mfma_peak_tflops": BF16_MFMA_PEAK_TFLOPS, "mfma_frac": tflops / BF16_MFMA_PEAK_TFLOPS,
            "loss_after": loss, "step": "host draws + stencils + vector gather + forward + loss + backward + Adam, "
                                          "one captured HIP graph per step",
            "eager_fixed_batch_ms_per_step": ms_eager, "precision": "bf16 MFMA, fp32 master weights, Adam"}


def load_alpha_nets(args):
    """The per-level networks of the adaptive training (Algorithm 2), keyed by
    level size, from weights/alpha_n<size>.bin beside the single network's
    checkpoint; None when there are none."""
    import glob

    from paper_2102_12071_amd import mgcnn
    files = sorted(glob.glob(os.path.join(os.path.dirname(args.weights), "alpha_n*.bin")))
    if not files:
        return None
    nets = {}
    for path in files:
        net = mgcnn.Net()
        net.load(path)
        nets[int(os.path.basename(path)[len("alpha_n"):-len(".bin")])] = net
    return nets


def hf_block(args, net, f, n, theta, eps):
    """The single network trained on the high-frequency loss, on the headline
    problem and tolerance (its own 7 x 7 coarsest grid), beside the per-level
    networks of the headline."""
    gc.collect()
    import torch

    from paper_2102_12071_amd import mgcnn
    A = mgcnn.stencil_q1_rotated(n, theta, eps)
    ctx = mgcnn.Context([A], mgcnn.Options(smoother=mgcnn.SMOOTHER_CNN))
    ctx.autotune(args.tune_reps)
    ctx.infer(net)
    ctx.solve([f], args.tol, args.maxit)  # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.solve([f], args.tol, args.maxit)
    ms = (time.perf_counter() - t0) * 1e3
    ctx.close()
    log(f"single HF network: {int(res.iters[0])} iterations, {ms:.1f} ms")
    return {"coarsest_n": 7, "iters": int(res.iters[0]), "status": int(res.status[0]),
            "relres": float(res.relres[0]), "solve_ms": ms}


def geometry_block(args, net, alpha_nets, n):
    """The learned smoothers, trained on the square only, on the paper's other
    domains (section 6): the square without its upper-right quadrant
    (L-shape) and without a disk of radius 1/5 about the centre (cylinder),
    zero Dirichlet values on the removed nodes, theta = pi/4, eps = 0.01;
    iterations and solve time to the headline tolerance of the single
    network, of the per-level networks when given (with the fallback to
    damped Jacobi), and of damped Jacobi; 7 x 7 coarsest grid."""
    gc.collect()
    import torch

    import mg_inputs
    from paper_2102_12071_amd import mgcnn
    out = {}
    runs = [("cnn", mgcnn.SMOOTHER_CNN, 7, lambda c: c.infer(net), 0),
            ("jacobi", mgcnn.SMOOTHER_JACOBI, 7, None, 0)]
    if alpha_nets:
        # the per-level networks with the per-problem fallback to damped Jacobi on stall or divergence
        runs.append(("alpha_cnn", mgcnn.SMOOTHER_CNN, 7, lambda c: c.infer_levels(alpha_nets), 1))
    for kind in ("lshape", "cylinder"):
        m = mg_inputs.domain_mask(n, kind)
        A = mgcnn.stencil_mask(mgcnn.stencil_q1_rotated(n, math.pi / 4, 0.01), torch.tensor(m, device="cuda"))
        f = torch.tensor(mg_inputs.rhs_uniform(n, 0) * m, dtype=torch.float64, device="cuda")
        row = {"inside_nodes": int(m.sum())}
        for name, sm, coarsest, infer, fallback in runs:
            ctx = mgcnn.Context([A], mgcnn.Options(smoother=sm, coarsest_n=coarsest, fallback=fallback))
            if infer:
                infer(ctx)
            ctx.solve([f], args.tol, args.maxit)  # warm-up (graph capture)
            if infer:
                infer(ctx)  # a fallback in the warm-up overwrote the learned smoother
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.solve([f], args.tol, args.maxit)
            row[name] = {"iters": int(res.iters[0]), "status": int(res.status[0]),
                         "solve_ms": (time.perf_counter() - t0) * 1e3}
            if fallback:
                row[name]["fell_back_to_jacobi"] = bool(ctx.fallbacks()[0])
            ctx.close()
        row["iteration_ratio"] = row["jacobi"]["iters"] / max(row["cnn"]["iters"], 1)
        row["time_ratio"] = row["jacobi"]["solve_ms"] / row["cnn"]["solve_ms"]
        log(f"{kind}: CNN {row['cnn']['iters']} vs Jacobi {row['jacobi']['iters']} iterations"
            + (f"; per-level networks {row['alpha_cnn']['iters']} (status {row['alpha_cnn']['status']}, "
               f"fallback {row['alpha_cnn']['fell_back_to_jacobi']})" if alpha_nets else ""))
        out[kind] = row
    return out


def fgmres_block(args, ctx_cnn, ctx_jac, f, n):
    """The same problem solved by flexible GMRES(restart) preconditioned by one
    V(1,1) cycle per iteration (the paper's incorporation with FGMRES), to the
    same tolerance: beside the headline, not part of it."""
    gc.collect()
    import torch
    out = {"restart": args.restart, "tol": args.tol}
    for name, ctx in (("cnn", ctx_cnn), ("jacobi", ctx_jac)):
        ctx.solve_fgmres([f], args.tol, 10, restart=args.restart)  # warm-up (workspace, code paths)
        times = []
        for _ in range(max(args.steps, 1)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.solve_fgmres([f], args.tol, args.maxit, restart=args.restart)
            times.append((time.perf_counter() - t0) * 1e3)
        ms = sum(times) / len(times)
        out[name] = {"iters": int(res.iters[0]), "relres": float(res.relres[0]), "status": int(res.status[0]),
                     "solve_ms": ms, "solve_device_ms": float(res.ms), "unknowns_per_s_solve": n * n / (ms * 1e-3)}
        log(f"fgmres {name}: {int(res.iters[0])} iterations, relres {res.relres[0]:.2e}, {ms:.1f} ms")
    return out


def load_net(args):
    import numpy as np

    import mg_inputs
    from paper_2102_12071_amd import mgcnn
    net = mgcnn.Net()
    if os.path.exists(args.weights):
        net.load(args.weights)
        return net, True
    net.set(mg_inputs.cnn_init(0).astype(np.float32))
    return net, False


def workload_c4(args):
    """Variable-coefficient diffusion -div(a grad u) = f on a 4095^2 grid, five-
    point face-average stencil of a = exp(g), g a Gaussian random field
    (squared-exponential covariance, length 0.1, sigma 1, seed 7); CNN smoother
    on every level, V(1,1), FP64 iterative refinement to 1e-10; damped Jacobi
    beside it."""
    gc.collect()
    import torch

    import mg_inputs
    from paper_2102_12071_amd import mgcnn
    n = args.n if args.n != 1023 else 4095
    tol = 1e-10
    t0 = time.perf_counter()
    a = torch.tensor(mg_inputs.lognormal_coefficient(n, 0.1, 1.0, 7), dtype=torch.float64, device="cuda")
    f = torch.tensor(mg_inputs.rhs_uniform(n, 7), dtype=torch.float64, device="cuda")
    log(f"c4 inputs generated on the host in {time.perf_counter() - t0:.1f} s")
    net, trained = load_net(args)
    A = mgcnn.stencil_cellavg5(a)
    out = {"workload": f"variable-coefficient 5-point, a = exp(GRF(0.1, 1, seed 7)), n={n}, V(1,1) to {tol:g}",
           "n": n, "unknowns": n * n, "weights": "trained" if trained else "untrained"}
    for name, sm in (("cnn", mgcnn.SMOOTHER_CNN), ("jacobi", mgcnn.SMOOTHER_JACOBI)):
        if args.only not in ("both", name):
            continue
        ctx = mgcnn.Context([A], mgcnn.Options(smoother=sm))
        ctx.autotune(args.tune_reps)
        times = []
        for k in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            ctx.restencil([mgcnn.stencil_cellavg5(a)])
            if sm == mgcnn.SMOOTHER_CNN:
                ctx.infer(net)
            res = ctx.solve([f], tol, args.maxit)
            times.append((time.perf_counter() - ts) * 1e3)
            log(f"c4 {name} step {k}: {int(res.iters[0])} iterations, relres {res.relres[0]:.2e}, "
                f"{times[-1]:.1f} ms")
        ms = sum(times[args.warmup:]) / args.steps
        kt = ctx.time_kernels(args.kernel_reps)
        key = "cnn" if sm == mgcnn.SMOOTHER_CNN else "jacobi"
        gbs = {k: BYTES_PER_NODE[key][k] * n * n / (kt[k] * 1e-3) / 1e9 for k in SOLVE_KERNELS}
        out[name] = {"iters": int(res.iters[0]), "relres": float(res.relres[0]), "status": int(res.status[0]),
                     "ms_per_step": ms, "solve_device_ms": res.ms, "unknowns_per_s": n * n / (ms * 1e-3),
                     "kernels_ms": {k: kt[k] for k in SOLVE_KERNELS + ("check", "bottom")},
                     "tiles": {k: ctx.tile(k, n)["shape"] for k in mgcnn.TILE_KERNELS},
                     "tile_ms": {k: ctx.tile(k, n)["ms"] for k in mgcnn.TILE_KERNELS},
                     "kernels_gbs": gbs, "kernels_hbm_frac": {k: v / HBM_PEAK_GBS for k, v in gbs.items()}}
        ctx.close()
    print(json.dumps({"metric": METRIC, "value": out.get("cnn", out.get("jacobi"))["unknowns_per_s"],
                      "unit": "unknowns/s", "config": out}), flush=True)


def workload_c5(args):
    """An uneven batch: problems with n uniform in {63, ..., 1023}, theta ~
    U[0, pi), log10 eps ~ U[-4, 0], RHS U(-1, 1), all in one context (one
    launch per size class and kernel), solved to 1e-8 with the CNN smoother and
    with damped Jacobi."""
    gc.collect()
    import numpy as np
    import torch

    import mg_inputs
    from paper_2102_12071_amd import mgcnn
    ns, theta, eps, seeds = mg_inputs.c5_draws(args.batch, 5)
    tol = 1e-8
    fs = [torch.tensor(mg_inputs.rhs_uniform(int(n), int(s)), dtype=torch.float64, device="cuda")
          for n, s in zip(ns, seeds)]
    stencils = [mgcnn.stencil_q1_rotated(int(n), float(t), float(e)) for n, t, e in zip(ns, theta, eps)]
    net, trained = load_net(args)
    N = int(sum(int(n) * int(n) for n in ns))
    out = {"workload": f"{args.batch} problems, n in {{63..1023}}, theta ~ U[0,pi), log10 eps ~ U[-4,0], "
                       f"V(1,1) to {tol:g}", "problems": int(args.batch), "unknowns": N,
           "weights": "trained" if trained else "untrained"}
    for name, sm in (("cnn", mgcnn.SMOOTHER_CNN), ("jacobi", mgcnn.SMOOTHER_JACOBI)):
        t0 = time.perf_counter()
        ctx = mgcnn.Context(stencils, mgcnn.Options(smoother=sm))
        setup_ms = (time.perf_counter() - t0) * 1e3
        ctx.autotune(args.tune_reps)
        times = []
        for k in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            ctx.restencil(stencils)
            if sm == mgcnn.SMOOTHER_CNN:
                ctx.infer(net)
            res = ctx.solve(fs, tol, args.maxit)
            times.append((time.perf_counter() - ts) * 1e3)
            log(f"c5 {name} step {k}: max {int(res.iters.max())} iterations, "
                f"{int((res.status == 0).sum())} converged, {times[-1]:.1f} ms")
        ms = sum(times[args.warmup:]) / args.steps
        out[name] = {"ms_per_step": ms, "unknowns_per_s": N / (ms * 1e-3), "allocation_setup_ms": setup_ms,
                     "iters_median": float(np.median(res.iters)), "iters_max": int(res.iters.max()),
                     "converged": int((res.status == 0).sum()), "not_converged": int((res.status == 1).sum()),
                     "diverged": int((res.status == -4).sum()),
                     "iters_by_n": {str(m): float(np.median(res.iters[ns == m])) for m in sorted(set(ns.tolist()))}}
        ctx.close()
    print(json.dumps({"metric": METRIC, "value": out["cnn"]["unknowns_per_s"], "unit": "unknowns/s",
                      "config": out}), flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, theta, eps, params, coarsest, tol, maxit, gpu_iters):
    """The FP64 oracle on the host cores, run in full on the headline problem:
    stencil, Galerkin hierarchy, CNN inference on every level with the same
    networks, and the V(1,1) solve to tol (nothing extrapolated); beside it the
    n = 63 problem (theta = pi/6, eps = 0.01, damped-Jacobi V(2,2) to 1e-10) on
    all threads and on one.  params: network parameters keyed by level size (a
    level takes the nearest trained size, as on the GPU; one key: every level)."""
    import mg_inputs
    import oracle

    threads = oracle.num_threads()
    sizes = sorted(params)

    def for_size(m):
        return params[min(sizes, key=lambda q: (abs(math.log2(q + 1) - math.log2(m + 1)), -q))]

    f = mg_inputs.rhs_uniform(n, 0)
    t0 = time.perf_counter()
    A = oracle.stencil_q1_rotated(n, theta, eps)
    h = oracle.Hierarchy(A, coarsest)
    t1 = time.perf_counter()
    for l in range(h.num_levels - 1):
        h.set_smoother(l, oracle.cnn_forward(h.stencil(l), for_size(h.level_n(l))))
    t2 = time.perf_counter()
    _, k, hist, conv = h.solve(f, tol, maxit, 1, 1)
    t3 = time.perf_counter()
    total = t3 - t0

    def c1_rate(nthreads):
        oracle.set_threads(nthreads)
        try:
            p = mg_inputs.config_c1()
            fc = mg_inputs.rhs_uniform(p.n, p.rhs_seed)
            ts = time.perf_counter()
            hc = oracle.Hierarchy(oracle.stencil_q1_rotated(p.n, p.theta, p.eps))
            _, kc, _, okc = hc.solve(fc, 1e-10, 1000, 2, 2)
            dt = time.perf_counter() - ts
        finally:
            oracle.set_threads(threads)
        return {"threads": nthreads, "iters": int(kc), "converged": bool(okc), "s": dt,
                "unknowns_per_s": p.n * p.n / dt}

    c1 = {"all_threads": c1_rate(threads), "one_thread": c1_rate(1)}
    return {"value": n * n / total, "unit": "unknowns/s", "cores": threads, "kind": "oracle",
            "run": f"full: the solve to {tol:g} run to the end, nothing extrapolated",
            "iters": int(k), "gpu_iters": int(gpu_iters), "converged": bool(conv), "relres": float(hist[-1]),
            "setup_s": t1 - t0, "infer_s": t2 - t1, "solve_s": t3 - t2, "total_s": total,
            "ms_per_cycle": (t3 - t2) / max(k, 1) * 1e3,
            "omp_threads": threads, "nproc": os.cpu_count(), "cpu_model": _cpu_model(), "c1": c1,
            "sample": f"FP64 oracle (C, OpenMP over rows, {threads} threads): the headline problem in full - "
                      f"stencil + Galerkin hierarchy ({t1 - t0:.2f} s), CNN inference on all levels "
                      f"({t2 - t1:.2f} s), V(1,1) solve to {tol:g} ({k} cycles, {t3 - t2:.2f} s)"}


if __name__ == "__main__":
    main()
