"""The committed weights: every stack training run is well formed (54 finite
weights per trained size, the problem it was trained for, the cycle form, the
command that wrote it) and loads through the trainer's loader."""
import glob
import json
import math
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2102_12071_amd", "weights")


def test_stack_runs_are_well_formed():
    from paper_2102_12071_amd.stack_train import load_stack_run
    paths = sorted(glob.glob(os.path.join(WEIGHTS, "stack_*.json")))
    assert len(paths) >= 4
    for p in paths:
        d = json.load(open(p))
        assert set(d["problem"]) == {"theta", "eps"} and 0 <= d["problem"]["theta"] < math.pi
        assert d["command"].startswith("python -m paper_2102_12071_amd.stack_train")
        assert d["command"].endswith(os.path.relpath(p, ROOT))
        assert (" --symmetric" in d["command"]) == bool(d.get("symmetric", False))
        stacks, symmetric = load_stack_run(p)
        assert symmetric == bool(d.get("symmetric", False))
        assert sorted(stacks) == [7, 15, 31, 63, 127, 255, 511, 1023]
        for w in stacks.values():
            assert w.shape == (6, 3, 3) and np.isfinite(w).all()
        evals = [r for r in d["records"] if "eval" in r]
        assert {r["eval"]["n"] for r in evals} == {63, 255, 1023}


def test_redblack_runs_are_well_formed():
    from paper_2102_12071_amd.rb_train import load_run
    paths = sorted(glob.glob(os.path.join(WEIGHTS, "rb_*.json")))
    assert len(paths) >= 2
    for p in paths:
        weights, centres, kinds, d = load_run(p)
        assert d["command"].startswith("python -m paper_2102_12071_amd.rb_train")
        assert d["command"].endswith(os.path.relpath(p, ROOT))
        assert sorted(weights) == list(range(6)) and sorted(centres) == list(range(6))
        assert [kinds[l] for l in range(6)] == ["full", "checker"] * 3
        for w in weights.values():
            assert w.shape == (2, 3, 3) and np.isfinite(w).all()
        assert all(c > 0 for c in centres.values())
        assert {e["n"] for e in d["evaluations"]} == {63, 255, 1023}
