"""C-ABI checks that need no GPU: the library loads, exports every entry point
the header declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgcnn.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2102_12071_amd import mgcnn
    return mgcnn.load_library()


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "mgcnn.h"\nint main(void){mg_options o; mg_options_default(&o); return o.nu_pre;}\n')
    import subprocess
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-c", "-I", os.path.join(ROOT, "include"), str(src),
                        "-o", str(tmp_path / "t.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_every_declared_symbol_is_exported(lib):
    from paper_2102_12071_amd import mgcnn
    names = _declared()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name
        assert name in mgcnn.SIGNATURES, f"binding lacks {name}"


def test_binding_structs_match_header_sizes():
    from paper_2102_12071_amd import mgcnn
    assert C.sizeof(mgcnn.COptions) == 48
    assert C.sizeof(mgcnn.Problem) == 16
    assert C.sizeof(mgcnn.TrainOpts) == 32
    assert C.sizeof(mgcnn.AlphaBatch) == 48


def test_status_strings_and_defaults(lib):
    from paper_2102_12071_amd import mgcnn
    assert lib.mg_status_str(0) == b"MG_OK"
    assert lib.mg_status_str(-4) == b"MG_ERR_DIVERGED"
    assert b"gfx950" in lib.mg_version()
    o = mgcnn.COptions()
    lib.mg_options_default(C.byref(o))
    assert (o.nu_pre, o.nu_post, o.coarsest_n, o.precision) == (1, 1, 7, 1)
    assert abs(o.omega - 2.0 / 3.0) < 1e-15
    t = mgcnn.TrainOpts()
    lib.mg_train_opts_default(C.byref(t))
    assert abs(t.lr - 1e-3) < 1e-9 and t.apply_update == 1


def test_argument_errors_before_device(lib):
    # validation happens before any device call, so these work without a GPU
    assert lib.mg_stencil_q1_rotated(8, 0.0, 0.1, C.c_void_p(16), None) == -1
    assert b"odd" in lib.mg_last_error()
    assert lib.mg_stencil_q1_rotated(7, 0.0, 0.0, C.c_void_p(16), None) == -1
    assert lib.mg_galerkin(1, C.c_void_p(16), C.c_void_p(16), None) == -1
    assert lib.mg_stencil_cellavg5(7, None, C.c_void_p(16), None) == -1
    from paper_2102_12071_amd import mgcnn
    h = C.c_void_p()
    assert lib.mg_setup(None, 0, None, None, C.byref(h)) == -1
    probs = (mgcnn.Problem * 1)(mgcnn.Problem(10, 16))
    assert lib.mg_setup(probs, 1, None, None, C.byref(h)) == -1
    assert b"2^k - 1" in lib.mg_last_error()
    opt = mgcnn.COptions()
    lib.mg_options_default(C.byref(opt))
    opt.coarsest_n = 5
    probs = (mgcnn.Problem * 1)(mgcnn.Problem(15, 16))
    assert lib.mg_setup(probs, 1, C.byref(opt), None, C.byref(h)) == -1
    assert lib.mg_solve(None, None, None, 1e-8, 10, None, None, None, None) == -1
    assert lib.mg_vcycle(None, None, None) == -1
    assert lib.mg_train_step(None, None, None, None, None) == -1
    assert lib.mg_net_get(None, None, 0) == -1
    assert lib.mg_alpha_step(None, None, None, None, None, None, None, None, None) == -1
    assert lib.mg_smoother_transpose(0, C.c_void_p(16), C.c_void_p(16), C.c_void_p(32), None) == -1
    assert lib.mg_smoother_transpose(7, C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), None) == -1
    assert b"same buffer" in lib.mg_last_error()
    assert lib.mg_smoother_infer_size(None, None, 7) == -1
    # the convolution-stack smoother's entry points
    assert lib.mg_set_stack(None, 0, 0, None, 0, 0) == -1
    assert lib.mg_stack_apply(0, 1, C.c_void_p(16), C.c_void_p(16), C.c_void_p(4096), 0, None) == -1
    assert lib.mg_stack_apply(7, 1, C.c_void_p(16), C.c_void_p(4096), C.c_void_p(4096 + 8 * 48), 0, None) == -1
    assert b"overlap" in lib.mg_last_error()
    assert lib.mg_stack_apply(7, 1, C.c_void_p(16), C.c_void_p(4096), C.c_void_p(8192), 2, None) == -1
    assert lib.mg_stack_alpha_step(None, None, None, None, None, None, 0, 0, None, None, None, None, None) == -1
    assert lib.mg_set_stack_post(None, 0, 0, None, 1, 0) == -1
    lib.mg_options_default(C.byref(opt))
    opt.smoother, opt.fallback = mgcnn.SMOOTHER_STACK, 1
    assert lib.mg_setup(probs, 1, C.byref(opt), None, C.byref(h)) == -1
    assert b"fallback" in lib.mg_last_error()
    opt.smoother, opt.fallback = 3, 0
    assert lib.mg_setup(probs, 1, C.byref(opt), None, C.byref(h)) == -1


def test_alpha_stage_sizes():
    from paper_2102_12071_amd.alpha_train import stage_sizes
    assert stage_sizes(63) == [7, 15, 31, 63]  # four stages of a 5-level hierarchy, coarse to fine
    assert stage_sizes(63, 7) == [15, 31, 63]
    assert stage_sizes(7) == [7]
    assert stage_sizes(3) == []


def test_product_path_has_no_oracle_dependency():
    # the library and its binding must not load or import the oracle
    pkg = os.path.join(ROOT, "paper_2102_12071_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "liboracle" not in text and "oracle.h" not in text, fn
