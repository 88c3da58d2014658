"""C ABI of the warm-start network, checked without a GPU: every cnn_*
entry point include/cnn.h declares is exported, the parameter count matches
the reference network, and argument validation happens before any HIP call."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import cnn_reference as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cnn.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2003_12693_amd import cnn, sr
    if not os.path.exists(sr.LIB_PATH):
        from paper_2003_12693_amd import build
        build.build()
    return cnn.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_2003_12693_amd import sr
    names = sorted(set(re.findall(r"^(?:int|void|const char\*)\s+(cnn_\w+)\s*\(", open(HEADER).read(), re.M)))
    assert len(names) == 11
    out = subprocess.run(["nm", "-D", "--defined-only", sr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(cnn_\w+)$", out, re.M))
    assert not [n for n in names if n not in exported]


def test_parameter_count_matches_reference(lib):
    n = C.c_int64()
    assert lib.cnn_num_params(C.byref(n)) == 0
    assert n.value == R.flatten(R.init_params(0)).size


@pytest.mark.parametrize("B,H,W,code", [(0, 64, 64, -2), (1, 48, 64, -2), (1, 64, 4096, -2),
                                        (1, 16, 64, -2), (4096, 2048, 2048, -2)])
def test_size_validation(lib, B, H, W, code):
    n = C.c_size_t()
    assert lib.cnn_workspace_size(B, H, W, C.byref(n)) == code
    assert lib.cnn_last_error()


def test_workspace_size_scales(lib):
    a, b = C.c_size_t(), C.c_size_t()
    assert lib.cnn_workspace_size(1, 512, 512, C.byref(a)) == 0
    assert lib.cnn_workspace_size(4, 512, 512, C.byref(b)) == 0
    per_px = (b.value - a.value) / (3 * 512 * 512)
    assert 500 < per_px < 1000          # activations + gradients, bytes per pixel


def test_create_validates_before_any_hip_call(lib):
    ctx = C.c_void_p()
    n = C.c_size_t()
    lib.cnn_workspace_size(1, 64, 64, C.byref(n))
    assert lib.cnn_create(C.byref(ctx), 1, 64, 64, None, n.value, None) == -1
    assert lib.cnn_create(C.byref(ctx), 1, 64, 64, 4096 + 8, n.value, None) == -3
    assert lib.cnn_create(C.byref(ctx), 1, 64, 64, 4096, n.value - 1, None) == -3
    assert lib.cnn_create(None, 1, 64, 64, 4096, n.value, None) == -1
    assert ctx.value is None
    assert lib.cnn_forward(None, None, None, None, 1, 8.0, None) == -1
    assert lib.cnn_backward(None, None, 8.0, None, None) == -1
    assert lib.cnn_adam_step(None, 1e-3, 0.9, 0.999, 1e-8) == -1
    lib.cnn_destroy(None)


def test_binding_layer_table_matches_reference():
    from paper_2003_12693_amd import cnn
    assert [(a, b, c) for a, b, c, _ in cnn.LAYERS] == R.LAYERS
    assert cnn.he_init(0).size == R.flatten(R.init_params(0)).size
    fwd, train = cnn.flops(1, 512, 512)
    # per pixel: sum over levels of 9*cin*cout*2 / 4^level, plus the head
    per_px = sum(2 * 9 * cin * cout / 4 ** lev for _, cin, cout, lev in cnn.LAYERS) + 2 * 16
    assert fwd == pytest.approx(per_px * 512 * 512)
    assert 2.9 < train / fwd < 3.0
