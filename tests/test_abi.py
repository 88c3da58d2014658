"""C ABI contract, checked without a GPU: the library loads, exports every
entry point include/sr.h declares, the ctypes structures match the C layout,
and argument validation happens before any HIP call."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sr.h")


@pytest.fixture(scope="module")
def sr():
    from paper_2003_12693_amd import sr as srmod
    if not os.path.exists(srmod.LIB_PATH):
        from paper_2003_12693_amd import build
        build.build()
    srmod.load()
    return srmod


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|void|const char\*)\s+(sr_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported(sr):
    names = declared_functions()
    assert len(names) >= 17
    out = subprocess.run(["nm", "-D", "--defined-only", sr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(sr_\w+)$", out, re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = sr.load()
    for n in names:
        assert getattr(lib, n) is not None


def test_struct_layout_matches_c(sr, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "sr.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(sr_params), sizeof(sr_step_info),"
        " sizeof(sr_batch_item), offsetof(sr_params, w0_mode), offsetof(sr_batch_item, params),"
        " offsetof(sr_batch_item, energy), offsetof(sr_params, tol_outer), offsetof(sr_params, w_sweeps),"
        " offsetof(sr_params, bc));"
        " return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()))
    assert vals == [C.sizeof(sr.sr_params), C.sizeof(sr.sr_step_info), C.sizeof(sr.sr_batch_item),
                    sr.sr_params.w0_mode.offset, sr.sr_batch_item.params.offset,
                    sr.sr_batch_item.energy.offset, sr.sr_params.tol_outer.offset, sr.sr_params.w_sweeps.offset,
                    sr.sr_params.bc.offset]


def test_defaults_are_the_two_circles_set(sr):
    p = sr.sr_params_default()
    assert p.struct_size == C.sizeof(sr.sr_params)
    assert (p.alpha, p.gamma, p.beta, p.mu, p.tau, p.S, p.band_l, p.d) == (4.0, 4.0, 0.2, 8.0, 0.1, 3, 1.0, 5.0)
    assert (p.w_solver, p.w_sweeps) == (0, 1)


@pytest.mark.parametrize("M,N,kw,code", [
    (1000, 1024, {}, -2), (4, 16, {}, -2), (8192, 8, {}, -2), (64, 64, dict(R=9), -2),
    (64, 64, dict(tau=0.0), -1), (64, 64, dict(mu=0.0), -1), (64, 64, dict(eps=-1.0), -1),
    (64, 64, dict(S=0), -1), (64, 64, dict(s_exp=3), -1), (64, 64, dict(check_every=0), -1),
    (64, 64, dict(sigma=6.0), -2), (64, 64, dict(w0_mode=2), -1), (64, 64, dict(gamma=float("nan")), -1),
])
def test_validation_codes(sr, M, N, kw, code):
    p = sr.sr_params_default(**kw)
    with pytest.raises(sr.SRError) as e:
        sr.sr_workspace_size(M, N, p)
    assert e.value.code == code
    assert sr.load().sr_last_error().decode()


def test_bad_struct_size_rejected(sr):
    p = sr.sr_params_default()
    p.struct_size = 8
    with pytest.raises(sr.SRError) as e:
        sr.sr_workspace_size(64, 64, p)
    assert e.value.code == sr.SR_EINVAL


def test_create_validates_before_any_hip_call(sr):
    lib = sr.load()
    p = sr.sr_params_default()
    ctx = C.c_void_p()
    n = sr.sr_workspace_size(128, 128, p)
    assert lib.sr_create(C.byref(ctx), 128, 128, C.byref(p), None, n, None) == sr.SR_EINVAL
    assert lib.sr_create(C.byref(ctx), 128, 128, C.byref(p), 4096 + 1, n, None) == sr.SR_EWORKSPACE
    assert lib.sr_create(C.byref(ctx), 128, 128, C.byref(p), 4096, n - 1, None) == sr.SR_EWORKSPACE
    assert lib.sr_create(None, 128, 128, C.byref(p), 4096, n, None) == sr.SR_EINVAL
    assert ctx.value is None
    lib.sr_destroy(None)


def test_null_context_calls(sr):
    lib = sr.load()
    info = sr.sr_step_info()
    assert lib.sr_step(None, 1, C.byref(info)) == sr.SR_EINVAL
    assert lib.sr_set_image(None, None, None, 0) == sr.SR_EINVAL
    E = C.c_double()
    assert lib.sr_energy(None, C.byref(E), None) == sr.SR_EINVAL


def test_workspace_size_scales(sr):
    p = sr.sr_params_default()
    a = sr.sr_workspace_size(1024, 1024, p)
    b = sr.sr_workspace_size(4096, 4096, p)
    assert 13 * 4 * 1024 * 1024 <= a < 20 * 4 * 1024 * 1024
    assert 15.5 < b / a < 16.5


def test_batch_validation_before_hip(sr):
    lib = sr.load()
    items = (sr.sr_batch_item * 2)()
    for it in items:
        it.M, it.N, it.max_iter = 64, 64, 10
        it.params = sr.sr_params_default()
    n = C.c_size_t()
    assert lib.sr_batch_workspace_size(items, 2, C.byref(n)) == sr.SR_OK and n.value > 0
    one = (sr.sr_batch_item * 1)(items[0])
    n1 = C.c_size_t()
    lib.sr_batch_workspace_size(one, 1, C.byref(n1))
    assert n.value < 2 * n1.value          # equal classes share one group layout
    items[1].M = 100
    assert lib.sr_batch_workspace_size(items, 2, C.byref(n)) == sr.SR_EUNSUPPORTED
    items[1].M = 64
    items[1].max_iter = 0
    assert lib.sr_batch_workspace_size(items, 2, C.byref(n)) == sr.SR_EINVAL
    items[1].max_iter = 10
    assert lib.sr_solve_batch(items, 2, None, 0, None) == sr.SR_EINVAL     # NULL buffers


def test_fixed_point_w_solver_parameters(sr):
    """w_solver / w_sweeps are validated before any HIP call, and the
    workspace carries the intermediate w of the sweeps (one 2-plane buffer
    for two sweeps, two from three on)."""
    base = sr.sr_workspace_size(64, 64, sr.sr_params_default())
    for bad in (dict(w_solver=2), dict(w_solver=1, w_sweeps=0), dict(w_solver=1, w_sweeps=17)):
        with pytest.raises(sr.SRError) as e:
            sr.sr_workspace_size(64, 64, sr.sr_params_default(**bad))
        assert e.value.code == sr.SR_EINVAL, bad
    vec = 2 * 64 * 64 * 4
    assert sr.sr_workspace_size(64, 64, sr.sr_params_default(w_solver=1, w_sweeps=1)) == base
    assert sr.sr_workspace_size(64, 64, sr.sr_params_default(w_solver=1, w_sweeps=2)) == base + vec
    assert sr.sr_workspace_size(64, 64, sr.sr_params_default(w_solver=1, w_sweeps=5)) == base + 2 * vec
    assert sr.sr_workspace_size(64, 64, sr.sr_params_default(w_solver=0, w_sweeps=5)) == base


def test_aos_phi_solver_parameters(sr):
    """phi_solver is validated before any HIP call: 0 / 1 only, a fixed S
    (tol_inner = 0), and sizes on which the inverse of (1 - 2 tau mu D)
    truncates within +-64 points (not 8 points at tau mu = 0.8)."""
    with pytest.raises(sr.SRError) as e:
        sr.sr_workspace_size(64, 64, sr.sr_params_default(phi_solver=2))
    assert e.value.code == sr.SR_EINVAL
    with pytest.raises(sr.SRError) as e:
        sr.sr_workspace_size(64, 64, sr.sr_params_default(phi_solver=1, tol_inner=1e-3))
    assert e.value.code == sr.SR_EUNSUPPORTED
    with pytest.raises(sr.SRError) as e:
        sr.sr_workspace_size(8, 64, sr.sr_params_default(phi_solver=1))
    assert e.value.code == sr.SR_EUNSUPPORTED
    assert sr.sr_workspace_size(64, 64, sr.sr_params_default(phi_solver=1)) == \
        sr.sr_workspace_size(64, 64, sr.sr_params_default())
    assert sr.sr_params_default().phi_solver == 0


def test_boundary_parameter(sr):
    """bc is validated before any HIP call: 0 (periodic) / 1 (Neumann) only.
    The Neumann solve is the DCT-II one on the grid itself: every size the
    periodic solve takes (up to 4096 per side, the inner stop rule allowed),
    and the same workspace as the periodic solve."""
    assert sr.sr_params_default().bc == 0
    with pytest.raises(sr.SRError) as e:
        sr.sr_workspace_size(64, 64, sr.sr_params_default(bc=2))
    assert e.value.code == sr.SR_EINVAL
    base = sr.sr_workspace_size(64, 64, sr.sr_params_default())
    assert sr.sr_workspace_size(64, 64, sr.sr_params_default(bc=1, phi_solver=1)) == base
    assert sr.sr_workspace_size(64, 64, sr.sr_params_default(bc=1)) == base
    assert sr.sr_workspace_size(64, 64, sr.sr_params_default(bc=1, tol_inner=1e-3)) == base
    assert sr.sr_workspace_size(4096, 4096, sr.sr_params_default(bc=1)) == sr.sr_workspace_size(
        4096, 4096, sr.sr_params_default())


def test_every_3d_symbol_is_exported_and_validated(sr):
    """include/sr3d.h: every declared entry point is exported, and the size
    and parameter checks run before any HIP call."""
    text = open(os.path.join(ROOT, "include", "sr3d.h")).read()
    names = sorted(set(re.findall(r"^(?:int|void)\s+(sr3_\w+)\s*\(", text, re.M)))
    assert len(names) == 8
    out = subprocess.run(["nm", "-D", "--defined-only", sr.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(sr3_\w+)$", out, re.M))
    assert not [n for n in names if n not in exported]
    p = sr.sr_params_default()
    n = sr.sr3_workspace_size(32, 16, 64, p)
    # 16 real planes (g, two phi, w, b, u, v, r) and the spectrum of k
    # frequencies 0..32 in 48 slots per k-line (whole groups of 16 lines)
    assert n >= 4 * 32 * 16 * 64 * 16 + 8 * 32 * 16 * 48
    for shape, kw in (((4, 16, 16), {}), ((16, 16, 512), {}), ((16, 24, 16), {}), ((16, 16, 16), dict(bc=1)),
                      ((16, 16, 16), dict(phi_solver=1)), ((16, 16, 16), dict(tol_inner=1e-3)),
                      ((16, 16, 16), dict(R=9))):
        with pytest.raises(sr.SRError) as e:
            sr.sr3_workspace_size(*shape, sr.sr_params_default(**kw))
        assert e.value.code in (sr.SR_EUNSUPPORTED, sr.SR_EINVAL)
