"""Python binding of libsr (include/sr.h): argument marshalling only.

Every step of the solver runs in the HIP kernels of libsr.so; this module
only converts arguments (torch tensors on the GPU -> device pointers, NumPy
arrays -> host pointers with SR_HOST) and raises on error codes.  There is
no CPU fallback: if libsr.so is missing or no GPU is present, calls fail.

The C entry points are exposed under their own names (``sr_create``,
``sr_step`` ...); ``Solver`` is a small convenience wrapper that owns the
workspace tensor.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SR_LIB") or os.path.join(_HERE, "libsr.so")

SR_OK = 0
SR_NOT_CONVERGED = 1
SR_EINVAL = -1
SR_EUNSUPPORTED = -2
SR_EWORKSPACE = -3
SR_EHIP = -4
SR_ENONFINITE = -5
SR_ESTATE = -6
SR_HOST = 1


class SRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsr error {code}: {msg}")
        self.code = code


class sr_params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("gamma", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
        ("mu", C.c_double), ("tau", C.c_double),
        ("eps", C.c_double), ("band_l", C.c_double), ("d", C.c_double),
        ("R", C.c_int32),
        ("sigma", C.c_double), ("rho", C.c_double),
        ("s_exp", C.c_int32), ("S", C.c_int32),
        ("tol_inner", C.c_double), ("tol_outer", C.c_double),
        ("min_iter", C.c_int32), ("check_every", C.c_int32), ("w0_mode", C.c_int32),
        ("zero_tol", C.c_double),
        ("w_solver", C.c_int32), ("w_sweeps", C.c_int32), ("phi_solver", C.c_int32),
        ("bc", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "struct_size"}


class sr_step_info(C.Structure):
    _fields_ = [
        ("iters_done", C.c_int64), ("k", C.c_int64), ("r_last", C.c_double),
        ("inner_steps", C.c_int64), ("converged", C.c_int32), ("reserved", C.c_int32),
    ]


class sr_batch_item(C.Structure):
    _fields_ = [
        ("M", C.c_int32), ("N", C.c_int32),
        ("f", C.c_void_p), ("phi0", C.c_void_p), ("phi_out", C.c_void_p),
        ("params", sr_params),
        ("max_iter", C.c_int32),
        ("iters", C.c_int32), ("status", C.c_int32), ("reserved", C.c_int32),
        ("r_last", C.c_double), ("energy", C.c_double),
        ("w_out", C.c_void_p), ("b_out", C.c_void_p),
    ]


_lib = None


def load(path=LIB_PATH):
    """Load libsr.so (built by paper_2003_12693_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2003_12693_amd.build`")
    lib = C.CDLL(path)
    P, I, D = C.c_void_p, C.c_int32, C.c_double
    sig = {
        "sr_params_default": (C.c_int, [C.POINTER(sr_params)]),
        "sr_workspace_size": (C.c_int, [I, I, C.POINTER(sr_params), C.POINTER(C.c_size_t)]),
        "sr_create": (C.c_int, [C.POINTER(P), I, I, C.POINTER(sr_params), P, C.c_size_t, P]),
        "sr_set_image": (C.c_int, [P, P, P, C.c_uint32]),
        "sr_step": (C.c_int, [P, I, C.POINTER(sr_step_info)]),
        "sr_get_phi": (C.c_int, [P, P, C.c_uint32]),
        "sr_get_g": (C.c_int, [P, P, C.c_uint32]),
        "sr_energy": (C.c_int, [P, C.POINTER(D), C.POINTER(D)]),
        "sr_get_state": (C.c_int, [P, P, P, P, C.POINTER(C.c_int64), C.c_uint32]),
        "sr_set_state": (C.c_int, [P, P, P, P, C.c_int64, C.c_uint32]),
        "sr_edge_map": (C.c_int, [P, P, P, C.c_uint32]),
        "sr_repulsion": (C.c_int, [P, P, P, P, C.c_uint32]),
        "sr_implicit_solve": (C.c_int, [P, P, P, C.c_uint32]),
        "sr_batch_workspace_size": (C.c_int, [C.POINTER(sr_batch_item), I, C.POINTER(C.c_size_t)]),
        "sr_solve_batch": (C.c_int, [C.POINTER(sr_batch_item), I, P, C.c_size_t, P]),
        "sr_profile_kernels": (C.c_int, [P, I, C.POINTER(D), C.POINTER(C.c_int64)]),
        "sr_autotune": (C.c_int, [P, I, C.POINTER(I), C.POINTER(D)]),
        "sr_prepare": (C.c_int, [P]),
        "sr_implicit_solve_noalloc": (C.c_int, [I, I, D, D, P, P, P]),
        "sr_build_id": (C.c_char_p, []),
        "sr_destroy": (None, [P]),
        "sr_last_error": (C.c_char_p, []),
        "sr3_workspace_size": (C.c_int, [I, I, I, C.POINTER(sr_params), C.POINTER(C.c_size_t)]),
        "sr3_create": (C.c_int, [C.POINTER(P), I, I, I, C.POINTER(sr_params), P, C.c_size_t, P]),
        "sr3_set_image": (C.c_int, [P, P, P]),
        "sr3_set_state": (C.c_int, [P, P, P, P, C.c_int64]),
        "sr3_step": (C.c_int, [P, I, C.POINTER(C.c_int64)]),
        "sr3_get_state": (C.c_int, [P, P, P, P, P]),
        "sr3_profile": (C.c_int, [P, I, C.POINTER(D), C.POINTER(C.c_int64)]),
        "sr3_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc, allow_warning=False):
    if rc == SR_OK or (allow_warning and rc > 0):
        return rc
    raise SRError(rc, load().sr_last_error().decode())


# ---------------------------------------------------------------------------
# same-name wrappers of the C entry points
# ---------------------------------------------------------------------------
def sr_params_default(**overrides):
    p = sr_params()
    _check(load().sr_params_default(C.byref(p)))
    for k, v in overrides.items():
        if not hasattr(p, k) or k == "struct_size":
            raise KeyError(k)
        setattr(p, k, v)
    return p


def sr_workspace_size(M, N, params):
    n = C.c_size_t()
    _check(load().sr_workspace_size(M, N, C.byref(params), C.byref(n)))
    return n.value


def _ptr(x, flags_host):
    """(pointer, is_host) of a torch tensor or NumPy array (float32, C-contiguous)."""
    try:
        import torch
        if isinstance(x, torch.Tensor):
            if x.dtype != torch.float32 or not x.is_contiguous():
                raise ValueError("tensors must be contiguous float32")
            if not x.is_cuda:
                raise ValueError("torch tensors must be on the GPU (pass NumPy arrays for host data)")
            return x.data_ptr(), False
    except ImportError:
        pass
    if isinstance(x, np.ndarray):
        if x.dtype != np.float32 or not x.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous float32")
        return x.ctypes.data, True
    raise TypeError(f"unsupported buffer type {type(x)}")


def _flags(*ptrs):
    hosts = {h for _, h in ptrs}
    if len(hosts) != 1:
        raise ValueError("pass either all GPU tensors or all host arrays")
    return SR_HOST if hosts.pop() else 0


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def sr_create(M, N, params, workspace, stream=None):
    import torch
    ctx = C.c_void_p()
    assert workspace.is_cuda and workspace.dtype == torch.uint8
    _check(load().sr_create(C.byref(ctx), M, N, C.byref(params), workspace.data_ptr(),
                            workspace.numel(), _stream_ptr(stream)))
    return ctx


def sr_set_image(ctx, f, phi0):
    a, b = _ptr(f, True), _ptr(phi0, True)
    _check(load().sr_set_image(ctx, a[0], b[0], _flags(a, b)))


def sr_step(ctx, n_iter):
    info = sr_step_info()
    rc = _check(load().sr_step(ctx, n_iter, C.byref(info)), allow_warning=True)
    return rc, info


def sr_get_phi(ctx, out):
    a = _ptr(out, True)
    _check(load().sr_get_phi(ctx, a[0], _flags(a)))
    return out


def sr_get_g(ctx, out):
    a = _ptr(out, True)
    _check(load().sr_get_g(ctx, a[0], _flags(a)))
    return out


def sr_energy(ctx):
    E = C.c_double()
    T = (C.c_double * 3)()
    _check(load().sr_energy(ctx, C.byref(E), T))
    return E.value, (T[0], T[1], T[2])


def sr_get_state(ctx, phi, w, b):
    a, bw, bb = _ptr(phi, True), _ptr(w, True), _ptr(b, True)
    k = C.c_int64()
    _check(load().sr_get_state(ctx, a[0], bw[0], bb[0], C.byref(k), _flags(a, bw, bb)))
    return k.value


def sr_set_state(ctx, phi, w, b, k):
    a, bw, bb = _ptr(phi, True), _ptr(w, True), _ptr(b, True)
    _check(load().sr_set_state(ctx, a[0], bw[0], bb[0], int(k), _flags(a, bw, bb)))


def sr_edge_map(ctx, f, g_out):
    a, b = _ptr(f, True), _ptr(g_out, True)
    _check(load().sr_edge_map(ctx, a[0], b[0], _flags(a, b)))
    return g_out


def sr_repulsion(ctx, w, phi, v_out):
    a, b, c = _ptr(w, True), _ptr(phi, True), _ptr(v_out, True)
    _check(load().sr_repulsion(ctx, a[0], b[0], c[0], _flags(a, b, c)))
    return v_out


def sr_implicit_solve(ctx, rhs, u_out):
    a, b = _ptr(rhs, True), _ptr(u_out, True)
    _check(load().sr_implicit_solve(ctx, a[0], b[0], _flags(a, b)))
    return u_out


KERNEL_KINDS = ("rhs_repulsion", "row_fft_fwd", "col_fft_solve", "row_fft_inv", "w_step")


def sr_profile_kernels(ctx, n_iter):
    """Average per-launch duration (ms) and launch count of each kernel kind."""
    ms = (C.c_double * 5)()
    cnt = (C.c_int64 * 5)()
    _check(load().sr_profile_kernels(ctx, n_iter, ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}


def sr_autotune(ctx, reps=5):
    """Stencil tile height chosen for the context: (rows, {rows: mean us})."""
    th = C.c_int32()
    us = (C.c_double * 3)()
    _check(load().sr_autotune(ctx, reps, C.byref(th), us))
    return th.value, {8: us[0], 16: us[1], 32: us[2]}


def sr_implicit_solve_noalloc(rhs, u_out, tau, mu, stream=None):
    """(1 - tau mu Lap) u = rhs through the entry point that allocates
    nothing (GPU tensors only)."""
    import torch
    for x in (rhs, u_out):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
            raise ValueError("sr_implicit_solve_noalloc takes contiguous float32 GPU tensors")
    M, N = rhs.shape
    _check(load().sr_implicit_solve_noalloc(M, N, float(tau), float(mu), rhs.data_ptr(), u_out.data_ptr(),
                                            _stream_ptr(stream)))
    return u_out


def sr_prepare(ctx):
    _check(load().sr_prepare(ctx))


def sr_build_id():
    return load().sr_build_id().decode()


def sr_destroy(ctx):
    if ctx:
        load().sr_destroy(ctx)


def sr_batch_workspace_size(items):
    arr = (sr_batch_item * len(items))(*items)
    n = C.c_size_t()
    _check(load().sr_batch_workspace_size(arr, len(items), C.byref(n)))
    return n.value


def sr_solve_batch(items, workspace, stream=None):
    """Solve a list of sr_batch_item in place (their outputs are filled)."""
    arr = (sr_batch_item * len(items))(*items)
    rc = load().sr_solve_batch(arr, len(items), workspace.data_ptr(), workspace.numel(), _stream_ptr(stream))
    _check(rc, allow_warning=True)
    for i in range(len(items)):
        items[i] = arr[i]
    return rc


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------
class Solver:
    """One image: owns the workspace tensor and the library context."""

    def __init__(self, M, N, params=None, device="cuda", stream=None, **overrides):
        import torch
        self.M, self.N = M, N
        self.params = params if params is not None else sr_params_default(**overrides)
        nbytes = sr_workspace_size(M, N, self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.stream = stream
        self.ctx = sr_create(M, N, self.params, self._ws, stream)

    def close(self):
        if self.ctx:
            sr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, *shape):
        import torch
        return torch.empty(*shape, dtype=torch.float32, device=self.workspace.device)

    def set_image(self, f, phi0):
        sr_set_image(self.ctx, f, phi0)

    def step(self, n):
        rc, info = sr_step(self.ctx, n)
        return {"rc": rc, "iters_done": info.iters_done, "k": info.k, "r_last": info.r_last,
                "inner_steps": info.inner_steps, "converged": bool(info.converged)}

    def phi(self):
        return sr_get_phi(self.ctx, self._empty(self.M, self.N))

    def g(self):
        return sr_get_g(self.ctx, self._empty(self.M, self.N))

    def energy(self):
        return sr_energy(self.ctx)

    def get_state(self):
        phi = self._empty(self.M, self.N)
        w = self._empty(2, self.M, self.N)
        b = self._empty(2, self.M, self.N)
        k = sr_get_state(self.ctx, phi, w, b)
        return phi, w, b, k

    def set_state(self, phi, w, b, k=0):
        sr_set_state(self.ctx, phi, w, b, k)

    def autotune(self, reps=5):
        return sr_autotune(self.ctx, reps)

    def prepare(self):
        sr_prepare(self.ctx)

    def edge_map(self, f):
        return sr_edge_map(self.ctx, f, self._empty(self.M, self.N))

    def repulsion(self, w, phi):
        return sr_repulsion(self.ctx, w, phi, self._empty(2, self.M, self.N))

    def implicit_solve(self, rhs):
        return sr_implicit_solve(self.ctx, rhs, self._empty(self.M, self.N))


def solve_batch(items, stream=None):
    """Batched solve.  `items` is a list of dicts with keys f, phi0 (contiguous
    float32 GPU tensors), max_iter, and optional params (an sr_params) or
    parameter overrides under "params_kw", and want_state (also return the
    final w and b).  Returns a list of dicts with phi (tensor), iters,
    status, r_last, energy (and w, b)."""
    import torch
    cs = []
    outs = []
    states = []
    for it in items:
        f, phi0 = it["f"], it["phi0"]
        M, N = f.shape
        p = it.get("params") or sr_params_default(**it.get("params_kw", {}))
        out = torch.empty_like(f)
        outs.append(out)
        bi = sr_batch_item()
        bi.M, bi.N = M, N
        bi.f, bi.phi0, bi.phi_out = _ptr(f, False)[0], _ptr(phi0, False)[0], out.data_ptr()
        bi.params = p
        bi.max_iter = int(it["max_iter"])
        if it.get("want_state"):   # final w and b as well
            wo = torch.empty((2, M, N), dtype=torch.float32, device=f.device)
            bo = torch.empty((2, M, N), dtype=torch.float32, device=f.device)
            states.append((wo, bo))
            bi.w_out, bi.b_out = wo.data_ptr(), bo.data_ptr()
        else:
            states.append(None)
        cs.append(bi)
    nbytes = sr_batch_workspace_size(cs)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=items[0]["f"].device)
    off = (-ws.data_ptr()) % 256
    rc = sr_solve_batch(cs, ws[off:off + nbytes], stream)
    res = [{"phi": outs[i], "iters": cs[i].iters, "status": cs[i].status, "r_last": cs[i].r_last,
            "energy": cs[i].energy} for i in range(len(cs))]
    for r, stt in zip(res, states):
        if stt is not None:
            r["w"], r["b"] = stt
    return rc, res


# ---------------------------------------------------------------------------
# 3-D solver (include/sr3d.h); device tensors only
# ---------------------------------------------------------------------------
KERNEL_KINDS_3D = ("window", "rhs", "fft", "w_step")


def _dev(x):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
        raise ValueError("the 3-D entry points take contiguous float32 GPU tensors")
    return x.data_ptr()


def sr3_workspace_size(M, N, P, params):
    n = C.c_size_t()
    _check(load().sr3_workspace_size(M, N, P, C.byref(params), C.byref(n)))
    return n.value


def sr3_create(M, N, P, params, workspace, stream=None):
    ctx = C.c_void_p()
    st = stream.cuda_stream if stream is not None else None
    _check(load().sr3_create(C.byref(ctx), M, N, P, C.byref(params), workspace.data_ptr(), workspace.numel(), st))
    return ctx


def sr3_set_image(ctx, f, phi0):
    _check(load().sr3_set_image(ctx, _dev(f), _dev(phi0)))


def sr3_set_state(ctx, phi, w, b, k):
    _check(load().sr3_set_state(ctx, _dev(phi), _dev(w), _dev(b), int(k)))


def sr3_step(ctx, n_iter):
    k = C.c_int64()
    _check(load().sr3_step(ctx, n_iter, C.byref(k)))
    return k.value


def sr3_get_state(ctx, phi=None, w=None, b=None, g=None):
    ptr = lambda x: _dev(x) if x is not None else None
    _check(load().sr3_get_state(ctx, ptr(phi), ptr(w), ptr(b), ptr(g)))


def sr3_profile(ctx, n_iter):
    ms = (C.c_double * 4)()
    cnt = (C.c_int64 * 4)()
    _check(load().sr3_profile(ctx, n_iter, ms, cnt))
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS_3D)}


def sr3_destroy(ctx):
    if ctx:
        load().sr3_destroy(ctx)


class Solver3D:
    """One M x N x P volume: owns the workspace tensor and the context."""

    def __init__(self, M, N, P, params=None, device="cuda", stream=None, **overrides):
        import torch
        self.shape = (M, N, P)
        self.params = params if params is not None else sr_params_default(**overrides)
        nbytes = sr3_workspace_size(M, N, P, self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.ctx = sr3_create(M, N, P, self.params, self._ws, stream)

    def close(self):
        if self.ctx:
            sr3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, *lead):
        import torch
        return torch.empty(*lead, *self.shape, dtype=torch.float32, device=self.workspace.device)

    def set_image(self, f, phi0):
        sr3_set_image(self.ctx, f, phi0)

    def set_state(self, phi, w, b, k):
        sr3_set_state(self.ctx, phi, w, b, k)

    def step(self, n):
        return sr3_step(self.ctx, n)

    def get_state(self):
        phi, w, b, g = self._empty(), self._empty(3), self._empty(3), self._empty()
        sr3_get_state(self.ctx, phi, w, b, g)
        return phi, w, b, g
