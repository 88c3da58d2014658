"""Python binding of the warm-start network ABI (include/cnn.h): argument
marshalling only.

The network's forward pass, loss, backward pass and Adam step run in the HIP
kernels of libsr.so (csrc/cnn.hip); this module converts torch tensors to
device pointers and raises on error codes.  No CPU fallback exists.

``Network`` owns the workspace tensor of one context.
"""
from __future__ import annotations

import ctypes as C

from .sr import SRError, _stream_ptr, load as _load_sr

_cnn_lib = None


def load():
    """libsr.so with the cnn_* signatures declared."""
    global _cnn_lib
    if _cnn_lib is not None:
        return _cnn_lib
    lib = _load_sr()
    P, I, F = C.c_void_p, C.c_int32, C.c_float
    sig = {
        "cnn_num_params": (C.c_int, [C.POINTER(C.c_int64)]),
        "cnn_workspace_size": (C.c_int, [I, I, I, C.POINTER(C.c_size_t)]),
        "cnn_create": (C.c_int, [C.POINTER(P), I, I, I, P, C.c_size_t, P]),
        "cnn_set_params": (C.c_int, [P, P]),
        "cnn_get_params": (C.c_int, [P, P]),
        "cnn_forward": (C.c_int, [P, P, P, P, I, F, P]),
        "cnn_get_activation": (C.c_int, [P, I, P]),
        "cnn_backward": (C.c_int, [P, P, F, C.POINTER(C.c_double), P]),
        "cnn_adam_step": (C.c_int, [P, F, F, F, F]),
        "cnn_destroy": (None, [P]),
        "cnn_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _cnn_lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise SRError(rc, load().cnn_last_error().decode())
    return rc


def _dev(x, allow_none=False):
    import torch
    if x is None and allow_none:
        return None
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous():
        raise ValueError("expected a contiguous float32 GPU tensor")
    return x.data_ptr()


# ---------------------------------------------------------------------------
# same-name wrappers
# ---------------------------------------------------------------------------
def cnn_num_params():
    n = C.c_int64()
    _check(load().cnn_num_params(C.byref(n)))
    return n.value


def cnn_workspace_size(batch, H, W):
    n = C.c_size_t()
    _check(load().cnn_workspace_size(batch, H, W, C.byref(n)))
    return n.value


def cnn_create(batch, H, W, workspace, stream=None):
    import torch
    assert workspace.is_cuda and workspace.dtype == torch.uint8
    ctx = C.c_void_p()
    _check(load().cnn_create(C.byref(ctx), batch, H, W, workspace.data_ptr(), workspace.numel(),
                             _stream_ptr(stream)))
    return ctx


def cnn_set_params(ctx, params):
    _check(load().cnn_set_params(ctx, _dev(params)))


def cnn_get_params(ctx, out):
    _check(load().cnn_get_params(ctx, _dev(out)))
    return out


def cnn_forward(ctx, f, g, phi0, n, clip, phi_pred=None):
    _check(load().cnn_forward(ctx, _dev(f), _dev(g), _dev(phi0), n, clip, _dev(phi_pred, True)))
    return phi_pred


def cnn_get_activation(ctx, which, out):
    _check(load().cnn_get_activation(ctx, which, _dev(out)))
    return out


def cnn_backward(ctx, target, clip, grad_out=None, want_loss=True):
    loss = C.c_double()
    _check(load().cnn_backward(ctx, _dev(target), clip, C.byref(loss) if want_loss else None,
                               _dev(grad_out, True)))
    return loss.value if want_loss else None


def cnn_adam_step(ctx, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(load().cnn_adam_step(ctx, lr, beta1, beta2, eps))


def cnn_destroy(ctx):
    load().cnn_destroy(ctx)


# (name, cin, cout, level) of the 3x3 layers in parameter order, then the
# 1x1 head (16 -> 1); the library's flat parameter vector follows this order
# with each layer's weights [cout][cin][3][3] before its biases.
LAYERS = [("L0a", 3, 16, 0), ("L0b", 16, 16, 0), ("L1a", 16, 32, 1), ("L1b", 32, 32, 1),
          ("L2a", 32, 64, 2), ("L2b", 64, 64, 2), ("L3a", 64, 128, 3), ("L3b", 128, 128, 3),
          ("U2", 128, 64, 2), ("D2", 128, 64, 2), ("U1", 64, 32, 1), ("D1", 64, 32, 1),
          ("U0", 32, 16, 0), ("D0", 32, 16, 0)]


def he_init(seed):
    """Flat FP32 parameter vector: He-normal weights, zero biases."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = []
    for _, cin, cout, _ in LAYERS:
        parts += [rng.normal(0.0, np.sqrt(2.0 / (9 * cin)), cout * cin * 9), np.zeros(cout)]
    parts += [rng.normal(0.0, np.sqrt(2.0 / 16), 16), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def flops(n, H, W):
    """(forward, training step) floating-point operations of the network on n
    images of H x W: 2 per multiply-add of every 3x3 layer and the head; a
    training step adds each layer's data gradient (not the first layer's)
    and weight gradient."""
    fwd = train = 0
    for i, (_, cin, cout, lev) in enumerate(LAYERS):
        px = n * (H >> lev) * (W >> lev)
        f = 2 * px * 9 * cin * cout
        fwd += f
        train += f * (3 if i else 2)
    head = 2 * n * H * W * 16
    return fwd + head, train + 3 * head


# channels and level of the tensors cnn_get_activation returns
ACT_SHAPE = {0: (16, 0), 1: (16, 0), 2: (32, 1), 3: (32, 1), 4: (64, 2), 5: (64, 2), 6: (128, 3),
             7: (128, 3), 8: (64, 2), 9: (64, 2), 10: (32, 1), 11: (32, 1), 12: (16, 0), 13: (16, 0),
             14: (4, 0), 15: (1, 0), 16: (16, 1), 17: (32, 2), 18: (64, 3)}
ACT_SHAPE.update({19 + i: ACT_SHAPE[i] for i in range(14)})   # masked output gradients


class Network:
    """A context plus its workspace (batch images of H x W at most)."""

    def __init__(self, batch, H, W, params=None, stream=None):
        import torch
        self.batch, self.H, self.W = batch, H, W
        self.ws = torch.empty(cnn_workspace_size(batch, H, W), dtype=torch.uint8, device="cuda")
        self.ctx = cnn_create(batch, H, W, self.ws, stream)
        self.np = cnn_num_params()
        if params is not None:
            self.set_params(params)

    def set_params(self, params):
        import torch
        t = torch.as_tensor(params, dtype=torch.float32).to("cuda").contiguous()
        if t.numel() != self.np:
            raise ValueError(f"expected {self.np} parameters, got {t.numel()}")
        cnn_set_params(self.ctx, t)

    def get_params(self):
        import torch
        out = torch.empty(self.np, dtype=torch.float32, device="cuda")
        return cnn_get_params(self.ctx, out)

    def forward(self, f, g, phi0, clip, want_output=True):
        import torch
        n = f.shape[0]
        out = torch.empty_like(f) if want_output else None
        cnn_forward(self.ctx, f, g, phi0, n, clip, out)
        return out

    def activation(self, which, n):
        """Stored tensor `which` of the last forward on n images, FP32 (n, H_l, W_l, C)."""
        import torch
        C_, lev = ACT_SHAPE[which]
        out = torch.empty((n, self.H >> lev, self.W >> lev, C_), dtype=torch.float32, device="cuda")
        return cnn_get_activation(self.ctx, which, out)

    def backward(self, target, clip, want_grad=False):
        import torch
        grad = torch.empty(self.np, dtype=torch.float32, device="cuda") if want_grad else None
        loss = cnn_backward(self.ctx, target, clip, grad)
        return loss, grad

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        cnn_adam_step(self.ctx, lr, beta1, beta2, eps)

    def close(self):
        if self.ctx is not None:
            cnn_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
