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
