"""FP64 NumPy reference of the warm-start network (test infrastructure only).

The learned warm start predicts a near-converged level set from (image f,
edge map g, initial phi^0); the Split Bregman solver then refines it.  The
network is a 4-level encoder-decoder: 3x3 convolutions (zero padding) with
16 -> 32 -> 64 -> 128 channels, two per level, ReLU, 2x2 average pooling
down, nearest upsampling followed by a 3x3 convolution up, concatenated skip
connections and a 1x1 head.  This module is the plain definition of that
network and of its gradient (written out by hand), used to check the HIP
implementation; it is pinned by finite differences in tests/test_cnn_reference.py.

Tensors are channels-last (N, H, W, C).  Parameters are a dict of arrays:
w[name] with shape (cout, cin, 3, 3) (or (cout, cin) for the head) and
b[name] with shape (cout,).
"""
from __future__ import annotations

import numpy as np

# (name, cin, cout) of the 3x3 convolutions in forward order, then the head.
LAYERS = [
    ("L0a", 3, 16), ("L0b", 16, 16),
    ("L1a", 16, 32), ("L1b", 32, 32),
    ("L2a", 32, 64), ("L2b", 64, 64),
    ("L3a", 64, 128), ("L3b", 128, 128),
    ("U2", 128, 64), ("D2", 128, 64),
    ("U1", 64, 32), ("D1", 64, 32),
    ("U0", 32, 16), ("D0", 32, 16),
]
HEAD = ("head", 16, 1)


def param_shapes():
    out = []
    for name, cin, cout in LAYERS:
        out.append((name, (cout, cin, 3, 3), (cout,)))
    out.append((HEAD[0], (HEAD[2], HEAD[1]), (HEAD[2],)))
    return out


def flatten(params):
    """Flat vector in the library's order: for each layer weights then bias."""
    parts = []
    for name, ws, bs in param_shapes():
        parts.append(params["w"][name].reshape(-1))
        parts.append(params["b"][name].reshape(-1))
    return np.concatenate(parts)


def unflatten(vec):
    params = {"w": {}, "b": {}}
    o = 0
    for name, ws, bs in param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        params["w"][name] = vec[o:o + nw].reshape(ws).astype(np.float64)
        o += nw
        params["b"][name] = vec[o:o + nb].reshape(bs).astype(np.float64)
        o += nb
    assert o == len(vec)
    return params


def init_params(seed):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    params = {"w": {}, "b": {}}
    for name, ws, bs in param_shapes():
        fan_in = int(np.prod(ws[1:]))
        params["w"][name] = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=ws)
        params["b"][name] = np.zeros(bs)
    return params


# --------------------------------------------------------------------------
# layers
# --------------------------------------------------------------------------
def conv3x3(x, w, b):
    """y[n,i,j,o] = b[o] + sum_{ky,kx,c} w[o,c,ky,kx] x[n,i+ky-1,j+kx-1,c], zero padding."""
    N, H, W, C = x.shape
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.zeros((N, H, W, w.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("nijc,oc->nijo", xp[:, ky:ky + H, kx:kx + W, :], w[:, :, ky, kx])
    return y


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 w.r.t. x, w, b given dy."""
    N, H, W, C = x.shape
    xp = np.zeros((N, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.einsum("nijc,nijo->oc", xp[:, ky:ky + H, kx:kx + W, :], dy)
            dxp[:, ky:ky + H, kx:kx + W, :] += np.einsum("nijo,oc->nijc", dy, w[:, :, ky, kx])
    return dxp[:, 1:-1, 1:-1, :], dw, dy.sum(axis=(0, 1, 2))


def relu(z):
    return np.maximum(z, 0.0)


def pool(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def upsample(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample_backward(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# --------------------------------------------------------------------------
# storage precision
# --------------------------------------------------------------------------
def bf16(x):
    """Round to bfloat16 (8 significant bits, float32 exponent range) to
    nearest, ties to even, via float32; returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(x):
    return x


# --------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------
def forward(params, x, q=None):
    """x: (N, H, W, 3) -> (prediction (N, H, W), cache of activations).

    q is the storage rounding of the network's tensors (None: exact FP64;
    bf16: the network as specified, with BF16 input, 3x3 weights and stored
    activations, every sum taken exactly).  The head weights and all biases
    stay unrounded."""
    q = q or _ident
    w, b = params["w"], params["b"]
    a = {}

    def cr(name, inp):
        a[name + ".in"] = inp
        z = conv3x3(inp, q(w[name]), b[name])
        out = q(relu(z))
        a[name] = out
        return out

    x = q(x)
    s0 = cr("L0b", cr("L0a", x))
    s1 = cr("L1b", cr("L1a", q(pool(s0))))
    s2 = cr("L2b", cr("L2a", q(pool(s1))))
    bott = cr("L3b", cr("L3a", q(pool(s2))))
    d2 = cr("D2", np.concatenate([cr("U2", upsample(bott)), s2], axis=3))
    d1 = cr("D1", np.concatenate([cr("U1", upsample(d2)), s1], axis=3))
    d0 = cr("D0", np.concatenate([cr("U0", upsample(d1)), s0], axis=3))
    a["head.in"] = d0
    y = np.einsum("nijc,oc->nijo", d0, w["head"]) + b["head"]
    return y[..., 0], a


def loss_and_grad(params, x, target, q=None):
    """Mean squared error of the prediction against `target` (N, H, W) and its
    gradient w.r.t. every parameter (same dict layout).  With q, the masked
    output gradient of every 3x3 layer is stored rounded by q as well."""
    qq = q or _ident
    w, b = params["w"], params["b"]
    y, a = forward(params, x, q)
    n = y.size
    diff = y - target
    loss = float(np.mean(diff * diff))
    gw, gb = {}, {}
    dy = (2.0 / n) * diff[..., None]
    gw["head"] = np.einsum("nijc,nijo->oc", a["head.in"], dy)
    gb["head"] = dy.sum(axis=(0, 1, 2))
    dd0 = np.einsum("nijo,oc->nijc", dy, w["head"])

    def back(name, dout):
        dz = qq(dout * (a[name] > 0))
        dx, gw[name], gb[name] = conv3x3_backward(a[name + ".in"], qq(w[name]), dz)
        return dx

    # decoder, level 0 -> 2
    dcat0 = back("D0", dd0)
    dd1 = upsample_backward(back("U0", dcat0[..., :16]))
    ds0 = dcat0[..., 16:]
    dcat1 = back("D1", dd1)
    dd2 = upsample_backward(back("U1", dcat1[..., :32]))
    ds1 = dcat1[..., 32:]
    dcat2 = back("D2", dd2)
    dbott = upsample_backward(back("U2", dcat2[..., :64]))
    ds2 = dcat2[..., 64:]
    # encoder, level 3 -> 0
    dp2 = back("L3a", back("L3b", dbott))
    ds2 = ds2 + pool_backward(dp2)
    dp1 = back("L2a", back("L2b", ds2))
    ds1 = ds1 + pool_backward(dp1)
    dp0 = back("L1a", back("L1b", ds1))
    ds0 = ds0 + pool_backward(dp0)
    back("L0a", back("L0b", ds0))
    return loss, {"w": gw, "b": gb}


def make_input(f, g, phi0, clip):
    """Network input channels (image, edge map, clipped / scaled phi^0)."""
    return np.stack([f, g, np.clip(phi0, -clip, clip) / clip], axis=-1)


def adam_step(p, m, v, g, t, lr, beta1, beta2, eps):
    """One Adam update (Kingma and Ba, 2015) with bias-corrected moments, on
    flat FP64 vectors; returns (p, m, v) after step number t (t >= 1)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
