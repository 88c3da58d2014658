"""The warm-start network at its benchmark size (512 x 512, spatially tiled
kernels for every layer but the first), checked on sampled outputs: each
stored activation and masked gradient at sampled pixels against the
reference layer on the library's own stored inputs (a 3x3 neighbourhood is
all a pixel reads), and three layers' weight gradients against the exact
sums over the library's own operands."""
import sys

import numpy as np
import pytest

from oracle import cnn_reference as R
from tests.helpers import f32
from tests.test_gpu_cnn import ACC_REL, CLIP, _inputs, _params

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

n, H, W = 2, 512, 512


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _patch(x, b, i, j):
    """3x3 neighbourhood of pixel (i, j) of image b, zeros outside (the layer's padding)."""
    Hh, Ww, C = x.shape[1:]
    out = np.zeros((3, 3, C))
    for dy in range(3):
        for dx in range(3):
            ii, jj = i + dy - 1, j + dx - 1
            if 0 <= ii < Hh and 0 <= jj < Ww:
                out[dy, dx] = x[b, ii, jj]
    return out


def _conv_at(x, w, bias, b, i, j):
    p = _patch(x, b, i, j)
    z = np.einsum("yxc,ocyx->o", p, w) + bias
    za = np.einsum("yxc,ocyx->o", np.abs(p), np.abs(w)) + np.abs(bias)
    return z, za


def _samples(Hh, Ww, rng, k=48):
    pts = [(0, 0, 0), (1, Hh - 1, Ww - 1), (0, 0, Ww - 1), (1, Hh - 1, 0), (0, 15, 16), (1, 16, 15),
           (0, Hh // 2, Ww // 2 - 1)]
    pts += [(int(rng.integers(n)), int(rng.integers(Hh)), int(rng.integers(Ww))) for _ in range(k)]
    return pts


def _check(got, want, z, za, what):
    d = np.abs(got - want)
    allowed = 2.0 ** -7 * np.maximum(np.abs(got), np.abs(want)) + ACC_REL * za
    assert np.all(d <= allowed), (what, float(d.max()))
    return int(np.sum(got != want))


def test_network_full_size_sampled():
    from paper_2003_12693_amd import cnn
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _note("network 2 x 512^2: sampled layers, masks and weight gradients")
    params = _params(21)
    f, g, phi0, target = _inputs(n, H, W, 22)
    net = cnn.Network(n, H, W, R.flatten(params))
    cu = lambda a: torch.from_numpy(f32(a)).cuda()
    net.forward(cu(f), cu(g), cu(phi0), CLIP, want_output=False)
    loss, grad = net.backward(cu(target), CLIP, want_grad=True)
    grad = grad.cpu().numpy().astype(np.float64)
    A = {k: net.activation(k, n).cpu().numpy().astype(np.float64) for k in range(19)}
    names = [l[0] for l in R.LAYERS]
    DZ = {nm: net.activation(19 + i, n).cpu().numpy().astype(np.float64) for i, nm in enumerate(names)}
    w = {k: R.bf16(v) for k, v in params["w"].items()}
    b = params["b"]
    up = lambda x: R.upsample(x)
    inputs = {"L0a": A[14][..., :3], "L0b": A[0], "L1a": A[16], "L1b": A[2], "L2a": A[17], "L2b": A[4],
              "L3a": A[18], "L3b": A[6], "U2": None, "D2": np.concatenate([A[8], A[5]], axis=3), "U1": None,
              "D1": np.concatenate([A[10], A[3]], axis=3), "U0": None, "D0": np.concatenate([A[12], A[1]], axis=3)}
    outputs = {"L0a": A[0], "L0b": A[1], "L1a": A[2], "L1b": A[3], "L2a": A[4], "L2b": A[5], "L3a": A[6],
               "L3b": A[7], "U2": A[8], "D2": A[9], "U1": A[10], "D1": A[11], "U0": A[12], "D0": A[13]}
    coarse = {"U2": A[7], "U1": A[9], "U0": A[11]}
    rng = np.random.default_rng(23)
    flips = 0
    for nm in names:
        out = outputs[nm]
        x = inputs[nm] if inputs[nm] is not None else up(coarse[nm])
        for (bi, i, j) in _samples(out.shape[1], out.shape[2], rng):
            z, za = _conv_at(x, w[nm], b[nm], bi, i, j)
            flips += _check(out[bi, i, j], R.bf16(R.relu(z)), z, za, f"{nm} at {(bi, i, j)}")
    # masked gradients fed by a 3x3 data gradient (L0a <- L0b) and by the 2x2 sum of
    # an upsampled layer's data gradient (L3b <- U2)
    wr = lambda nm: w[nm][:, :, ::-1, ::-1].transpose(1, 0, 2, 3)     # turned stencil, [cin][cout]
    for (bi, i, j) in _samples(H, W, rng, 24):
        dx, dxa = _conv_at(DZ["L0b"], wr("L0b"), np.zeros(16), bi, i, j)
        want = R.bf16(dx * (A[0][bi, i, j] > 0))
        flips += _check(DZ["L0a"][bi, i, j], want, dx, dxa, f"dz L0a at {(bi, i, j)}")
    for (bi, i, j) in _samples(H >> 3, W >> 3, rng, 24):
        s, sa = np.zeros(128), np.zeros(128)
        for di in range(2):
            for dj in range(2):
                dx, dxa = _conv_at(DZ["U2"], wr("U2"), np.zeros(128), bi, 2 * i + di, 2 * j + dj)
                s, sa = s + dx, sa + dxa
        want = R.bf16(s * (A[7][bi, i, j] > 0))
        flips += _check(DZ["L3b"][bi, i, j], want, s, sa, f"dz L3b at {(bi, i, j)}")
    # weight / bias gradients of three layers: exact sums over the library's operands
    off, o = {}, 0
    for name, ws, bs in R.param_shapes():
        nw_, nb_ = int(np.prod(ws)), int(np.prod(bs))
        off[name] = (o, o + nw_, o + nw_ + nb_)
        o += nw_ + nb_
    for nm, x in (("L3b", inputs["L3b"]), ("U2", up(coarse["U2"])), ("L0a", inputs["L0a"])):
        _, gw_, gb_ = R.conv3x3_backward(x, w[nm], DZ[nm])
        _, aw, ab = R.conv3x3_backward(np.abs(x), np.abs(w[nm]), np.abs(DZ[nm]))
        a0, a1, a2 = off[nm]
        assert np.all(np.abs(grad[a0:a1].reshape(gw_.shape) - gw_) <= ACC_REL * aw + 1e-12), nm
        assert np.all(np.abs(grad[a1:a2] - gb_) <= ACC_REL * ab + 1e-12), nm
    _note(f"  loss {loss:.5f}; {flips} sampled values one bf16 rounding step from the reference")
