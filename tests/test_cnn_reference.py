"""Pins of the FP64 warm-start network reference: its hand-written gradient
against central finite differences of its own loss, and the layer adjoints
against their definitions (<A x, y> = <x, A^T y>)."""
import numpy as np
import pytest

from oracle import cnn_reference as C

RNG = np.random.default_rng(7)


def test_layer_adjoints():
    x = RNG.normal(size=(2, 8, 8, 3))
    w = RNG.normal(size=(5, 3, 3, 3))
    b = RNG.normal(size=5)
    dy = RNG.normal(size=(2, 8, 8, 5))
    dx, dw, db = C.conv3x3_backward(x, w, dy)
    y0 = C.conv3x3(x, w, np.zeros(5))
    assert np.sum(y0 * dy) == pytest.approx(np.sum(x * dx), rel=1e-12)
    assert np.sum(C.conv3x3(x, w, b) - y0) == pytest.approx(np.sum(b) * 2 * 8 * 8, rel=1e-12)
    e = RNG.normal(size=w.shape)
    # linear in w: <conv(x; e), dy> = <e, dw>
    assert np.sum(C.conv3x3(x, e, np.zeros(5)) * dy) == pytest.approx(np.sum(e * dw), rel=1e-12)
    p = RNG.normal(size=(2, 8, 8, 4))
    q = RNG.normal(size=(2, 4, 4, 4))
    assert np.sum(C.pool(p) * q) == pytest.approx(np.sum(p * C.pool_backward(q)), rel=1e-12)
    r = RNG.normal(size=(2, 4, 4, 4))
    assert np.sum(C.upsample(r) * p) == pytest.approx(np.sum(r * C.upsample_backward(p)), rel=1e-12)


def test_conv_brute_force():
    x = RNG.normal(size=(1, 5, 6, 2))
    w = RNG.normal(size=(3, 2, 3, 3))
    b = RNG.normal(size=3)
    y = C.conv3x3(x, w, b)
    for i in range(5):
        for j in range(6):
            for o in range(3):
                s = b[o]
                for ky in range(3):
                    for kx in range(3):
                        ii, jj = i + ky - 1, j + kx - 1
                        if 0 <= ii < 5 and 0 <= jj < 6:
                            s += np.dot(w[o, :, ky, kx], x[0, ii, jj, :])
                assert y[0, i, j, o] == pytest.approx(s, rel=1e-12, abs=1e-12)


def test_gradient_by_finite_differences():
    params = C.init_params(3)
    for k in params["b"]:
        params["b"][k] = RNG.normal(scale=0.1, size=params["b"][k].shape)
    x = RNG.normal(size=(2, 16, 16, 3))
    target = RNG.normal(size=(2, 16, 16))
    loss, grads = C.loss_and_grad(params, x, target)
    flat = C.flatten(params)
    gflat = C.flatten(grads)
    idx = RNG.choice(len(flat), size=60, replace=False)
    h = 1e-6
    for i in idx:
        fp = flat.copy(); fp[i] += h
        fm = flat.copy(); fm[i] -= h
        lp, _ = C.loss_and_grad(C.unflatten(fp), x, target)
        lm, _ = C.loss_and_grad(C.unflatten(fm), x, target)
        fd = (lp - lm) / (2 * h)
        assert gflat[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_parameter_count():
    n = sum(int(np.prod(ws)) + int(np.prod(bs)) for _, ws, bs in C.param_shapes())
    assert n == len(C.flatten(C.init_params(0)))
    assert 400_000 < n < 700_000


def test_adam_first_step_is_signed_learning_rate():
    # from zero moments the bias-corrected first step is lr*g/(|g|+eps)
    rng = np.random.default_rng(3)
    g = rng.normal(size=50)
    p0 = rng.normal(size=50)
    p1, m, v = C.adam_step(p0, np.zeros(50), np.zeros(50), g, 1, 1e-3, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(p0 - p1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_keeps_unit_steps():
    # a constant gradient keeps the corrected ratio m_hat/sqrt(v_hat) at sign(g)
    g = np.array([2.0, -0.5, 1e-3])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 30):
        q, m, v = C.adam_step(p, m, v, g, t, 0.01, 0.9, 0.999, 0.0)
        np.testing.assert_allclose(p - q, 0.01 * np.sign(g), rtol=1e-10)
        p = q


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, size=4000),
                        1.0 + np.arange(64) * 2.0 ** -9,          # halfway cases
                        [0.0, -0.0, 1e-40, -3.0e38, 65504.0]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(C.bf16(x), want)


def test_bf16_network_close_to_exact_network():
    # storage rounding perturbs the prediction at the level of the bf16 unit
    # roundoff (2^-9) times the depth, not more
    rng = np.random.default_rng(5)
    params = C.init_params(2)
    x = rng.normal(size=(1, 16, 16, 3))
    y, _ = C.forward(params, x)
    yq, _ = C.forward(params, x, C.bf16)
    rel = np.linalg.norm(yq - y) / np.linalg.norm(y)
    assert 1e-4 < rel < 15 * 2.0 ** -9
