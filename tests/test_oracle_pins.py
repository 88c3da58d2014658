"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names what it pins and what it compares against: closed forms,
derivative relations between the paper's equations checked by finite
differences, SciPy routines, brute-force sums written independently here,
the residual of the linear system the FFT solve claims to solve, and
symmetries of the whole iteration.
"""
import math

import numpy as np
import pytest
from scipy import ndimage, optimize

from oracle import sr_oracle as O

RNG = np.random.default_rng(12345)


# --------------------------------------------------------------------------
# eqs (5), (6), (11), (28), (29)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("eps", [1.0, 1.5, 2.0])
def test_heaviside_dirac_closed_values(eps):
    assert O.heaviside(0.0, eps) == pytest.approx(0.5, abs=1e-15)
    assert O.heaviside(eps, eps) == pytest.approx(1.0, abs=1e-15)
    assert O.heaviside(-eps, eps) == pytest.approx(0.0, abs=1e-15)
    assert O.heaviside(3 * eps, eps) == 1.0 and O.heaviside(-3 * eps, eps) == 0.0
    assert O.dirac(0.0, eps) == pytest.approx(1.0 / eps, rel=1e-15)
    assert O.dirac(eps, eps) == pytest.approx(0.0, abs=1e-15)
    assert O.dirac(1.01 * eps, eps) == 0.0
    # H(-x) = 1 - H(x): the smoothed Heaviside is point-symmetric about (0, 1/2)
    x = np.linspace(-2 * eps, 2 * eps, 101)
    np.testing.assert_allclose(O.heaviside(-x, eps), 1.0 - O.heaviside(x, eps), atol=1e-15)
    # unit mass of the Dirac (Simpson rule on its support)
    xs = np.linspace(-eps, eps, 20001)
    from scipy.integrate import simpson
    assert simpson(O.dirac(xs, eps), x=xs) == pytest.approx(1.0, abs=1e-12)


@pytest.mark.parametrize("eps,l", [(1.0, 1.0), (1.5, 1.0), (2.0, 1.0), (1.5, 2.0)])
def test_derivative_relations_by_finite_differences(eps, l):
    """delta = dH/dphi, delta' = d delta/dphi (eq 29), h' = dh/dphi (eq 28)."""
    x = np.linspace(-3 * eps - l, 3 * eps + l, 997) + 1e-3   # avoid the kink points
    e = 1e-6
    fd = lambda fun: (fun(x + e) - fun(x - e)) / (2 * e)
    np.testing.assert_allclose(O.dirac(x, eps), fd(lambda z: O.heaviside(z, eps)), atol=2e-8)
    np.testing.assert_allclose(O.dirac_prime(x, eps), fd(lambda z: O.dirac(z, eps)), atol=2e-8)
    np.testing.assert_allclose(O.band_prime(x, eps, l), fd(lambda z: O.band(z, eps, l)), atol=2e-8)


def test_band_values():
    """h(0) = H(l)(1 - H(-l)) = H(l)^2 by the point symmetry; h is 1 deep in
    the band when l > eps and vanishes beyond l + eps."""
    for eps, l in [(1.5, 1.0), (2.0, 1.0), (1.0, 1.0)]:
        H = float(O.heaviside(l, eps))
        assert O.band(0.0, eps, l) == pytest.approx(H * H, rel=1e-14)
        assert O.band(l + eps + 1e-9, eps, l) == 0.0
        assert O.band(-(l + eps + 1e-9), eps, l) == 0.0
    # with eps = 1.5, l = 1: H(1) = (1 + 2/3 + sin(2 pi/3)/pi)/2
    H1 = 0.5 * (1 + 2 / 3 + math.sqrt(3) / 2 / math.pi)
    assert O.band(0.0, 1.5, 1.0) == pytest.approx(H1 ** 2, rel=1e-14)
    assert O.band(0.0, 0.5, 2.0) == 1.0


# --------------------------------------------------------------------------
# eqs (35), (36): discrete operators
# --------------------------------------------------------------------------
def test_divergence_is_negative_adjoint_of_gradient():
    u = RNG.normal(size=(9, 13))
    p, q = RNG.normal(size=(9, 13)), RNG.normal(size=(9, 13))
    g1, g2 = O.grad_fwd(u)
    lhs = np.sum(g1 * p + g2 * q)
    rhs = -np.sum(u * O.div_bwd(p, q))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    np.testing.assert_allclose(O.laplacian(u), O.div_bwd(*O.grad_fwd(u)), atol=1e-13)


def test_operators_pointwise_brute_force():
    u = RNG.normal(size=(5, 6))
    M, N = u.shape
    g1, g2 = O.grad_fwd(u)
    p, q = RNG.normal(size=(5, 6)), RNG.normal(size=(5, 6))
    dv = O.div_bwd(p, q)
    lap = O.laplacian(u)
    for i in range(M):
        for j in range(N):
            assert g1[i, j] == pytest.approx(u[(i + 1) % M, j] - u[i, j], abs=1e-14)
            assert g2[i, j] == pytest.approx(u[i, (j + 1) % N] - u[i, j], abs=1e-14)
            assert dv[i, j] == pytest.approx(p[i, j] - p[i - 1, j] + q[i, j] - q[i, j - 1], abs=1e-14)
            nb = u[i - 1, j] + u[(i + 1) % M, j] + u[i, j - 1] + u[i, (j + 1) % N]
            assert lap[i, j] == pytest.approx(nb - 4 * u[i, j], abs=1e-13)


def test_laplacian_fourier_mode():
    M, N, a, c = 16, 32, 3, 5
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    u = np.cos(2 * np.pi * a * i / M) * np.cos(2 * np.pi * c * j / N)
    lam = (2 * math.cos(2 * math.pi * a / M) - 2) + (2 * math.cos(2 * math.pi * c / N) - 2)
    np.testing.assert_allclose(O.laplacian(u), lam * u, atol=1e-13)


# --------------------------------------------------------------------------
# eq (1): Gaussian smoothing and the edge map
# --------------------------------------------------------------------------
@pytest.mark.parametrize("sigma", [0.5, 1.0, 1.5, 2.0])
def test_gaussian_matches_scipy(sigma):
    f = RNG.normal(size=(24, 40))
    ref = ndimage.gaussian_filter1d(f, sigma, axis=1, mode="wrap", truncate=3.0)
    ref = ndimage.gaussian_filter1d(ref, sigma, axis=0, mode="wrap", truncate=3.0)
    # SciPy's radius int(3 sigma + 0.5) equals ceil(3 sigma) for these sigmas
    assert int(3 * sigma + 0.5) == math.ceil(3 * sigma)
    np.testing.assert_allclose(O.gaussian_smooth(f, sigma), ref, atol=1e-13)


def test_edge_map_constant_and_scipy():
    assert np.all(O.edge_map(np.full((16, 16), 0.3), 1.5, 1000.0, 2) == 1.0)
    f = RNG.uniform(size=(32, 48))
    fs = ndimage.gaussian_filter(f, 1.5, mode="wrap", truncate=3.0)
    gx = ndimage.correlate1d(fs, [-0.5, 0.0, 0.5], axis=0, mode="wrap")
    gy = ndimage.correlate1d(fs, [-0.5, 0.0, 0.5], axis=1, mode="wrap")
    for s in (1, 2):
        ref = 1.0 / (1.0 + 1000.0 * np.hypot(gx, gy) ** s)
        np.testing.assert_allclose(O.edge_map(f, 1.5, 1000.0, s), ref, rtol=1e-12)


# --------------------------------------------------------------------------
# the repulsion window sum
# --------------------------------------------------------------------------
def _window_sum_loops(w1, w2, phi, eps, l, d, R):
    M, N = phi.shape
    hh = O.band(phi, eps, l)
    v1 = np.zeros((M, N))
    v2 = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            for p in range(-R, R + 1):
                for q in range(-R, R + 1):
                    k = math.exp(-(p * p + q * q) / (d * d))
                    ii, jj = (i + p) % M, (j + q) % N
                    v1[i, j] += k * w1[ii, jj] * hh[ii, jj]
                    v2[i, j] += k * w2[ii, jj] * hh[ii, jj]
    return v1, v2


@pytest.mark.parametrize("shape,R,d", [((7, 9), 2, 2.0), ((8, 8), 3, 5.0), ((12, 11), 5, 5.0)])
def test_repulsion_brute_force(shape, R, d):
    phi = RNG.uniform(-4, 4, size=shape)
    w1, w2 = RNG.normal(size=shape), RNG.normal(size=shape)
    ref = _window_sum_loops(w1, w2, phi, 1.5, 1.0, d, R)
    got = O.repulsion_field(w1, w2, phi, 1.5, 1.0, d, R)
    np.testing.assert_allclose(got[0], ref[0], atol=1e-12)
    np.testing.assert_allclose(got[1], ref[1], atol=1e-12)


@pytest.mark.parametrize("R,d", [(3, 3.0), (4, 4.0), (5, 5.0), (3, 5.0)])
def test_repulsion_constant_field(R, d):
    """Constant w = e and phi = c give v = e h(c) (sum_p exp(-p^2/d^2))^2."""
    shape = (16, 16)
    e = (0.6, -0.8)
    c = 0.3
    a = sum(math.exp(-p * p / (d * d)) for p in range(-R, R + 1))
    v1, v2 = O.repulsion_field(np.full(shape, e[0]), np.full(shape, e[1]), np.full(shape, c), 1.5, 1.0, d, R)
    hc = float(O.band(c, 1.5, 1.0))
    np.testing.assert_allclose(v1, e[0] * hc * a * a, rtol=1e-13)
    np.testing.assert_allclose(v2, e[1] * hc * a * a, rtol=1e-13)


# --------------------------------------------------------------------------
# eqs (30)-(33): the semi-implicit solve
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,tau,mu", [((16, 16), 0.1, 8.0), ((8, 32), 0.4, 0.1), ((64, 32), 1.0, 3.0)])
def test_implicit_solve_residual(shape, tau, mu):
    F = RNG.normal(size=shape) * 50.0
    phi = O.implicit_solve(F, tau, mu)
    resid = phi - tau * mu * O.laplacian(phi) - F
    assert np.linalg.norm(resid) / np.linalg.norm(F) < 1e-13


def test_implicit_solve_modes():
    M, N, tau, mu = 32, 16, 0.1, 8.0
    # DC passes unchanged: the symbol is 1 at (0, 0)
    np.testing.assert_allclose(O.implicit_solve(np.full((M, N), 7.25), tau, mu), 7.25, atol=1e-12)
    # a single mode is scaled by 1 / (1 + tau mu (2 - 2 cos(2 pi a / M)))
    a = 5
    i = np.arange(M)[:, None] + np.zeros((1, N))
    F = np.cos(2 * np.pi * a * i / M)
    scale = 1.0 / (1.0 + tau * mu * (2 - 2 * math.cos(2 * math.pi * a / M)))
    np.testing.assert_allclose(O.implicit_solve(F, tau, mu), scale * F, atol=1e-13)


# --------------------------------------------------------------------------
# eqs (22), (26), (30), (37): the rhs is the negative gradient of the split energy
# --------------------------------------------------------------------------
def _kernel_matrix(M, N, R, d):
    """Dense K(x, y) on the periodic grid, truncated to the square window."""
    n = M * N
    K = np.zeros((n, n))
    for i in range(M):
        for j in range(N):
            for p in range(-R, R + 1):
                for q in range(-R, R + 1):
                    K[i * N + j, ((i + p) % M) * N + (j + q) % N] += math.exp(-(p * p + q * q) / (d * d))
    return K


def _split_energy(phi, w1, w2, b1, b2, g, P, K):
    """E(phi, w) of eq (22) on the grid, written directly from the definition
    with a dense kernel matrix for the double integral."""
    wn = np.sqrt(w1 ** 2 + w2 ** 2)
    Eg = np.sum(g * wn * O.dirac(phi, P.eps))
    Ea = np.sum(g * (1 - O.heaviside(phi, P.eps)))
    hv = O.band(phi, P.eps, P.band_l).ravel()
    W1, W2 = w1.ravel(), w2.ravel()
    Er = -(np.einsum("x,y,xy->", W1 * hv, W1 * hv, K) + np.einsum("x,y,xy->", W2 * hv, W2 * hv, K))
    M, N = phi.shape
    d1 = np.roll(phi, -1, 0) - phi
    d2 = np.roll(phi, -1, 1) - phi
    Es = 0.5 * P.mu * np.sum((w1 - d1 - b1) ** 2 + (w2 - d2 - b2) ** 2)
    return P.gamma * Eg + P.alpha * Ea + P.beta * Er + Es


def test_rhs_is_negative_gradient_of_split_energy():
    """(F - phi)/tau + mu Lap(phi) must equal -dE/dphi of eq (22) (the
    gradient flow of eq 26): pins every sign, the factor 2 beta, the window
    and the divergence/gradient pairing."""
    M, N = 8, 9
    P = O.Params(gamma=1.3, alpha=0.7, beta=0.45, mu=2.0, tau=0.3, eps=1.5, band_l=1.0, d=3.0, R=3)
    phi = RNG.uniform(-2.8, 2.8, size=(M, N))
    w1, w2 = RNG.normal(size=(M, N)), RNG.normal(size=(M, N))
    b1, b2 = 0.3 * RNG.normal(size=(M, N)), 0.3 * RNG.normal(size=(M, N))
    g = RNG.uniform(0.05, 1.0, size=(M, N))
    K = _kernel_matrix(M, N, P.R, P.d)
    F = O.phi_rhs(phi, w1, w2, b1, b2, g, P)
    flow = (F - phi) / P.tau + P.mu * O.laplacian(phi)
    h = 1e-6
    grad = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            pp = phi.copy(); pp[i, j] += h
            pm = phi.copy(); pm[i, j] -= h
            grad[i, j] = (_split_energy(pp, w1, w2, b1, b2, g, P, K)
                          - _split_energy(pm, w1, w2, b1, b2, g, P, K)) / (2 * h)
    np.testing.assert_allclose(flow, -grad, atol=2e-6 * np.abs(grad).max())


def test_shrink_input_is_linearised_w_energy():
    """mu B of eq (41) is mu (grad phi + b) minus the gradient in w of the
    repulsion part of eq (22) at w = w^k (the frozen integral of eq 41)."""
    M, N = 7, 8
    P = O.Params(gamma=1.0, alpha=1.0, beta=0.6, mu=1.7, tau=0.2, eps=1.5, band_l=1.0, d=2.5, R=3)
    phi = RNG.uniform(-2.8, 2.8, size=(M, N))
    w1, w2 = RNG.normal(size=(M, N)), RNG.normal(size=(M, N))
    b1, b2 = RNG.normal(size=(M, N)), RNG.normal(size=(M, N))
    g = RNG.uniform(0.05, 1.0, size=(M, N))
    K = _kernel_matrix(M, N, P.R, P.d)
    hv = O.band(phi, P.eps, P.band_l).ravel()

    def Er(W1, W2):
        return -P.beta * (np.einsum("x,y,xy->", W1 * hv, W1 * hv, K) + np.einsum("x,y,xy->", W2 * hv, W2 * hv, K))

    e = 1e-6
    gr1 = np.zeros(M * N)
    gr2 = np.zeros(M * N)
    W1, W2 = w1.ravel().copy(), w2.ravel().copy()
    for x in range(M * N):
        for comp, out in ((W1, gr1), (W2, gr2)):
            old = comp[x]
            comp[x] = old + e; ep = Er(W1, W2)
            comp[x] = old - e; em = Er(W1, W2)
            comp[x] = old
            out[x] = (ep - em) / (2 * e)
    B1, B2, t = O.shrink_input(phi, w1, w2, b1, b2, g, P)
    G1, G2 = O.grad_fwd(phi)
    np.testing.assert_allclose(P.mu * B1, P.mu * (G1 + b1) - gr1.reshape(M, N), atol=1e-6)
    np.testing.assert_allclose(P.mu * B2, P.mu * (G2 + b2) - gr2.reshape(M, N), atol=1e-6)
    np.testing.assert_allclose(t, (P.gamma / P.mu) * g * O.dirac(phi, P.eps), rtol=1e-15)


# --------------------------------------------------------------------------
# eqs (40), (42): shrinkage and projection
# --------------------------------------------------------------------------
def test_shrink_closed_forms():
    s = O.shrink(np.array([3.0, 0.3, 0.0]), np.array([4.0, 0.4, 0.0]), np.array([2.0, 1.0, 0.5]))
    np.testing.assert_allclose(s[0], [1.8, 0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(s[1], [2.4, 0.0, 0.0], atol=1e-15)
    p = O.project(s[0], s[1])
    np.testing.assert_allclose(p[0], [0.6, 0.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(p[1], [0.8, 0.0, 0.0], atol=1e-15)


def test_shrink_is_pointwise_minimiser():
    """max(|B| - t, 0) B/|B| minimises t |w| + 1/2 |w - B|^2 (the w energy of
    eq 22 per pixel, repulsion frozen, divided by mu)."""
    for _ in range(40):
        B = RNG.normal(size=2) * RNG.uniform(0.1, 3)
        t = RNG.uniform(0, 3)
        fun = lambda w: t * math.hypot(w[0], w[1]) + 0.5 * ((w[0] - B[0]) ** 2 + (w[1] - B[1]) ** 2)
        best = min((optimize.minimize(fun, x0, method="Nelder-Mead",
                                      options={"xatol": 1e-10, "fatol": 1e-14, "maxiter": 4000})
                    for x0 in (B, np.zeros(2) + 1e-9, 0.5 * B)), key=lambda r: r.fun)
        s = O.shrink(np.array([B[0]]), np.array([B[1]]), np.array([t]))
        got = np.array([s[0][0], s[1][0]])
        assert fun(got) <= best.fun + 1e-9
        np.testing.assert_allclose(got, best.x, atol=1e-4)


def test_projection_unit_or_zero():
    w1, w2 = RNG.normal(size=50), RNG.normal(size=50)
    w1[:5] = 0.0
    w2[:5] = 0.0
    p1, p2 = O.project(w1, w2)
    n = np.hypot(p1, p2)
    np.testing.assert_allclose(n[5:], 1.0, atol=1e-15)
    assert np.all(n[:5] == 0.0)
    np.testing.assert_allclose(p1[5:] * w2[5:] - p2[5:] * w1[5:], 0.0, atol=1e-14)   # same direction
    assert np.all(p1[5:] * w1[5:] + p2[5:] * w2[5:] > 0)


# --------------------------------------------------------------------------
# eq (7)-(10): energy
# --------------------------------------------------------------------------
def test_energy_circle_length_and_area():
    """For g = 1 and an SDF circle: E_g ~ perimeter, E_a ~ enclosed area."""
    M = N = 128
    r = 30.0
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    phi = np.sqrt((i - 63.5) ** 2 + (j - 63.5) ** 2) - r
    P = O.Params(gamma=1.0, alpha=1.0, beta=0.0, eps=1.5)
    Eg, Ea, Er = O.energy_terms(phi, np.ones((M, N)), P)
    # forward differences measure the digital perimeter, between 2 pi r and 8 r
    assert 2 * math.pi * r * 0.99 < Eg < 8 * r
    assert Eg == pytest.approx(2 * math.pi * r, rel=0.12)
    assert Ea == pytest.approx(math.pi * r * r, rel=0.01)
    assert Er == 0.0


def test_energy_equals_split_energy_at_consistent_w():
    """E(phi) of eq (7) equals E(phi, w) of eq (22) at w = grad phi, b = 0."""
    M, N = 8, 8
    P = O.Params(gamma=1.1, alpha=0.9, beta=0.7, mu=3.0, eps=1.5, band_l=1.0, d=3.0, R=3)
    phi = RNG.uniform(-3, 3, size=(M, N))
    g = RNG.uniform(0.1, 1, size=(M, N))
    w1, w2 = O.grad_fwd(phi)
    z = np.zeros((M, N))
    K = _kernel_matrix(M, N, P.R, P.d)
    assert O.energy(phi, g, P) == pytest.approx(_split_energy(phi, w1, w2, z, z, g, P, K), rel=1e-12)


# --------------------------------------------------------------------------
# Algorithm 1: whole-iteration symmetries
# --------------------------------------------------------------------------
def _small_problem(M=32, N=40, seed=7):
    r = np.random.default_rng(seed)
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    f = ((i - 15.3) ** 2 / 49 + (j - 12.2) ** 2 / 25 < 1).astype(float)
    f += ((i - 14.1) ** 2 / 36 + (j - 27.9) ** 2 / 36 < 1)
    f += 0.1 * r.normal(size=(M, N))
    phi0 = np.sqrt((i - 15.5) ** 2 + (j - 19.5) ** 2) - 13.0
    return f, phi0


PSMALL = O.Params(gamma=4, alpha=4, beta=0.2, mu=8, tau=0.1, eps=1.5, band_l=1, d=5, R=3, S=3)


def test_translation_equivariance():
    f, phi0 = _small_problem()
    a, b = 5, -7
    st, _, _ = O.solve(f, phi0, PSMALL, 4)
    st2, _, _ = O.solve(np.roll(f, (a, b), (0, 1)), np.roll(phi0, (a, b), (0, 1)), PSMALL, 4)
    for x, y in ((st.phi, st2.phi), (st.w1, st2.w1), (st.w2, st2.w2), (st.b1, st2.b1)):
        np.testing.assert_allclose(np.roll(x, (a, b), (0, 1)), y, atol=1e-10)


def test_transpose_symmetry():
    f, phi0 = _small_problem(M=32, N=32)
    st, _, _ = O.solve(f, phi0, PSMALL, 4)
    st2, _, _ = O.solve(f.T.copy(), phi0.T.copy(), PSMALL, 4)
    np.testing.assert_allclose(st.phi.T, st2.phi, atol=1e-10)
    np.testing.assert_allclose(st.w1.T, st2.w2, atol=1e-10)
    np.testing.assert_allclose(st.w2.T, st2.w1, atol=1e-10)
    np.testing.assert_allclose(st.b1.T, st2.b2, atol=1e-10)


def test_initial_state_and_bregman_increment():
    """Algorithm 1 initialisation (w^0 = grad phi^0, b^0 = 0), and one iteration
    leaves b^1 = grad phi^1 - w^1 (eq 23 from b^0 = 0), w^1 in {0} u unit circle."""
    f, phi0 = _small_problem()
    st0 = O.initial_state(phi0)
    np.testing.assert_array_equal(st0.b1, 0.0)
    g = O.edge_map(f, PSMALL.sigma, PSMALL.rho, PSMALL.s_exp)
    st1, info = O.sb_iteration(st0, g, PSMALL)
    G1 = np.roll(st1.phi, -1, 0) - st1.phi
    np.testing.assert_allclose(st1.b1, G1 - st1.w1, atol=1e-13)
    n = np.hypot(st1.w1, st1.w2)
    assert np.all((n == 0) | (np.abs(n - 1) < 1e-12))
    assert info["inner_steps"] == PSMALL.S


def test_shrink_zero_tolerance_reading():
    """zero_tol = 0 is the paper's literal 0 (0/|0|) = 0: a rounding-level B
    survives (and projects to a unit vector of arbitrary direction); with
    zero_tol > 0 such a B is the zero vector, larger B are unaffected."""
    B1, B2 = np.array([3e-9, 0.6]), np.array([-4e-9, 0.8])
    t = np.zeros(2)
    s = O.shrink(B1, B2, t, 0.0)
    np.testing.assert_array_equal(s[0], B1)
    p = O.project(*s)
    np.testing.assert_allclose(np.hypot(*p), 1.0, atol=1e-15)
    s = O.shrink(B1, B2, t, 1e-3)
    np.testing.assert_array_equal(s[0], [0.0, 0.6])
    np.testing.assert_array_equal(s[1], [0.0, 0.8])
    assert O.Params().zero_tol == 1e-3


# --------------------------------------------------------------------------
# fixed-point iteration for w, eqs (38)-(40)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("sweeps", [1, 2, 3, 5])
def test_w_fixed_point_uniform_field_recurrence(sweeps):
    """On uniform fields (phi = c inside the band, so grad phi = 0, h and
    delta constant; b = b0, w^k = a unit vector at angle th0) every sweep is
    the planar map w <- (mu b0 + kappa w) / |mu b0 + kappa w| with
    kappa = 2 beta h(c)^2 (sum_p a_p)^2: eq (38) gives v = h(c) (sum a)^2 w
    for the full window.  The recurrence is iterated here with angles and
    compared with the oracle."""
    P = O.Params(R=3, d=3.0, beta=0.3, mu=0.5, gamma=1.0, eps=1.5, band_l=1.0, w_solver=1, w_sweeps=sweeps)
    M = N = 16
    c = 0.4
    h0 = float(O.band(np.array(c), P.eps, P.band_l))
    s_a = sum(math.exp(-(p * p) / (P.d * P.d)) for p in range(-P.R, P.R + 1))
    kappa = 2.0 * P.beta * h0 * h0 * s_a * s_a
    b0 = (0.3, -0.7)
    th = 2.1
    phi = np.full((M, N), c)
    g = np.full((M, N), 0.8)
    w1, w2 = np.full((M, N), math.cos(th)), np.full((M, N), math.sin(th))
    b1, b2 = np.full((M, N), b0[0]), np.full((M, N), b0[1])
    got1, got2 = O.w_fixed_point(phi, w1, w2, b1, b2, g, P)
    x, y = math.cos(th), math.sin(th)
    for _ in range(sweeps):
        nx, ny = P.mu * b0[0] + kappa * x, P.mu * b0[1] + kappa * y
        r = math.hypot(nx, ny)
        x, y = nx / r, ny / r
    np.testing.assert_allclose(got1, x, atol=1e-12)
    np.testing.assert_allclose(got2, y, atol=1e-12)


def test_w_fixed_point_one_sweep_is_open_gate_shrink():
    """One sweep divides B of eq (41) (times mu) by a positive factor and
    projects: where the soft-thresholding gate of eq (42) is open (|B| > t)
    it gives the same unit vector as eqs (41)-(42)-(40); where the gate is
    closed it still gives B/|B|, not 0."""
    M, N = 24, 20
    rng = np.random.default_rng(7)
    phi = rng.uniform(-3, 3, (M, N))
    w1, w2 = O.project(rng.normal(size=(M, N)), rng.normal(size=(M, N)))
    b1, b2 = rng.normal(0, 0.5, (M, N)), rng.normal(0, 0.5, (M, N))
    g = rng.uniform(0.1, 1.0, (M, N))
    P = O.Params(R=2, d=2.0, w_solver=1, w_sweeps=1, zero_tol=1e-9)
    f1, f2 = O.w_fixed_point(phi, w1, w2, b1, b2, g, P)
    s1, s2 = O.w_subproblem(phi, w1, w2, b1, b2, g, P)
    B1, B2, t = O.shrink_input(phi, w1, w2, b1, b2, g, P)
    nb = np.hypot(B1, B2)
    open_ = nb > t + 1e-9
    closed = (nb < t - 1e-9) & (nb > 1e-6)
    assert open_.sum() > 50 and closed.sum() > 5
    np.testing.assert_allclose(f1[open_], s1[open_], atol=1e-12)
    np.testing.assert_allclose(f2[open_], s2[open_], atol=1e-12)
    np.testing.assert_allclose(f1[closed], (B1 / nb)[closed], atol=1e-12)
    np.testing.assert_allclose(f2[closed], (B2 / nb)[closed], atol=1e-12)
    assert np.all(s1[closed] == 0.0) and np.all(s2[closed] == 0.0)


def test_w_fixed_point_converges_to_a_fixed_point():
    """With a weak repulsion the sweeps contract: after many of them w solves
    its own fixed-point equation, w = project(numerator of eq 39 built from
    w), to rounding, and the result does not depend on the starting w."""
    M, N = 20, 18
    rng = np.random.default_rng(3)
    phi = rng.uniform(-2, 2, (M, N))
    g = rng.uniform(0.2, 1.0, (M, N))
    b1, b2 = rng.normal(0, 1.0, (M, N)) + 1.5, rng.normal(0, 1.0, (M, N))
    P = O.Params(R=2, d=2.0, beta=0.002, mu=1.0, w_solver=1, w_sweeps=60, zero_tol=0.0)
    wa = O.w_fixed_point(phi, *O.project(rng.normal(size=(M, N)), rng.normal(size=(M, N))), b1, b2, g, P)
    wb = O.w_fixed_point(phi, *O.project(rng.normal(size=(M, N)), rng.normal(size=(M, N))), b1, b2, g, P)
    np.testing.assert_allclose(wa[0], wb[0], atol=1e-10)
    np.testing.assert_allclose(wa[1], wb[1], atol=1e-10)
    G1, G2 = O.grad_fwd(phi)
    v1, v2 = O.repulsion_field(wa[0], wa[1], phi, P.eps, P.band_l, P.d, P.R)
    h = O.band(phi, P.eps, P.band_l)
    n1 = P.mu * (G1 + b1) + 2 * P.beta * h * v1
    n2 = P.mu * (G2 + b2) + 2 * P.beta * h * v2
    r1, r2 = O.project(n1, n2)
    np.testing.assert_allclose(wa[0], r1, atol=1e-10)
    np.testing.assert_allclose(wa[1], r2, atol=1e-10)


def test_w_fixed_point_iteration_translation_equivariant():
    """A whole outer iteration with the fixed-point w solver commutes with
    periodic shifts of its inputs."""
    M, N = 32, 24
    rng = np.random.default_rng(11)
    f = rng.uniform(0, 1, (M, N))
    phi0 = np.add.outer(np.arange(M) - 15.5, np.zeros(N)) ** 2 / 20.0 - 4.0 + rng.normal(0, 0.1, (M, N))
    P = O.Params(R=3, d=3.0, w_solver=1, w_sweeps=3)
    a, ga, _ = O.solve(f, phi0, P, 2)
    sh = (5, -7)
    b, gb, _ = O.solve(np.roll(f, sh, (0, 1)), np.roll(phi0, sh, (0, 1)), P, 2)
    np.testing.assert_allclose(b.phi, np.roll(a.phi, sh, (0, 1)), atol=1e-10)
    np.testing.assert_allclose(b.w1, np.roll(a.w1, sh, (0, 1)), atol=1e-10)


# --------------------------------------------------------------------------
# AOS solve of the phi sub-problem with constant A_l (end of Sec. 4)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [3, 4, 7, 16, 33])
def test_thomas_cyclic_against_dense_solve(n):
    """The cyclic Thomas solve against a dense solve of the full periodic
    tridiagonal matrix, built here entry by entry."""
    rng = np.random.default_rng(n)
    off, diag = -0.37, 1.0 + 4 * 0.37 + 0.05
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] += diag
        A[i, (i - 1) % n] += off
        A[i, (i + 1) % n] += off
    F = rng.normal(size=(n, 5))
    np.testing.assert_allclose(O.thomas_cyclic(off, diag, F), np.linalg.solve(A, F), atol=1e-12)


@pytest.mark.parametrize("tau,mu,a,b", [(0.1, 8.0, 3, 5), (0.4, 0.1, 1, 0), (0.1, 8.0, 0, 7)])
def test_aos_solve_separable_mode(tau, mu, a, b):
    """A separable Fourier mode is an eigenvector of both 1-D operators:
    v_l = F / (1 + 2 tau mu (2 - 2 cos(2 pi k_l / n_l))), phi = (v_1 + v_2) / 2."""
    M, N = 24, 16
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    F = np.cos(2 * np.pi * a * i / M + 0.3) * np.cos(2 * np.pi * b * j / N - 0.7)
    s1 = 1 + 2 * tau * mu * (2 - 2 * math.cos(2 * math.pi * a / M))
    s2 = 1 + 2 * tau * mu * (2 - 2 * math.cos(2 * math.pi * b / N))
    np.testing.assert_allclose(O.aos_solve(F, tau, mu), 0.5 * (F / s1 + F / s2), atol=1e-12)


def test_aos_solve_keeps_constants_and_is_first_order_close_to_fft():
    """Constants pass unchanged (each 1-D operator has unit row sums); on a
    smooth field the AOS solve differs from the exact FFT solve of
    (1 - tau mu Delta) by O((tau mu)^2) times the mixed fourth differences."""
    M, N = 32, 32
    np.testing.assert_allclose(O.aos_solve(np.full((M, N), 3.25), 0.1, 8.0), 3.25, atol=1e-13)
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    F = np.sin(2 * np.pi * i / M) + np.cos(2 * np.pi * 2 * j / N) + 0.5 * np.sin(2 * np.pi * (i + j) / M)
    for tm, bound in ((0.001, 1e-5), (0.01, 1e-3)):
        d = np.abs(O.aos_solve(F, tm, 1.0) - O.implicit_solve(F, tm, 1.0)).max()
        assert d < bound, (tm, d)


def test_aos_iteration_translation_equivariant():
    """A whole outer iteration with the AOS phi solver commutes with periodic
    shifts of its inputs."""
    M, N = 32, 24
    rng = np.random.default_rng(21)
    f = rng.uniform(0, 1, (M, N))
    phi0 = np.add.outer(np.arange(M) - 15.5, np.zeros(N)) ** 2 / 20.0 - 4.0 + rng.normal(0, 0.1, (M, N))
    P = O.Params(R=3, d=3.0, phi_solver=1)
    a, _, _ = O.solve(f, phi0, P, 2)
    sh = (-9, 4)
    b, _, _ = O.solve(np.roll(f, sh, (0, 1)), np.roll(phi0, sh, (0, 1)), P, 2)
    np.testing.assert_allclose(b.phi, np.roll(a.phi, sh, (0, 1)), atol=1e-10)


# --------------------------------------------------------------------------
# Neumann boundaries (eq 17's and eq 27's zero normal derivative; bc = 1):
# mirror ghosts, the adjoint divergence, the DCT-II solve, the plain
# tridiagonal AOS solve
# --------------------------------------------------------------------------
def _mirror(i, n):
    """Half-sample mirror of an index, written out case by case."""
    if i < 0:
        return -1 - i
    if i >= n:
        return 2 * n - 1 - i
    return i


def _neumann_second_difference(n):
    """Dense 1-D second difference with the Neumann end rows (u_1 - u_0 and
    u_{n-2} - u_{n-1}), entry by entry."""
    D = np.zeros((n, n))
    for i in range(n):
        for k in (i - 1, i + 1):
            D[i, _mirror(k, n)] += 1.0
        D[i, i] -= 2.0
    return D


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_mirror_index_matches_numpy_symmetric_pad(n):
    """at(.., bc=1) is NumPy's 'symmetric' padding (the edge sample repeated)."""
    u = RNG.normal(size=(n, 3))
    pad = np.pad(u, ((n, n), (0, 0)), mode="symmetric")
    for k in range(-n, n + 1):
        np.testing.assert_array_equal(O.at(u, k, 0, 1), pad[n + k:n + k + n])


def test_neumann_gradient_divergence_laplacian():
    """Forward differences vanish on the last row / column; the divergence is
    the negative adjoint of the gradient; div grad is the Laplacian, equal to
    the Kronecker sum of dense Neumann second differences; its sum vanishes."""
    M, N = 7, 10
    u = RNG.normal(size=(M, N))
    g1, g2 = O.grad_fwd(u, 1)
    assert np.all(g1[-1] == 0.0) and np.all(g2[:, -1] == 0.0)
    np.testing.assert_array_equal(g1[:-1], u[1:] - u[:-1])
    np.testing.assert_array_equal(g2[:, :-1], u[:, 1:] - u[:, :-1])
    p, q = RNG.normal(size=(M, N)), RNG.normal(size=(M, N))
    assert np.sum(g1 * p + g2 * q) == pytest.approx(-np.sum(u * O.div_bwd(p, q, 1)), rel=1e-13)
    lap = O.laplacian(u, 1)
    np.testing.assert_allclose(lap, O.div_bwd(*O.grad_fwd(u, 1), 1), atol=1e-13)
    L = np.kron(_neumann_second_difference(M), np.eye(N)) + np.kron(np.eye(M), _neumann_second_difference(N))
    np.testing.assert_allclose(lap.ravel(), L @ u.ravel(), atol=1e-13)
    assert abs(lap.sum()) < 1e-12


@pytest.mark.parametrize("sigma", [0.5, 1.5, 2.0])
def test_neumann_gaussian_and_edge_map_match_scipy_reflect(sigma):
    """SciPy's 'reflect' mode is the half-sample mirror."""
    f = RNG.uniform(size=(20, 33))
    ref = ndimage.gaussian_filter1d(f, sigma, axis=1, mode="reflect", truncate=3.0)
    ref = ndimage.gaussian_filter1d(ref, sigma, axis=0, mode="reflect", truncate=3.0)
    np.testing.assert_allclose(O.gaussian_smooth(f, sigma, 1), ref, atol=1e-13)
    fs = ndimage.gaussian_filter(f, 1.5, mode="reflect", truncate=3.0)
    gx = ndimage.correlate1d(fs, [-0.5, 0.0, 0.5], axis=0, mode="reflect")
    gy = ndimage.correlate1d(fs, [-0.5, 0.0, 0.5], axis=1, mode="reflect")
    np.testing.assert_allclose(O.edge_map(f, 1.5, 1000.0, 2, 1), 1.0 / (1.0 + 1000.0 * np.hypot(gx, gy) ** 2),
                               rtol=1e-12)


@pytest.mark.parametrize("shape,R,d", [((7, 9), 2, 2.0), ((12, 11), 5, 5.0), ((6, 6), 5, 3.0)])
def test_neumann_repulsion_brute_force(shape, R, d):
    M, N = shape
    phi = RNG.uniform(-4, 4, size=shape)
    w1, w2 = RNG.normal(size=shape), RNG.normal(size=shape)
    hh = O.band(phi, 1.5, 1.0)
    v1 = np.zeros(shape)
    v2 = np.zeros(shape)
    for i in range(M):
        for j in range(N):
            for p in range(-R, R + 1):
                for q in range(-R, R + 1):
                    k = math.exp(-(p * p + q * q) / (d * d))
                    ii, jj = _mirror(i + p, M), _mirror(j + q, N)
                    v1[i, j] += k * w1[ii, jj] * hh[ii, jj]
                    v2[i, j] += k * w2[ii, jj] * hh[ii, jj]
    got = O.repulsion_field(w1, w2, phi, 1.5, 1.0, d, R, 1)
    np.testing.assert_allclose(got[0], v1, atol=1e-12)
    np.testing.assert_allclose(got[1], v2, atol=1e-12)


@pytest.mark.parametrize("shape,tau,mu", [((16, 16), 0.1, 8.0), ((8, 32), 0.4, 0.1), ((9, 14), 1.0, 3.0)])
def test_dct_solve_residual_and_mirror_extension(shape, tau, mu):
    """The DCT solve satisfies (1 - tau mu Lap_N) phi = F, and equals the
    periodic FFT solve on the 2M x 2N mirror extension of F, restricted."""
    M, N = shape
    F = RNG.normal(size=shape) * 20.0
    phi = O.implicit_solve(F, tau, mu, 1)
    np.testing.assert_allclose(phi - tau * mu * O.laplacian(phi, 1), F, atol=1e-11)
    ext = np.concatenate([F, F[::-1]], axis=0)
    ext = np.concatenate([ext, ext[:, ::-1]], axis=1)
    sym = 1.0 - tau * mu * (2 * np.cos(2 * np.pi * np.arange(2 * M) / (2 * M))[:, None]
                            + 2 * np.cos(2 * np.pi * np.arange(2 * N) / (2 * N))[None, :] - 4)
    per = np.real(np.fft.ifft2(np.fft.fft2(ext) / sym))[:M, :N]
    np.testing.assert_allclose(phi, per, atol=1e-11)


def test_dct_solve_cosine_mode():
    M, N, a, b, tau, mu = 12, 20, 3, 7, 0.1, 8.0
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    F = np.cos(np.pi * a * (i + 0.5) / M) * np.cos(np.pi * b * (j + 0.5) / N)
    s = 1 + tau * mu * (4 - 2 * math.cos(math.pi * a / M) - 2 * math.cos(math.pi * b / N))
    np.testing.assert_allclose(O.implicit_solve(F, tau, mu, 1), F / s, atol=1e-13)


@pytest.mark.parametrize("shape", [(5, 8), (16, 9)])
def test_aos_neumann_against_dense_solves(shape):
    """(1 - 2 tau mu D_l) v_l = F with the dense Neumann D_l in each
    direction, phi = (v_1 + v_2) / 2; constants pass unchanged."""
    M, N = shape
    tau, mu = 0.1, 8.0
    F = RNG.normal(size=shape)
    v1 = np.linalg.solve(np.eye(M) - 2 * tau * mu * _neumann_second_difference(M), F)
    v2 = np.linalg.solve(np.eye(N) - 2 * tau * mu * _neumann_second_difference(N), F.T).T
    np.testing.assert_allclose(O.aos_solve(F, tau, mu, 1), 0.5 * (v1 + v2), atol=1e-12)
    np.testing.assert_allclose(O.aos_solve(np.full(shape, -1.75), tau, mu, 1), -1.75, atol=1e-13)


def _kernel_matrix_neumann(M, N, R, d):
    """Dense window operator with mirrored indices (symmetric: a mirrored
    pair of points sees each other with the same total weight)."""
    K = np.zeros((M * N, M * N))
    for i in range(M):
        for j in range(N):
            for p in range(-R, R + 1):
                for q in range(-R, R + 1):
                    K[i * N + j, _mirror(i + p, M) * N + _mirror(j + q, N)] += math.exp(-(p * p + q * q) / (d * d))
    return K


def _split_energy_neumann(phi, w1, w2, b1, b2, g, P, K):
    """E(phi, w) of eq (22) with Neumann forward differences (zero on the
    last row / column), written directly."""
    wn = np.sqrt(w1 ** 2 + w2 ** 2)
    Eg = np.sum(g * wn * O.dirac(phi, P.eps))
    Ea = np.sum(g * (1 - O.heaviside(phi, P.eps)))
    hv = O.band(phi, P.eps, P.band_l).ravel()
    W1, W2 = w1.ravel(), w2.ravel()
    Er = -(np.einsum("x,y,xy->", W1 * hv, W1 * hv, K) + np.einsum("x,y,xy->", W2 * hv, W2 * hv, K))
    d1 = np.zeros_like(phi)
    d2 = np.zeros_like(phi)
    d1[:-1] = phi[1:] - phi[:-1]
    d2[:, :-1] = phi[:, 1:] - phi[:, :-1]
    Es = 0.5 * P.mu * np.sum((w1 - d1 - b1) ** 2 + (w2 - d2 - b2) ** 2)
    return P.gamma * Eg + P.alpha * Ea + P.beta * Er + Es


def test_neumann_rhs_is_negative_gradient_of_split_energy():
    """With Neumann boundaries (F - phi)/tau + mu Lap_N(phi) is -dE/dphi of
    eq (22): pins the mirrored window, the adjoint divergence and the
    boundary rows of the gradient."""
    M, N = 7, 8
    P = O.Params(gamma=1.3, alpha=0.7, beta=0.45, mu=2.0, tau=0.3, eps=1.5, band_l=1.0, d=3.0, R=3, bc=1)
    phi = RNG.uniform(-2.8, 2.8, size=(M, N))
    w1, w2 = RNG.normal(size=(M, N)), RNG.normal(size=(M, N))
    b1, b2 = 0.3 * RNG.normal(size=(M, N)), 0.3 * RNG.normal(size=(M, N))
    g = RNG.uniform(0.05, 1.0, size=(M, N))
    K = _kernel_matrix_neumann(M, N, P.R, P.d)
    assert np.allclose(K, K.T)
    F = O.phi_rhs(phi, w1, w2, b1, b2, g, P)
    flow = (F - phi) / P.tau + P.mu * O.laplacian(phi, 1)
    h = 1e-6
    grad = np.zeros((M, N))
    for i in range(M):
        for j in range(N):
            pp = phi.copy(); pp[i, j] += h
            pm = phi.copy(); pm[i, j] -= h
            grad[i, j] = (_split_energy_neumann(pp, w1, w2, b1, b2, g, P, K)
                          - _split_energy_neumann(pm, w1, w2, b1, b2, g, P, K)) / (2 * h)
    np.testing.assert_allclose(flow, -grad, atol=2e-6 * np.abs(grad).max())


def test_neumann_energy_equals_split_energy_at_consistent_w():
    M, N = 8, 7
    P = O.Params(gamma=1.1, alpha=0.9, beta=0.7, mu=3.0, eps=1.5, band_l=1.0, d=3.0, R=3, bc=1)
    phi = RNG.uniform(-3, 3, size=(M, N))
    g = RNG.uniform(0.1, 1, size=(M, N))
    w1, w2 = O.grad_fwd(phi, 1)
    z = np.zeros((M, N))
    K = _kernel_matrix_neumann(M, N, P.R, P.d)
    assert O.energy(phi, g, P) == pytest.approx(_split_energy_neumann(phi, w1, w2, z, z, g, P, K), rel=1e-12)


@pytest.mark.parametrize("phi_solver", [0, 1])
def test_neumann_transpose_symmetry(phi_solver):
    f, phi0 = _small_problem(M=32, N=32)
    P = O.Params(**{**PSMALL.__dict__, "bc": 1, "phi_solver": phi_solver,
                    "tau": 0.04 if phi_solver else PSMALL.tau})
    st, _, _ = O.solve(f, phi0, P, 4)
    st2, _, _ = O.solve(f.T.copy(), phi0.T.copy(), P, 4)
    np.testing.assert_allclose(st.phi.T, st2.phi, atol=1e-10)
    np.testing.assert_allclose(st.w1.T, st2.w2, atol=1e-10)
    np.testing.assert_allclose(st.b2.T, st2.b1, atol=1e-10)

