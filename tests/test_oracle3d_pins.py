"""Pins of the 3-D oracle against facts that do not come from it: the
independently pinned 2-D oracle on volumes that are constant along the third
axis, SciPy's Gaussian filter, brute-force window sums, the residual of the
linear system the FFT solve claims to solve, finite differences of the 3-D
split energy, and the symmetry of the iteration under axis permutations."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import sr_oracle as O
from oracle import sr_oracle3d as O3

RNG = np.random.default_rng(3303)
P3 = O.Params(gamma=4, alpha=4, beta=0.2, mu=3, tau=0.05, eps=1.5, band_l=1, d=4, R=2, S=3)


def _a(R, d):
    return sum(math.exp(-p * p / (d * d)) for p in range(-R, R + 1))


def _planar_problem(M=24, N=20):
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    f = ((i - 11.3) ** 2 / 36 + (j - 9.2) ** 2 / 16 < 1).astype(float) + 0.1 * RNG.normal(size=(M, N))
    phi0 = np.sqrt((i - 11.5) ** 2 + (j - 9.5) ** 2) - 8.0
    return f, phi0


def test_constant_along_third_axis_reduces_to_2d():
    """A volume constant along k is a stack of the 2-D problem: one 3-D
    iteration equals one 2-D iteration whose beta is scaled by the window's
    third-axis factor sum_r exp(-r^2/d^2); the third components stay zero."""
    f, phi0 = _planar_problem()
    Pz = 5
    f3 = np.repeat(f[:, :, None], Pz, axis=2)
    p3 = np.repeat(phi0[:, :, None], Pz, axis=2)
    st3, g3 = O3.solve(f3, p3, P3, 2)
    P2 = O.Params(**{**P3.__dict__, "beta": P3.beta * _a(P3.R, P3.d)})
    st2, g2, _ = O.solve(f, phi0, P2, 2)
    for k in range(Pz):
        np.testing.assert_allclose(g3[:, :, k], g2, atol=1e-12)
        np.testing.assert_allclose(st3.phi[:, :, k], st2.phi, atol=1e-9)
        np.testing.assert_allclose(st3.w[0][:, :, k], st2.w1, atol=1e-9)
        np.testing.assert_allclose(st3.w[1][:, :, k], st2.w2, atol=1e-9)
        np.testing.assert_allclose(st3.b[1][:, :, k], st2.b2, atol=1e-9)
    assert np.abs(st3.w[2]).max() < 1e-9 and np.abs(st3.b[2]).max() < 1e-9
    E3 = O3.energy_terms(p3, g3, P3)
    E2 = O.energy_terms(phi0, g2, P2)
    for a, b in zip(E3, E2):
        assert a == pytest.approx(Pz * b, rel=1e-11)


def test_operators_adjoint_laplacian_mode():
    u = RNG.normal(size=(5, 6, 7))
    p = [RNG.normal(size=u.shape) for _ in range(3)]
    G = O3.grad_fwd(u)
    assert sum(np.sum(G[a] * p[a]) for a in range(3)) == pytest.approx(-np.sum(u * O3.div_bwd(p)), rel=1e-13)
    np.testing.assert_allclose(O3.laplacian(u), O3.div_bwd(G), atol=1e-13)
    M, N, K = 8, 12, 10
    i, j, k = np.meshgrid(np.arange(M), np.arange(N), np.arange(K), indexing="ij")
    mode = np.cos(2 * np.pi * (2 * i / M + 3 * j / N + 1 * k / K))
    lam = sum(2 * math.cos(2 * math.pi * c / n) - 2 for c, n in ((2, M), (3, N), (1, K)))
    np.testing.assert_allclose(O3.laplacian(mode), lam * mode, atol=1e-12)


@pytest.mark.parametrize("sigma", [0.5, 1.5])
def test_gaussian_matches_scipy(sigma):
    f = RNG.normal(size=(10, 12, 14))
    ref = ndimage.gaussian_filter(f, sigma, mode="wrap", truncate=3.0)
    np.testing.assert_allclose(O3.gaussian_smooth(f, sigma), ref, atol=1e-13)


@pytest.mark.parametrize("R,d", [(1, 2.0), (2, 4.0)])
def test_repulsion_brute_force(R, d):
    M, N, K = 4, 5, 6
    phi = RNG.uniform(-3, 3, size=(M, N, K))
    w = [RNG.normal(size=(M, N, K)) for _ in range(3)]
    h = O.band(phi, 1.5, 1.0)
    ref = [np.zeros((M, N, K)) for _ in range(3)]
    for i in range(M):
        for j in range(N):
            for k in range(K):
                for p in range(-R, R + 1):
                    for q in range(-R, R + 1):
                        for r in range(-R, R + 1):
                            wt = math.exp(-(p * p + q * q + r * r) / (d * d))
                            ii, jj, kk = (i + p) % M, (j + q) % N, (k + r) % K
                            for c in range(3):
                                ref[c][i, j, k] += wt * w[c][ii, jj, kk] * h[ii, jj, kk]
    got = O3.repulsion_field(w, phi, 1.5, 1.0, d, R)
    for c in range(3):
        np.testing.assert_allclose(got[c], ref[c], atol=1e-12)


def test_fft_solve_residual():
    F = RNG.normal(size=(8, 16, 12)) * 10
    for tau, mu in ((0.05, 3.0), (0.4, 0.1)):
        phi = O3.implicit_solve(F, tau, mu)
        np.testing.assert_allclose(phi - tau * mu * O3.laplacian(phi), F, atol=1e-11)


def _dense_kernel(shape, R, d):
    M, N, K = shape
    n = M * N * K
    A = np.zeros((n, n))
    idx = lambda i, j, k: (i % M) * N * K + (j % N) * K + (k % K)
    for i in range(M):
        for j in range(N):
            for k in range(K):
                for p in range(-R, R + 1):
                    for q in range(-R, R + 1):
                        for r in range(-R, R + 1):
                            A[idx(i, j, k), idx(i + p, j + q, k + r)] += math.exp(-(p * p + q * q + r * r) / (d * d))
    return A


def test_rhs_is_negative_gradient_of_split_energy():
    """(F - phi)/tau + mu Lap phi = -dE/dphi of the 3-D split energy (eq 22
    with 3-component w, b, the cube window as a dense matrix)."""
    shape = (4, 4, 5)
    P = O.Params(gamma=1.3, alpha=0.7, beta=0.45, mu=2.0, tau=0.3, eps=1.5, band_l=1.0, d=3.0, R=1)
    phi = RNG.uniform(-2.8, 2.8, size=shape)
    w = tuple(RNG.normal(size=shape) for _ in range(3))
    b = tuple(0.3 * RNG.normal(size=shape) for _ in range(3))
    g = RNG.uniform(0.05, 1.0, size=shape)
    A = _dense_kernel(shape, P.R, P.d)

    def energy(ph):
        wn = np.sqrt(sum(c ** 2 for c in w))
        Eg = np.sum(g * wn * O.dirac(ph, P.eps))
        Ea = np.sum(g * (1 - O.heaviside(ph, P.eps)))
        hv = O.band(ph, P.eps, P.band_l).ravel()
        Er = -sum(np.einsum("x,y,xy->", c.ravel() * hv, c.ravel() * hv, A) for c in w)
        d = [np.roll(ph, -1, a) - ph for a in range(3)]
        Es = 0.5 * P.mu * sum(np.sum((w[a] - d[a] - b[a]) ** 2) for a in range(3))
        return P.gamma * Eg + P.alpha * Ea + P.beta * Er + Es

    F = O3.phi_rhs(phi, w, b, g, P)
    flow = (F - phi) / P.tau + P.mu * O3.laplacian(phi)
    hstep = 1e-6
    grad = np.zeros(shape)
    for ix in np.ndindex(shape):
        pp = phi.copy(); pp[ix] += hstep
        pm = phi.copy(); pm[ix] -= hstep
        grad[ix] = (energy(pp) - energy(pm)) / (2 * hstep)
    np.testing.assert_allclose(flow, -grad, atol=2e-6 * np.abs(grad).max())


def test_axis_permutation_symmetry():
    """Permuting the volume's axes permutes the components of w and b."""
    M, N, K = 12, 10, 8
    i, j, k = np.meshgrid(np.arange(M), np.arange(N), np.arange(K), indexing="ij")
    phi0 = np.sqrt((i - 5.7) ** 2 + (j - 4.6) ** 2 + (k - 3.4) ** 2) - 3.0
    f = (phi0 < -0.5).astype(float) + 0.05 * RNG.normal(size=(M, N, K))
    st, _ = O3.solve(f, phi0, P3, 2)
    perm = (1, 2, 0)
    st2, _ = O3.solve(f.transpose(perm), phi0.transpose(perm), P3, 2)
    np.testing.assert_allclose(st2.phi, st.phi.transpose(perm), atol=1e-10)
    for a in range(3):
        np.testing.assert_allclose(st2.w[a], st.w[perm[a]].transpose(perm), atol=1e-10)
        np.testing.assert_allclose(st2.b[a], st.b[perm[a]].transpose(perm), atol=1e-10)
