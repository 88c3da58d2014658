"""FP64 CPU oracle for the 3-D extension of the Split Bregman solver of the
Self-repelling Snake model (the paper's 3-D application, Sec. 5, Fig. 6).

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import this module:
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use it.  It shares no code, tables or helpers with the HIP library.

The paper applies the method to volumes without writing the 3-D equations
out; they are the 2-D ones with a third axis (reading): phi, f, g are
M x N x P volumes (axis 0 = i, 1 = j, 2 = k), w and b have three components,
grad is the forward difference along each axis, div the backward one, Lap
the seven-point Laplacian, the Gaussian of eq (1) and the repulsion window
are cubes ((2R+1)^3 taps, weights exp(-(p^2+q^2+r^2)/d^2)), and the FFT
symbol of eq (32) gains the third frequency.  Boundaries are periodic.  The
scalar functions (H_eps, delta_eps, h_eps and their derivatives, eqs 5, 6,
11, 28, 29), the shrink and projection (eqs 40, 42 applied to 3-vectors) and
the stop rules are the 2-D oracle's.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from oracle import sr_oracle as O

Params = O.Params
heaviside, dirac, dirac_prime, band, band_prime = O.heaviside, O.dirac, O.dirac_prime, O.band, O.band_prime


def grad_fwd(u):
    """Forward differences along the three axes (eq 35 with a third axis)."""
    return tuple(np.roll(u, -1, axis=a) - u for a in range(3))


def div_bwd(p):
    """Backward-difference divergence of a 3-component field (eq 36)."""
    return sum(p[a] - np.roll(p[a], 1, axis=a) for a in range(3))


def laplacian(u):
    """Seven-point Laplacian."""
    return sum(np.roll(u, 1, axis=a) + np.roll(u, -1, axis=a) for a in range(3)) - 6.0 * u


def gaussian_smooth(f, sigma):
    """G_sigma * f: the 2-D oracle's sampled, truncated, normalised taps
    along each of the three axes in turn, periodic."""
    offs, k = O.gaussian_taps(sigma)
    out = np.asarray(f, dtype=np.float64)
    for a in (2, 1, 0):
        acc = np.zeros_like(out)
        for t, kt in zip(offs, k):
            acc += kt * np.roll(out, -t, axis=a)
        out = acc
    return out


def edge_map(f, sigma, rho, s_exp):
    """g = 1 / (1 + rho |grad(G_sigma * f)|^s), eq (1), central differences."""
    fs = gaussian_smooth(f, sigma)
    m2 = sum((0.5 * (np.roll(fs, -1, axis=a) - np.roll(fs, 1, axis=a))) ** 2 for a in range(3))
    return 1.0 / (1.0 + rho * np.sqrt(m2) ** s_exp)


def repulsion_field(w, phi, eps, l, d, R):
    """v = sum over the (2R+1)^3 cube of exp(-(p^2+q^2+r^2)/d^2) w h_eps(phi)
    at the shifted voxel, periodic, centre included.  Direct sum."""
    h = band(phi, eps, l)
    u = [wc * h for wc in w]
    v = [np.zeros_like(h) for _ in range(3)]
    for p in range(-R, R + 1):
        for q in range(-R, R + 1):
            for r in range(-R, R + 1):
                k = np.exp(-(p * p + q * q + r * r) / (d * d))
                for c in range(3):
                    v[c] += k * np.roll(u[c], (-p, -q, -r), axis=(0, 1, 2))
    return tuple(v)


def symbol(shape, tau, mu):
    """Fourier symbol of (1 - tau mu Lap) on the periodic M x N x P grid."""
    z = [2.0 * np.pi * np.arange(n, dtype=np.float64) / n for n in shape]
    return (1.0 - tau * mu * (2.0 * np.cos(z[0])[:, None, None] + 2.0 * np.cos(z[1])[None, :, None]
                              + 2.0 * np.cos(z[2])[None, None, :] - 6.0))


def implicit_solve(F, tau, mu):
    """(1 - tau mu Lap) phi = F by the 3-D FFT (eq 33 with a third axis)."""
    return np.real(np.fft.ifftn(np.fft.fftn(F) / symbol(F.shape, tau, mu)))


def phi_rhs(phi_s, w, b, g, P: Params):
    """F of eq (37) with 3-component w, b:
    phi_s + tau (-gamma g |w| delta' + alpha g delta + 2 beta h' w . v + mu div(b - w))."""
    v = repulsion_field(w, phi_s, P.eps, P.band_l, P.d, P.R)
    wnorm = np.sqrt(sum(c * c for c in w))
    force = (-P.gamma * g * wnorm * dirac_prime(phi_s, P.eps)
             + P.alpha * g * dirac(phi_s, P.eps)
             + 2.0 * P.beta * band_prime(phi_s, P.eps, P.band_l) * sum(w[c] * v[c] for c in range(3))
             + P.mu * div_bwd([b[c] - w[c] for c in range(3)]))
    return phi_s + P.tau * force


def shrink(B, t, zero_tol=0.0):
    """Eq (42) on 3-vectors: max(|B| - t, 0) B / |B|, zero where |B| <= zero_tol."""
    nb = np.sqrt(sum(c * c for c in B))
    live = nb > zero_tol
    scale = np.where(live, np.maximum(nb - t, 0.0) / np.where(nb > 0, nb, 1.0), 0.0)
    return tuple(scale * c for c in B)


def project(w):
    """Eq (40): w / |w|, zero stays zero."""
    n = np.sqrt(sum(c * c for c in w))
    safe = np.where(n > 0, n, 1.0)
    return tuple(np.where(n > 0, c / safe, 0.0) for c in w)


def w_subproblem(phi_new, w, b, g, P: Params):
    """B of eq (41) with v from w^k and h(phi^{k+1}), shrink (eq 42), project (eq 40)."""
    G = grad_fwd(phi_new)
    v = repulsion_field(w, phi_new, P.eps, P.band_l, P.d, P.R)
    h = band(phi_new, P.eps, P.band_l)
    c = 2.0 * P.beta / P.mu
    B = tuple(G[a] + b[a] + c * h * v[a] for a in range(3))
    t = (P.gamma / P.mu) * g * dirac(phi_new, P.eps)
    return project(shrink(B, t, P.zero_tol))


@dataclasses.dataclass
class State:
    phi: np.ndarray
    w: tuple
    b: tuple
    k: int = 0


def initial_state(phi0):
    """phi^0, w^0 = grad phi^0, b^0 = 0."""
    phi0 = np.asarray(phi0, dtype=np.float64)
    z = np.zeros_like(phi0)
    return State(phi0.copy(), grad_fwd(phi0), (z.copy(), z.copy(), z.copy()), 0)


def sb_iteration(st: State, g, P: Params):
    """One outer iteration of Algorithm 1 in 3-D: S semi-implicit steps of
    eq (37) (fixed S), w by eqs (41), (42), (40), b by eq (23)."""
    phi_s = st.phi
    for _ in range(P.S):
        phi_s = implicit_solve(phi_rhs(phi_s, st.w, st.b, g, P), P.tau, P.mu)
    w_new = w_subproblem(phi_s, st.w, st.b, g, P)
    G = grad_fwd(phi_s)
    b_new = tuple(st.b[a] + G[a] - w_new[a] for a in range(3))
    r = np.linalg.norm(phi_s - st.phi) / (np.linalg.norm(st.phi) + 1e-6)
    return State(phi_s, w_new, b_new, st.k + 1), {"r": r}


def solve(f, phi0, P: Params, iters):
    g = edge_map(f, P.sigma, P.rho, P.s_exp)
    st = initial_state(phi0)
    for _ in range(iters):
        st, _ = sb_iteration(st, g, P)
    return st, g


def energy_terms(phi, g, P: Params):
    """(gamma E_g, alpha E_a, beta E_r) of eqs (7)-(10) on the voxel grid,
    the repulsion integral truncated to the cube window."""
    G = grad_fwd(phi)
    Eg = np.sum(g * np.sqrt(sum(c * c for c in G)) * dirac(phi, P.eps))
    Ea = np.sum(g * (1.0 - heaviside(phi, P.eps)))
    h = band(phi, P.eps, P.band_l)
    v = repulsion_field(G, phi, P.eps, P.band_l, P.d, P.R)
    Er = -np.sum(sum(G[c] * h * v[c] for c in range(3)))
    return P.gamma * Eg, P.alpha * Ea, P.beta * Er
