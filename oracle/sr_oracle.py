"""FP64 CPU oracle for the Split Bregman solver of the Self-repelling Snake model.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import this module:
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use it.  It shares no code, tables or helpers with the HIP library.

It is a plain, slow, literal transcription of the method of Pan et al.,
"Using the Split Bregman Algorithm to Solve the Self-repelling Snake Model"
(arXiv:2003.12693), in float64 with NumPy:

  * edge-stopping function g ............................ eq (1)
  * compactly supported H_eps, delta_eps ................. eqs (5), (6)
  * narrow band h_eps and h'_eps, delta'_eps ............. eqs (11), (28), (29)
  * SR energy E = gamma E_g + alpha E_a + beta E_r ....... eqs (7)-(10)
  * discrete forward gradient, 5-point Laplacian,
    backward divergence (unit spacing) ................... eqs (35), (36)
  * repulsion window sum v (square window, Gaussian taps)  Sec. 4, after eq (37)
  * semi-implicit FFT solve of the phi sub-problem ....... eqs (30)-(33), (37)
  * or, with Neumann boundaries (eq 17's boundary condition,
    eq 27's), its DCT-II solve .......................... eqs (17), (27), (32)
  * or its AOS solve with constant A_l (Thomas algorithm)  eqs (18), (20), end of Sec. 4
  * generalised soft thresholding of w ................... eqs (41), (42)
  * the alternative fixed-point iteration for w .......... eqs (38), (39)
  * projection onto |w| = 1 .............................. eq (40)
  * Bregman update ....................................... eq (23)
  * outer/inner loop ..................................... Algorithm 1, Sec. 4

Readings of passages the paper leaves open (periodic boundaries by default,
Neumann ones as the alternative with mirror stencils and window, the
Frobenius norm in the stop rule, phi^{k+1,s} inside F^{k,s}, the window
bounds, w^0 = grad phi^0, shrink -> project -> Bregman order, the discrete
energy) are listed in the design notes of the repository; each function
below names the reading it takes.

Every function is pinned by a test in tests/test_oracle_*.py against
something other than itself (closed forms, finite-difference gradients of
the split energy, a brute-force window sum in pure Python, the linear-system
residual, SciPy's Gaussian filter, numerical minimisation of the pointwise w
energy, translation / transpose symmetry, topology preservation).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Params:
    """Model and solver parameters, named as in the paper.

    gamma, alpha, beta : weights of E_g, E_a, E_r (eq 7)
    mu                 : splitting penalty (eq 22), also the implicit
                         Laplacian weight of eq (30)
    tau                : time step of the semi-implicit scheme (eq 30)
    eps                : half-width of the smoothed Heaviside / Dirac (eqs 5-6)
    band_l             : narrow-band half-width l of h_eps (eq 11)
    d                  : Gaussian scale of the repulsion kernel (eq 10)
    R                  : half-width of the square repulsion window,
                         (2R+1) x (2R+1) taps (Sec. 4, window sum)
    sigma, rho, s_exp  : Gaussian pre-smoothing, scaling and exponent of g (eq 1)
    S                  : number of inner phi iterations (eq 37)
    tol_inner          : inner stop tolerance (Sec. 4, after eq 37); 0 = always S
    zero_tol           : |B| at or below this counts as the zero vector of
                         eq (42) (reading: the paper's 0 (0/|0|) = 0 applied to
                         B at rounding level, whose direction is noise); 0 is
                         the literal rule
    w_solver           : 0: w by soft thresholding (eqs 41, 42) then eq (40);
                         1: by the fixed-point iteration of eqs (38), (39) with
                         the projection of eq (40) after every sweep
    w_sweeps           : sweeps of that iteration, i.e. the paper's r = 0..R
                         with R = w_sweeps - 1 (one sweep: the paper's
                         "a single iteration is often enough")
    phi_solver         : 0: the FFT solve of eqs (30)-(33); 1: the AOS scheme
                         the paper names as the alternative (end of Sec. 4):
                         phi = (v + w) / 2 with (1 - 2 tau A_l) v = F along
                         columns and rows, A_l = mu x the periodic second
                         difference (constant A_l), each solved by the
                         Thomas algorithm
    bc                 : boundaries. 0: periodic (every operator wraps, the
                         FFT symbol of eq 32); 1: Neumann (eq 17's and eq
                         27's zero normal derivative): half-sample mirror
                         ghost values for every stencil, the Gaussian and the
                         repulsion window, the forward difference zero on
                         the last row / column, the divergence its negative
                         adjoint, and the DCT-II in place of the FFT
    """

    gamma: float = 1.0
    alpha: float = 1.0
    beta: float = 0.05
    mu: float = 0.1
    tau: float = 0.4
    eps: float = 1.5
    band_l: float = 1.0
    d: float = 3.0
    R: int = 3
    sigma: float = 1.5
    rho: float = 1000.0
    s_exp: int = 2
    S: int = 3
    tol_inner: float = 0.0
    zero_tol: float = 1e-3
    w_solver: int = 0
    w_sweeps: int = 1
    phi_solver: int = 0
    bc: int = 0


# --------------------------------------------------------------------------
# regularised Heaviside / Dirac and the narrow band  (eqs 5, 6, 11, 28, 29)
# --------------------------------------------------------------------------
def heaviside(phi, eps):
    """H_eps of eq (5): 1/2 (1 + phi/eps + sin(pi phi/eps)/pi) on |phi| <= eps,
    1 above, 0 below."""
    phi = np.asarray(phi, dtype=np.float64)
    inside = np.abs(phi) <= eps
    smooth = 0.5 * (1.0 + phi / eps + np.sin(np.pi * phi / eps) / np.pi)
    return np.where(inside, smooth, np.where(phi > eps, 1.0, 0.0))


def dirac(phi, eps):
    """delta_eps of eq (6): (1 + cos(pi phi/eps)) / (2 eps) on |phi| <= eps."""
    phi = np.asarray(phi, dtype=np.float64)
    inside = np.abs(phi) <= eps
    return np.where(inside, (1.0 + np.cos(np.pi * phi / eps)) / (2.0 * eps), 0.0)


def dirac_prime(phi, eps):
    """delta'_eps of eq (29): -(pi / (2 eps^2)) sin(pi phi/eps) on |phi| <= eps."""
    phi = np.asarray(phi, dtype=np.float64)
    inside = np.abs(phi) <= eps
    return np.where(inside, -(np.pi / (2.0 * eps * eps)) * np.sin(np.pi * phi / eps), 0.0)


def band(phi, eps, l):
    """Narrow band h_eps of eq (11): H_eps(phi + l) (1 - H_eps(phi - l))."""
    return heaviside(phi + l, eps) * (1.0 - heaviside(phi - l, eps))


def band_prime(phi, eps, l):
    """h'_eps of eq (28):
    delta_eps(phi + l)(1 - H_eps(phi - l)) - H_eps(phi + l) delta_eps(phi - l)."""
    return (dirac(phi + l, eps) * (1.0 - heaviside(phi - l, eps))
            - heaviside(phi + l, eps) * dirac(phi - l, eps))


# --------------------------------------------------------------------------
# discrete operators, unit spacing  (eqs 35, 36)
# --------------------------------------------------------------------------
# Array axis 0 is the row index i (first gradient component), axis 1 is the
# column index j (second component).  at(u, k, axis, bc) is u at index i + k
# along `axis`: periodic (bc = 0), or mirrored about the half-sample points
# -1/2 and n - 1/2 (bc = 1: the ghost value beyond an edge repeats the edge,
# ... u1 u0 | u0 u1 ... u_{n-1} | u_{n-1} u_{n-2} ...), which is the zero
# normal derivative of the Neumann condition.

def at(u, k, axis, bc=0):
    """u[i + k] along `axis` (|k| <= n), periodic or half-sample mirrored."""
    n = u.shape[axis]
    idx = np.arange(n) + k
    if bc == 0:
        idx = idx % n
    else:
        idx = np.where(idx < 0, -1 - idx, idx)
        idx = np.where(idx >= n, 2 * n - 1 - idx, idx)
    return np.take(u, idx, axis=axis)


def grad_fwd(u, bc=0):
    """Forward-difference gradient of eq (35): (u[i+1,j]-u[i,j], u[i,j+1]-u[i,j]);
    with Neumann boundaries the mirror ghost makes it zero on the last row
    (first component) and the last column (second component)."""
    return (at(u, 1, 0, bc) - u, at(u, 1, 1, bc) - u)


def _div1(p, axis, bc):
    if bc == 0:
        return p - at(p, -1, axis, 0)
    # negative adjoint of the Neumann forward difference along `axis`:
    # p[i] [i < n-1] - p[i-1] [i > 0]
    n = p.shape[axis]
    i = np.arange(n).reshape([-1 if a == axis else 1 for a in range(p.ndim)])
    return np.where(i < n - 1, p, 0.0) - np.where(i > 0, at(p, -1, axis, 1), 0.0)


def div_bwd(p, q, bc=0):
    """Backward-difference divergence of eq (36): (p[i,j]-p[i-1,j]) + (q[i,j]-q[i,j-1]),
    periodic; with Neumann boundaries the negative adjoint of grad_fwd (p
    taken as zero at index -1 and at the last index), so that
    div(grad u) is the mirrored Laplacian."""
    return _div1(p, 0, bc) + _div1(q, 1, bc)


def laplacian(u, bc=0):
    """Five-point Laplacian of eq (35) (mirror ghosts for Neumann boundaries)."""
    return (at(u, -1, 0, bc) + at(u, 1, 0, bc)
            + at(u, -1, 1, bc) + at(u, 1, 1, bc) - 4.0 * u)


# --------------------------------------------------------------------------
# edge-stopping function  (eq 1)
# --------------------------------------------------------------------------
def gaussian_taps(sigma):
    """Sampled Gaussian of standard deviation sigma, truncated at ceil(3 sigma)
    and normalised to unit sum (eq 1's G_sigma; truncation is a reading)."""
    r = int(math.ceil(3.0 * sigma))
    t = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-t * t / (2.0 * sigma * sigma))
    return t.astype(int), k / k.sum()


def gaussian_smooth(f, sigma, bc=0):
    """G_sigma * f with periodic wrap (or mirror): a row pass then a column pass."""
    offs, k = gaussian_taps(sigma)
    f = np.asarray(f, dtype=np.float64)
    rows = np.zeros_like(f)
    for t, kt in zip(offs, k):          # along axis 1 (within each row)
        rows += kt * at(f, t, 1, bc)
    out = np.zeros_like(f)
    for t, kt in zip(offs, k):          # along axis 0 (within each column)
        out += kt * at(rows, t, 0, bc)
    return out


def edge_map(f, sigma, rho, s_exp, bc=0):
    """g = 1 / (1 + rho |grad(G_sigma * f)|^s), eq (1), with central
    differences for the gradient of the smoothed image."""
    fs = gaussian_smooth(f, sigma, bc)
    gx = 0.5 * (at(fs, 1, 0, bc) - at(fs, -1, 0, bc))
    gy = 0.5 * (at(fs, 1, 1, bc) - at(fs, -1, 1, bc))
    mag = np.sqrt(gx * gx + gy * gy)
    return 1.0 / (1.0 + rho * mag ** s_exp)


# --------------------------------------------------------------------------
# repulsion window sum  (Sec. 4, the discrete v after eq 37)
# --------------------------------------------------------------------------
def repulsion_weights(R, d):
    """K[p+R, q+R] = exp(-(p^2 + q^2) / d^2) for p, q in [-R, R]."""
    p = np.arange(-R, R + 1, dtype=np.float64)
    return np.exp(-(p[:, None] ** 2 + p[None, :] ** 2) / (d * d))


def repulsion_field(w1, w2, phi, eps, l, d, R, bc=0):
    """v[i,j] = sum_{p,q=-R..R} exp(-(p^2+q^2)/d^2) w[i+p,j+q] h_eps(phi[i+p,j+q]),
    periodic (or mirrored) indices, centre tap included.  Direct (2R+1)^2-term sum."""
    h = band(phi, eps, l)
    u1, u2 = w1 * h, w2 * h
    K = repulsion_weights(R, d)
    v1 = np.zeros_like(u1)
    v2 = np.zeros_like(u2)
    for p in range(-R, R + 1):
        for q in range(-R, R + 1):
            kpq = K[p + R, q + R]
            v1 += kpq * at(at(u1, p, 0, bc), q, 1, bc)
            v2 += kpq * at(at(u2, p, 0, bc), q, 1, bc)
    return v1, v2


# --------------------------------------------------------------------------
# phi sub-problem: semi-implicit FFT scheme  (eqs 30-33, 37)
# --------------------------------------------------------------------------
def symbol(M, N, tau, mu):
    """Fourier symbol of (1 - tau mu Delta) on an M x N periodic grid, eq (32),
    with 0-based frequencies l1 (rows) and l2 (columns)."""
    z1 = 2.0 * np.pi * np.arange(M, dtype=np.float64) / M
    z2 = 2.0 * np.pi * np.arange(N, dtype=np.float64) / N
    return 1.0 - tau * mu * (2.0 * np.cos(z1)[:, None] + 2.0 * np.cos(z2)[None, :] - 4.0)


def implicit_solve(F, tau, mu, bc=0):
    """phi = Re( IFFT( FFT(F) / symbol ) ), eq (33): the solution of
    (1 - tau mu Delta) phi = F on the periodic grid; with Neumann
    boundaries the same solve in the DCT-II basis (the eigenvectors of the
    mirrored Laplacian)."""
    M, N = F.shape
    if bc == 1:
        return dct_solve(F, tau, mu)
    return np.real(np.fft.ifft2(np.fft.fft2(F) / symbol(M, N, tau, mu)))


def symbol_neumann(M, N, tau, mu):
    """Eigenvalues of (1 - tau mu Delta) for the mirrored Laplacian on the
    DCT-II modes cos(pi l (i + 1/2) / M) cos(pi m (j + 1/2) / N):
    1 + tau mu (4 - 2 cos(pi l / M) - 2 cos(pi m / N))."""
    z1 = np.pi * np.arange(M, dtype=np.float64) / M
    z2 = np.pi * np.arange(N, dtype=np.float64) / N
    return 1.0 + tau * mu * (4.0 - 2.0 * np.cos(z1)[:, None] - 2.0 * np.cos(z2)[None, :])


def dct_solve(F, tau, mu):
    """(1 - tau mu Delta) phi = F with Neumann boundaries: orthonormal
    DCT-II in both directions, division by the symbol, inverse transform."""
    from scipy import fft as sfft
    M, N = F.shape
    spec = sfft.dctn(np.asarray(F, dtype=np.float64), type=2, norm="ortho")
    return sfft.idctn(spec / symbol_neumann(M, N, tau, mu), type=2, norm="ortho")


def thomas(off, d, F):
    """Solve off x_{i-1} + d_i x_i + off x_{i+1} = F_i, i = 0..n-1 (no
    wrap-around), for every column of F (axis 0 is i): LR decomposition,
    forward substitution, backward substitution."""
    n = len(d)
    l = np.zeros(n)
    r = np.zeros(n)
    r[0] = d[0]
    for i in range(1, n):
        l[i] = off / r[i - 1]
        r[i] = d[i] - l[i] * off
    y = np.array(F, dtype=np.float64, copy=True)
    for i in range(1, n):                    # forward substitution (L y = F)
        y[i] = y[i] - l[i] * y[i - 1]
    x = np.empty_like(y)
    x[n - 1] = y[n - 1] / r[n - 1]
    for i in range(n - 2, -1, -1):           # backward substitution (R x = y)
        x[i] = (y[i] - off * x[i + 1]) / r[i]
    return x


def thomas_cyclic(off, diag, F):
    """Solve off x_{i-1} + diag x_i + off x_{i+1} = F_i, i = 0..n-1, with
    periodic indices, for every column of F (axis 0 is i), by the Thomas
    algorithm (LR decomposition, forward and backward substitution) on the
    tridiagonal part and the Sherman-Morrison formula for the two corner
    entries of the cyclic matrix."""
    F = np.asarray(F, dtype=np.float64)
    n = F.shape[0]
    gam = -diag
    # T = A - u v^T: corners removed, T[0,0] = diag - gam, T[n-1,n-1] = diag - off^2 / gam,
    # with u = (gam, 0, ..., 0, off), v = (1, 0, ..., 0, off / gam)
    d = np.full(n, diag, dtype=np.float64)
    d[0] -= gam
    d[-1] -= off * off / gam

    u = np.zeros(n)
    u[0], u[-1] = gam, off
    y = thomas(off, d, F)
    z = thomas(off, d, u if F.ndim == 1 else u[:, None] * np.ones((1,) + F.shape[1:]))
    vy = y[0] + (off / gam) * y[-1]
    vz = z[0] + (off / gam) * z[-1]
    return y - (vy / (1.0 + vz)) * z


def aos_solve(F, tau, mu, bc=0):
    """AOS solve of the phi sub-problem with constant A_l (the paper's
    alternative to the FFT, end of Sec. 4, in the form of eqs 18 and 20):
    (1 - 2 tau mu D_l) v_l = F for the periodic second difference D_l along
    columns (l = 1, index i) and rows (l = 2, index j); phi = (v_1 + v_2) / 2.
    With Neumann boundaries D_l is the mirrored second difference (end rows
    u_1 - u_0 and u_{n-2} - u_{n-1}): a plain tridiagonal system whose end
    diagonal entries are 1 + 2 tau mu."""
    off = -2.0 * tau * mu
    diag = 1.0 + 4.0 * tau * mu
    if bc == 1:
        def solve1(G):
            d = np.full(G.shape[0], diag)
            d[0] = d[-1] = 1.0 + 2.0 * tau * mu
            return thomas(off, d, G)
        return 0.5 * (solve1(F) + solve1(F.T).T)
    v1 = thomas_cyclic(off, diag, F)
    v2 = thomas_cyclic(off, diag, F.T).T
    return 0.5 * (v1 + v2)


def phi_rhs(phi_s, w1, w2, b1, b2, g, P: Params):
    """F^{k,s} of eq (37), evaluated at phi^{k+1,s} (reading: the inner iterate),
    with w^k, b^k fixed over the inner loop:
      F = phi_s + tau ( -gamma g |w| delta'(phi_s) + alpha g delta(phi_s)
                        + 2 beta h'(phi_s) w . v + mu div(b - w) )."""
    v1, v2 = repulsion_field(w1, w2, phi_s, P.eps, P.band_l, P.d, P.R, P.bc)
    wnorm = np.sqrt(w1 * w1 + w2 * w2)
    force = (-P.gamma * g * wnorm * dirac_prime(phi_s, P.eps)
             + P.alpha * g * dirac(phi_s, P.eps)
             + 2.0 * P.beta * band_prime(phi_s, P.eps, P.band_l) * (w1 * v1 + w2 * v2)
             + P.mu * div_bwd(b1 - w1, b2 - w2, P.bc))
    return phi_s + P.tau * force


def phi_subproblem(phi_k, w1, w2, b1, b2, g, P: Params):
    """Inner loop of Algorithm 1: phi^{k+1,0} = phi^k, then up to S semi-implicit
    steps (eq 37); stop early when ||phi^{k+1,s+1} - phi^{k+1,s}||_F /
    (||phi^{k+1,s}||_F + 1e-6) <= tol_inner (if tol_inner > 0).
    Returns (phi^{k+1}, number of inner steps taken)."""
    phi_s = phi_k
    steps = 0
    for _ in range(P.S):
        F = phi_rhs(phi_s, w1, w2, b1, b2, g, P)
        if P.phi_solver == 1:
            phi_new = aos_solve(F, P.tau, P.mu, P.bc)
        else:
            phi_new = implicit_solve(F, P.tau, P.mu, P.bc)
        steps += 1
        rel = np.linalg.norm(phi_new - phi_s) / (np.linalg.norm(phi_s) + 1e-6)
        phi_s = phi_new
        if P.tol_inner > 0 and rel <= P.tol_inner:
            break
    return phi_s, steps


# --------------------------------------------------------------------------
# w sub-problem: soft thresholding + projection, Bregman  (eqs 40-42, 23)
# --------------------------------------------------------------------------
def shrink(B1, B2, t, zero_tol=0.0):
    """Generalised soft thresholding of eq (42):
    max(|B| - t, 0) B / |B|, with the zero vector where |B| <= zero_tol
    (zero_tol = 0: exactly the paper's 0 (0/|0|) = 0)."""
    nb = np.sqrt(B1 * B1 + B2 * B2)
    live = nb > zero_tol
    scale = np.where(live, np.maximum(nb - t, 0.0) / np.where(nb > 0, nb, 1.0), 0.0)
    return scale * B1, scale * B2


def project(w1, w2):
    """Projection of eq (40) onto |w| = 1; the zero vector stays zero."""
    n = np.sqrt(w1 * w1 + w2 * w2)
    safe = np.where(n > 0, n, 1.0)
    return np.where(n > 0, w1 / safe, 0.0), np.where(n > 0, w2 / safe, 0.0)


def shrink_input(phi_new, w1, w2, b1, b2, g, P: Params):
    """B^{k+1} of eq (41) and the threshold of eq (42):
    B = grad phi^{k+1} + b^k + (2 beta / mu) h(phi^{k+1}) v, with v built from
    w^k and h(phi^{k+1}); t = (gamma / mu) g delta(phi^{k+1})."""
    G1, G2 = grad_fwd(phi_new, P.bc)
    v1, v2 = repulsion_field(w1, w2, phi_new, P.eps, P.band_l, P.d, P.R, P.bc)
    h = band(phi_new, P.eps, P.band_l)
    c = 2.0 * P.beta / P.mu
    B1 = G1 + b1 + c * h * v1
    B2 = G2 + b2 + c * h * v2
    t = (P.gamma / P.mu) * g * dirac(phi_new, P.eps)
    return B1, B2, t


def w_subproblem(phi_new, w1, w2, b1, b2, g, P: Params):
    """w^{k+1}: soft thresholding of eq (42) applied to B of eq (41), then the
    projection of eq (40) (the paper applies it afterwards)."""
    B1, B2, t = shrink_input(phi_new, w1, w2, b1, b2, g, P)
    s1, s2 = shrink(B1, B2, t, P.zero_tol)
    return project(s1, s2)


def w_fixed_point(phi_new, w1, w2, b1, b2, g, P: Params):
    """w^{k+1} by the fixed-point iteration of eqs (38)-(40): w^{k+1,0} = w^k;
    sweep r builds v^{k+1,r} (eq 38) from w^{k+1,r} and h(phi^{k+1}), then
      w~ = (mu grad phi^{k+1} + mu b^k + 2 beta h(phi^{k+1}) v^{k+1,r})
           / (gamma g delta(phi^{k+1}) + mu)                       (eq 39)
    and w^{k+1,r+1} = w~ / |w~| (eq 40); P.w_sweeps sweeps.  Zero rule
    (the reading taken for eq 42, applied to the same vector): where the
    numerator over mu -- B of eq (41) built from w^{k+1,r} -- has
    |B| <= zero_tol, w^{k+1,r+1} is the zero vector."""
    G1, G2 = grad_fwd(phi_new, P.bc)
    h = band(phi_new, P.eps, P.band_l)
    den = P.gamma * g * dirac(phi_new, P.eps) + P.mu
    wr1, wr2 = w1, w2
    for _ in range(P.w_sweeps):
        v1, v2 = repulsion_field(wr1, wr2, phi_new, P.eps, P.band_l, P.d, P.R, P.bc)
        n1 = P.mu * G1 + P.mu * b1 + 2.0 * P.beta * h * v1
        n2 = P.mu * G2 + P.mu * b2 + 2.0 * P.beta * h * v2
        t1, t2 = project(n1 / den, n2 / den)
        live = np.sqrt(n1 * n1 + n2 * n2) / P.mu > P.zero_tol
        wr1, wr2 = np.where(live, t1, 0.0), np.where(live, t2, 0.0)
    return wr1, wr2


def bregman(b1, b2, phi_new, w1_new, w2_new, bc=0):
    """b^{k+1} = b^k + grad phi^{k+1} - w^{k+1}, eq (23)."""
    G1, G2 = grad_fwd(phi_new, bc)
    return b1 + G1 - w1_new, b2 + G2 - w2_new


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
@dataclasses.dataclass
class State:
    phi: np.ndarray
    w1: np.ndarray
    w2: np.ndarray
    b1: np.ndarray
    b2: np.ndarray
    k: int = 0


def initial_state(phi0, bc=0):
    """Initialisation of Algorithm 1: phi^0 given (a signed distance function),
    w^0 = grad phi^0, b^0 = 0."""
    phi0 = np.asarray(phi0, dtype=np.float64)
    w1, w2 = grad_fwd(phi0, bc)
    z = np.zeros_like(phi0)
    return State(phi0.copy(), w1, w2, z.copy(), z.copy(), 0)


def sb_iteration(st: State, g, P: Params):
    """One outer iteration k of Algorithm 1: inner phi loop (eq 37),
    w by eq (42) then eq (40) (or by eqs 38-40 when P.w_solver = 1), b by
    eq (23).  Returns (new state, info)."""
    phi_new, steps = phi_subproblem(st.phi, st.w1, st.w2, st.b1, st.b2, g, P)
    w_update = w_fixed_point if P.w_solver == 1 else w_subproblem
    w1n, w2n = w_update(phi_new, st.w1, st.w2, st.b1, st.b2, g, P)
    b1n, b2n = bregman(st.b1, st.b2, phi_new, w1n, w2n, P.bc)
    r = np.linalg.norm(phi_new - st.phi) / (np.linalg.norm(st.phi) + 1e-6)
    return State(phi_new, w1n, w2n, b1n, b2n, st.k + 1), {"r": r, "inner_steps": steps}


def solve(f, phi0, P: Params, iters, tol_outer=0.0, min_iters=0, callback=None):
    """Algorithm 1 from the image f and phi^0 for at most `iters` outer
    iterations; stops early when the relative phi change r_k < tol_outer
    (after min_iters).  Returns (final state, g, list of r_k)."""
    g = edge_map(f, P.sigma, P.rho, P.s_exp, P.bc)
    st = initial_state(phi0, P.bc)
    hist = []
    for _ in range(iters):
        st, info = sb_iteration(st, g, P)
        hist.append(info["r"])
        if callback is not None:
            callback(st)
        if tol_outer > 0 and st.k >= min_iters and info["r"] < tol_outer:
            break
    return st, g, hist


# --------------------------------------------------------------------------
# SR energy  (eqs 7-10)
# --------------------------------------------------------------------------
def energy_terms(phi, g, P: Params):
    """(gamma E_g, alpha E_a, beta E_r) of eqs (7)-(10) on the grid, unit cell
    area, with the forward gradient and the repulsion integral truncated to the
    same (2R+1)^2 window as the solver:
      E_g = sum g |grad phi| delta(phi)
      E_a = sum g (1 - H(phi))
      E_r = - sum_x (grad phi h)(x) . sum_y K(x-y) (grad phi h)(y)."""
    G1, G2 = grad_fwd(phi, P.bc)
    Eg = np.sum(g * np.sqrt(G1 * G1 + G2 * G2) * dirac(phi, P.eps))
    Ea = np.sum(g * (1.0 - heaviside(phi, P.eps)))
    h = band(phi, P.eps, P.band_l)
    v1, v2 = repulsion_field(G1, G2, phi, P.eps, P.band_l, P.d, P.R, P.bc)
    Er = -np.sum(G1 * h * v1 + G2 * h * v2)
    return P.gamma * Eg, P.alpha * Ea, P.beta * Er


def energy(phi, g, P: Params):
    """E = gamma E_g + alpha E_a + beta E_r, eq (7)."""
    return float(sum(energy_terms(phi, g, P)))
