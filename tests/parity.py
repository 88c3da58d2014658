"""Element-wise parity bars of one outer iteration of Algorithm 1 computed
by the FP32 library against the FP64 oracle from the same (FP32-valued)
state -- teacher forcing.

phi.  The library adds the increment of each inner step to phi_s in FP32
(the increment form of eq 30), so its error at a pixel is a few roundings of
phi itself plus the FP32 error of the increments, which the FFT spreads over
the grid at the scale of the largest increment.  The bar at each pixel is

    |phi_gpu - phi_ora| <= 4 ulp32(phi_ora) + 1e-5 max |phi_ora - phi_start|,

so a wrong update shows wherever it exceeds 1e-5 of the update (a whole-field
relative L2 bar on phi cannot: one iteration changes a 1024^2 signed distance
function by ~1e-4 of its norm).  The AOS solve of the phi sub-problem is not
in increment form: each inner step convolves values of the size of phi with
up to 2K + 1 = 55 taps in FP32, a rounding of about sqrt(2K + 1) / 2 ulp of
phi per step, so its bar takes 4 ulp per inner step (ulps = 4 S).

w and b.  w = B / |B| behind the gate |B| > max(t, zero_tol) (eqs 40-42).
The library's B differs from the oracle's by the error of grad+ phi^{k+1}
(from the phi bar at the pixel and its forward neighbours) plus the FP32
rounding of b and of the repulsion term, the threshold t by the error of
g delta(phi).  A gate decision may differ only where |B| lies within four
times those errors of the threshold (a flip); every other pixel must agree:
closed on both sides (w = 0 exactly), or open with |w_gpu - w_ora| within
four times error(B) / |B|.  b = b^k + grad+ phi^{k+1} - w^{k+1} (eq 23) then
agrees to the gradient error plus the w error, except at flips, where w
differs by a unit vector; flips are counted and returned so that a caller
comparing later iterations can mask their stencil neighbourhood.
"""
import numpy as np


def ulp32(x):
    """Spacing of float32 numbers at |x|."""
    return np.spacing(np.abs(np.asarray(x, dtype=np.float64)).astype(np.float32)).astype(np.float64)


def phi_tol(ref_phi, start_phi, ulps=4.0):
    upd = float(np.abs(ref_phi - start_phi).max())
    return ulps * ulp32(ref_phi) + 1e-5 * upd


def check_phi(gphi, ref_phi, start_phi, what="phi", ulps=4.0):
    """The element-wise phi bar above; returns the worst ratio error / bar."""
    gphi = np.asarray(gphi, dtype=np.float64)
    tol = phi_tol(ref_phi, start_phi, ulps)
    err = np.abs(gphi - ref_phi)
    ratio = err / tol
    worst = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    assert ratio[worst] <= 1.0, (f"{what}: worst pixel {worst}: |gpu - oracle| = {err[worst]:.3e} > bar "
                                 f"{tol[worst]:.3e} (phi {ref_phi[worst]:.4f}, max update "
                                 f"{np.abs(ref_phi - start_phi).max():.3e})")
    return float(ratio[worst])


def _fwd(a, axis):
    return np.roll(a, -1, axis)


def check_w_b(gw, gb, ref_w, ref_b, start_b, B, t, zero_tol, g, delta, ddelta_max, gamma_over_mu, ptol,
              max_flip_frac=1e-3):
    """w and b of one iteration, gate-aware (see the module docstring).

    gw, gb, ref_w, ref_b, start_b, B: lists of components (2-D or 3-D);
    t: the oracle's threshold of eq (42) (zeros for the fixed-point solver);
    g, delta: the oracle's g and delta_eps(phi^{k+1}); ddelta_max: bound of
    |delta'_eps|; ptol: the phi bar (phi_tol) of this iteration.
    Returns the flip mask."""
    nd = len(B)
    gw = [np.asarray(c, dtype=np.float64) for c in gw]
    gb = [np.asarray(c, dtype=np.float64) for c in gb]
    # error of grad+ phi^{k+1}, per component: the bar at the pixel and at its forward neighbour
    eG = [ptol + _fwd(ptol, a) for a in range(nd)]
    eGm = np.maximum.reduce(eG)
    nb = np.sqrt(sum(c * c for c in B))
    bmag = np.sqrt(sum(c * c for c in start_b))
    eB = np.sqrt(nd) * eGm + 1e-5 * (1.0 + bmag)
    et = gamma_over_mu * g * (2e-6 * delta + ddelta_max * ptol) + 1e-7 * t
    thr = np.maximum(t, zero_tol)
    near = np.abs(nb - thr) <= 4.0 * (eB + et)
    n_ref = np.sqrt(sum(c * c for c in ref_w))
    n_gpu = np.sqrt(sum(c * c for c in gw))
    open_ref, open_gpu = n_ref > 0.5, n_gpu > 0.5
    flips = open_ref != open_gpu
    bad = flips & ~near
    assert not bad.any(), (f"{int(bad.sum())} gate decisions differ away from the gate, e.g. at "
                           f"{tuple(np.argwhere(bad)[0])}: |B| = {nb[bad][0]:.4e}, threshold {thr[bad][0]:.4e}")
    assert flips.mean() <= max_flip_frac, flips.mean()
    closed = ~open_ref & ~flips
    assert np.all(n_gpu[closed] == 0.0), "w must be exactly zero where both gates are closed"
    both = open_ref & ~flips
    wtol = 4.0 * eB / np.where(nb > 0, nb, 1.0) + 4e-7
    werr = np.sqrt(sum((a - b) ** 2 for a, b in zip(gw, ref_w)))
    r = np.where(both, werr / wtol, 0.0)
    worst = np.unravel_index(int(np.argmax(r)), r.shape)
    assert r[worst] <= 1.0, (f"w at {worst}: error {werr[worst]:.3e} > {wtol[worst]:.3e} (|B| = {nb[worst]:.4e}, "
                             f"threshold {thr[worst]:.4e})")
    ok = ~flips
    for a in range(nd):
        btol = eG[a] + np.where(both, wtol, 0.0) + 2.0 * ulp32(ref_b[a]) + 2.0 * ulp32(start_b[a])
        berr = np.abs(gb[a] - ref_b[a])
        rb = np.where(ok, berr / btol, 0.0)
        wb = np.unravel_index(int(np.argmax(rb)), rb.shape)
        assert rb[wb] <= 1.0, f"b[{a}] at {wb}: error {berr[wb]:.3e} > {btol[wb]:.3e}"
    return flips


def flip_neighbourhood(flips, radius):
    """Pixels within `radius` (periodic, Chebyshev distance) of a flip."""
    out = flips.copy()
    for a in range(flips.ndim):
        acc = out.copy()
        for s in range(1, radius + 1):
            acc |= np.roll(out, s, a) | np.roll(out, -s, a)
        out = acc
    return out
