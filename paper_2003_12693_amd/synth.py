"""Seeded synthetic inputs: images f and initial level sets phi^0.

This module holds no arithmetic of the segmentation method itself; it only
draws test images and analytic signed distance functions.  Both the HIP
library's tests/benchmarks and the FP64 oracle's tests take their inputs from
here, so the two sides always see identical data (float64 here; the GPU side
receives a float32 cast).

The paper's own images (two circles, a synthetic hand, cells, wheat grains,
CT slices) are not available, so these generators stand in for them:

* ``two_disks``      - two unit-intensity disks with a 4 px gap and one
                       enclosing circular initial contour: the splitting-
                       prevention set-up of the paper's first experiment.
* ``ellipses``       - many ellipses with 2-6 px gaps, a low-frequency bias
                       field and Gaussian noise (the "adhesive cells / grains"
                       situation: close objects that must not merge).
* ``annuli``         - annuli and ellipses with holes, some crossed by
                       occluding bars (large-grid stress case).
* ``batch_items``    - many uneven-size ``ellipses`` instances.

Geometry conventions: pixel (i, j) has centre (i, j); i is the row index.
Level sets are negative inside (the paper's sign convention).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import ndimage


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _grid(M, N):
    i = np.arange(M, dtype=np.float64)[:, None]
    j = np.arange(N, dtype=np.float64)[None, :]
    return i, j


def circle_sdf(M, N, radius, center=None):
    """Signed distance to a circle (negative inside)."""
    c = ((M - 1) / 2.0, (N - 1) / 2.0) if center is None else center
    i, j = _grid(M, N)
    return np.sqrt((i - c[0]) ** 2 + (j - c[1]) ** 2) - radius


def rect_sdf(M, N, inset):
    """Signed distance to the rectangle [inset, M-1-inset] x [inset, N-1-inset]."""
    i, j = _grid(M, N)
    lo_i, hi_i = float(inset), float(M - 1 - inset)
    lo_j, hi_j = float(inset), float(N - 1 - inset)
    di = np.maximum(lo_i - i, i - hi_i)          # >0 outside along i
    dj = np.maximum(lo_j - j, j - hi_j)
    outside = np.sqrt(np.maximum(di, 0.0) ** 2 + np.maximum(dj, 0.0) ** 2)
    inside = np.minimum(np.maximum(di, dj), 0.0)  # <=0 inside: -(distance to edge)
    return outside + inside


# --------------------------------------------------------------------------
# two disks (128 x 128 by default)
# --------------------------------------------------------------------------
def two_disks(M=128, N=128, seed=1, radius=20.0, gap=4.0, noise=0.1, phi_radius=60.0):
    """Two disks of radius `radius`, intensity 1, edge gap `gap`, on 0, plus
    i.i.d. N(0, noise^2).  phi^0 = circle of radius `phi_radius` about the
    image centre.  Returns (f, phi0)."""
    rng = _rng(seed)
    c = ((M - 1) / 2.0, (N - 1) / 2.0)
    off = radius + gap / 2.0
    i, j = _grid(M, N)
    f = np.zeros((M, N))
    for s in (-1.0, 1.0):
        f[(i - c[0]) ** 2 + (j - (c[1] + s * off)) ** 2 <= radius * radius] = 1.0
    f = f + rng.normal(0.0, noise, size=(M, N))
    return f, circle_sdf(M, N, phi_radius, c)


# --------------------------------------------------------------------------
# ellipses with small gaps (1024 x 1024 by default)
# --------------------------------------------------------------------------
def _ellipse_mask(M, N, ci, cj, a, b, th, box):
    i0, i1, j0, j1 = box
    ii = np.arange(i0, i1, dtype=np.float64)[:, None] - ci
    jj = np.arange(j0, j1, dtype=np.float64)[None, :] - cj
    ct, st = math.cos(th), math.sin(th)
    u = ct * ii + st * jj
    v = -st * ii + ct * jj
    return (u / a) ** 2 + (v / b) ** 2 <= 1.0


def _place_shapes(M, N, n, axis_lo, axis_hi, rng, clearance, gap_lo=2.0, gap_hi=6.0,
                  max_reject=1000):
    """Rejection placement of n ellipses: each new ellipse keeps >= gap_lo px
    (pixels strictly between the masks) to all placed ones and, except the
    first, lies <= gap_hi px from its nearest neighbour.  A new shape is
    proposed next to a random placed one, along a random direction, at the
    distance where its gap is about the middle of [gap_lo, gap_hi]
    (bisection).  Gaps are tested against masks of the placed shapes grown
    by Euclidean distance (one distance transform per placed shape)."""
    d_lo, d_mid, d_hi = gap_lo + 1.0, 0.5 * (gap_lo + gap_hi) + 1.0, gap_hi + 1.0
    near_lo = np.zeros((M, N), dtype=bool)   # distance to placed shapes < d_lo
    near_mid = np.zeros((M, N), dtype=bool)  # < d_mid
    near_hi = np.zeros((M, N), dtype=bool)   # <= d_hi
    shapes = []
    scale = 1.0
    rejects = 0
    grow = int(math.ceil(d_hi)) + 1

    def box_of(ci, cj, rmax):
        box = (int(ci - rmax) - 1, int(ci + rmax) + 3, int(cj - rmax) - 1, int(cj + rmax) + 3)
        if box[0] < 0 or box[2] < 0 or box[1] > M or box[3] > N:
            return None
        return box

    def hits(mask, box, cand):
        return bool((mask[box[0]:box[1], box[2]:box[3]] & cand).any())

    def add(box, cand):
        a0, a1 = max(box[0] - grow, 0), min(box[1] + grow, M)
        b0, b1 = max(box[2] - grow, 0), min(box[3] + grow, N)
        c = np.zeros((a1 - a0, b1 - b0), dtype=bool)
        c[box[0] - a0:box[1] - a0, box[2] - b0:box[3] - b0] = cand
        dist = ndimage.distance_transform_edt(~c)
        near_lo[a0:a1, b0:b1] |= dist < d_lo
        near_mid[a0:a1, b0:b1] |= dist < d_mid
        near_hi[a0:a1, b0:b1] |= dist <= d_hi

    while len(shapes) < n:
        a = rng.uniform(axis_lo, axis_hi) * scale
        b = rng.uniform(axis_lo, axis_hi) * scale
        th = rng.uniform(0.0, math.pi)
        rmax = max(a, b)
        lo_i, hi_i = clearance + rmax, M - 1 - clearance - rmax
        lo_j, hi_j = clearance + rmax, N - 1 - clearance - rmax
        if lo_i >= hi_i or lo_j >= hi_j:
            scale *= 0.9
            continue
        ok = False
        if shapes:
            k = shapes[rng.integers(len(shapes))]
            ang = rng.uniform(0.0, 2.0 * math.pi)
            di, dj = math.cos(ang), math.sin(ang)
            t_lo, t_hi = 0.0, max(k[2], k[3]) + rmax + gap_hi + 4.0
            for _ in range(12):
                t = 0.5 * (t_lo + t_hi)
                bx = box_of(k[0] + t * di, k[1] + t * dj, rmax)
                if bx is None:
                    break
                cand = _ellipse_mask(M, N, k[0] + t * di, k[1] + t * dj, a, b, th, bx)
                if hits(near_mid, bx, cand):
                    t_lo = t
                else:
                    t_hi = t
            ci, cj = k[0] + t_hi * di, k[1] + t_hi * dj
            box = box_of(ci, cj, rmax)
            if box is not None and lo_i <= ci <= hi_i and lo_j <= cj <= hi_j:
                cand = _ellipse_mask(M, N, ci, cj, a, b, th, box)
                ok = (not hits(near_lo, box, cand)) and hits(near_hi, box, cand)
        else:
            ci = rng.uniform(lo_i, hi_i)
            cj = rng.uniform(lo_j, hi_j)
            box = box_of(ci, cj, rmax)
            if box is not None:
                cand = _ellipse_mask(M, N, ci, cj, a, b, th, box)
                ok = True
        if ok:
            add(box, cand)
            shapes.append((ci, cj, a, b, th))
            rejects = 0
        else:
            rejects += 1
            if rejects >= max_reject:
                scale *= 0.9
                rejects = 0
    return shapes


def ellipses(M=1024, N=1024, seed=2, n_shapes=12, axis_lo=30.0, axis_hi=120.0,
             noise=0.15, bias=0.2, inset=16, fg=(0.6, 1.0), bg=(0.0, 0.2)):
    """Ellipses (intensity U[fg]) with 2-6 px gaps on a U[bg] background,
    multiplied by a one-sinusoid bias field of amplitude `bias`, plus
    N(0, noise^2).  phi^0 = rectangle inset by `inset` px.  Returns (f, phi0)."""
    rng = _rng(seed)
    shapes = _place_shapes(M, N, n_shapes, axis_lo, axis_hi, rng, clearance=inset + 8)
    f = np.full((M, N), rng.uniform(*bg))
    for (ci, cj, a, b, th) in shapes:
        rmax = max(a, b)
        box = (max(int(ci - rmax) - 1, 0), min(int(ci + rmax) + 3, M),
               max(int(cj - rmax) - 1, 0), min(int(cj + rmax) + 3, N))
        m = _ellipse_mask(M, N, ci, cj, a, b, th, box)
        f[box[0]:box[1], box[2]:box[3]][m] = rng.uniform(*fg)
    if bias > 0:
        ang = rng.uniform(0.0, 2.0 * math.pi)
        psi = rng.uniform(0.0, 2.0 * math.pi)
        i, j = _grid(M, N)
        f = f * (1.0 + bias * np.sin(2.0 * math.pi * (math.cos(ang) * i + math.sin(ang) * j) / 1024.0 + psi))
    f = f + rng.normal(0.0, noise, size=(M, N))
    return f, rect_sdf(M, N, inset)


# --------------------------------------------------------------------------
# annuli / holed ellipses with occluding bars (4096 x 4096 by default)
# --------------------------------------------------------------------------
def annuli(M=4096, N=4096, seed=3, n_shapes=64, axis_lo=60.0, axis_hi=240.0,
           noise=0.2, bar_frac=0.1, inset=16):
    """Half annuli, half ellipses with concentric elliptical holes (hole scale
    q ~ U[0.3, 0.6]); about `bar_frac` of the shapes are crossed by a bar of
    background intensity (width U[4, 12] px).  Returns (f, phi0)."""
    rng = _rng(seed)
    shapes = _place_shapes(M, N, n_shapes, axis_lo, axis_hi, rng, clearance=inset + 8)
    bg = rng.uniform(0.0, 0.2)
    f = np.full((M, N), bg)
    for idx, (ci, cj, a, b, th) in enumerate(shapes):
        if idx % 2 == 0:   # annulus: circle of the larger axis
            a = b = max(a, b)
        q = rng.uniform(0.3, 0.6)
        rmax = max(a, b)
        box = (max(int(ci - rmax) - 1, 0), min(int(ci + rmax) + 3, M),
               max(int(cj - rmax) - 1, 0), min(int(cj + rmax) + 3, N))
        outer = _ellipse_mask(M, N, ci, cj, a, b, th, box)
        inner = _ellipse_mask(M, N, ci, cj, q * a, q * b, th, box)
        sub = f[box[0]:box[1], box[2]:box[3]]
        sub[outer & ~inner] = rng.uniform(0.6, 1.0)
        if rng.uniform() < bar_frac:
            wbar = rng.uniform(4.0, 12.0)
            ang = rng.uniform(0.0, math.pi)
            ii = np.arange(box[0], box[1], dtype=np.float64)[:, None] - ci
            jj = np.arange(box[2], box[3], dtype=np.float64)[None, :] - cj
            dist = np.abs(-math.sin(ang) * ii + math.cos(ang) * jj)
            along = np.abs(math.cos(ang) * ii + math.sin(ang) * jj)
            sub[(dist <= wbar / 2.0) & (along <= rmax)] = bg
    f = f + rng.normal(0.0, noise, size=(M, N))
    return f, rect_sdf(M, N, inset)


# --------------------------------------------------------------------------
# many uneven instances
# --------------------------------------------------------------------------
BATCH_SIZES = ((128, 128), (256, 256), (512, 512), (256, 512), (512, 1024))


def batch_sizes(count=256, size_seed=4999):
    """(M, N, R) of the first `count` instances of the batched workload:
    sizes drawn uniformly from BATCH_SIZES, R ~ U{3, 4, 5}."""
    rs = _rng(size_seed)
    out = []
    for _ in range(count):
        M, N = BATCH_SIZES[rs.integers(len(BATCH_SIZES))]
        out.append((M, N, int(rs.integers(3, 6))))
    return out


def batch_instance(k, M, N, seed0=4000):
    """Image and initial level set of instance k (size M x N): an
    ``ellipses`` image whose shape count and axes scale with the area."""
    area = M * N / (1024.0 * 1024.0)
    n = max(1, int(round(12 * area)))
    s = math.sqrt(area)
    lo = min(max(30.0 * s, 8.0), 0.3 * min(M, N))
    hi = min(max(120.0 * s, 8.0), 0.3 * min(M, N))
    return ellipses(M, N, seed=seed0 + k, n_shapes=n, axis_lo=lo, axis_hi=hi)


def batch_items(count=256, size_seed=4999, seed0=4000):
    """Instance list: (M, N, R, f, phi0) of the batched workload."""
    return [(M, N, R) + tuple(batch_instance(k, M, N, seed0))
            for k, (M, N, R) in enumerate(batch_sizes(count, size_seed))]


def batch_subset(n=32, count=256, size_seed=4999):
    """Indices of a size-stratified subset of the batched workload: the
    first instances of each size class in turn (round robin over the
    classes in the order of BATCH_SIZES), n in all."""
    sizes = batch_sizes(count, size_seed)
    by = {sz: [k for k, (M, N, R) in enumerate(sizes) if (M, N) == sz] for sz in BATCH_SIZES}
    out, r = [], 0
    while len(out) < n:
        for sz in BATCH_SIZES:
            if r < len(by[sz]) and len(out) < n:
                out.append(by[sz][r])
        r += 1
    return sorted(out)


# --------------------------------------------------------------------------
# volumes for the 3-D solver: touching balls (a stand-in for the paper's CT
# volume, which is not available)
# --------------------------------------------------------------------------
def balls3d(M=128, N=128, P=128, seed=6, n_balls=6, r_lo=0.08, r_hi=0.16, noise=0.15, bias=0.2, inset=0.08):
    """f: n_balls balls of radius r_lo..r_hi (fractions of the smallest side),
    centres drawn so that neighbours nearly touch (gaps of 1-4 voxels where
    the draw allows), intensity 1 inside, `bias` background, Gaussian noise;
    phi0: signed distance to the box inset by `inset` of each side (negative
    inside), the initial contour enclosing every ball."""
    rng = _rng(seed)
    s = float(min(M, N, P))
    i = np.arange(M, dtype=np.float64)[:, None, None]
    j = np.arange(N, dtype=np.float64)[None, :, None]
    k = np.arange(P, dtype=np.float64)[None, None, :]
    lo = np.array([inset * M, inset * N, inset * P]) + r_hi * s + 2
    hi = np.array([M, N, P]) - lo
    balls = []
    for _ in range(200):
        if len(balls) == n_balls:
            break
        r = rng.uniform(r_lo, r_hi) * s
        if balls and rng.uniform() < 0.7:       # next to an earlier ball, a small gap apart
            c0, r0 = balls[rng.integers(len(balls))]
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            c = c0 + u * (r0 + r + rng.uniform(1.0, 4.0))
        else:
            c = rng.uniform(lo, hi)
        if np.any(c < lo) or np.any(c > hi):
            continue
        if any(np.linalg.norm(c - c1) < r + r1 + 1.0 for c1, r1 in balls):
            continue
        balls.append((c, r))
    f = np.full((M, N, P), bias)
    for c, r in balls:
        f[(i - c[0]) ** 2 + (j - c[1]) ** 2 + (k - c[2]) ** 2 <= r * r] = 1.0
    f = f + noise * rng.normal(size=(M, N, P))
    d = [np.maximum(inset * n - x, x - (n - 1 - inset * n)) for x, n in ((i, M), (j, N), (k, P))]
    outside = np.sqrt(sum(np.maximum(a, 0.0) ** 2 for a in d))
    inside = np.minimum(np.maximum(np.maximum(d[0], d[1]), d[2]), 0.0)
    return f.astype(np.float32), (outside + inside).astype(np.float32)
