"""GPU tests of the batched solve (sr_solve_batch) through the C ABI."""
import sys

import numpy as np
import pytest

from oracle import sr_oracle as O
from paper_2003_12693_amd import synth
from tests.helpers import as64, f32, gpu_params, oracle_params, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sr():
    from paper_2003_12693_amd import sr as srmod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    srmod.load()
    return srmod


def _cuda(x):
    return torch.from_numpy(f32(x)).cuda()


def _instances():
    out = []
    for k, (M, N, R) in enumerate([(64, 64, 3), (64, 128, 3), (128, 128, 4), (64, 64, 5), (64, 128, 3),
                                   (128, 64, 4)]):
        f, phi0 = synth.ellipses(M, N, seed=100 + k, n_shapes=2, axis_lo=6.0, axis_hi=14.0, inset=8)
        out.append((M, N, R, f, phi0))
    return out


def test_batch_matches_single_instance_solves(sr):
    _note("batch vs single")
    inst = _instances()
    items = [dict(f=_cuda(f), phi0=_cuda(p), max_iter=7, params=gpu_params(R=R, d=float(R)))
             for (M, N, R, f, p) in inst]
    rc, res = sr.solve_batch(items)
    assert rc == 0
    for (M, N, R, f, p), r in zip(inst, res):
        assert r["iters"] == 7 and r["status"] == 0
        s = sr.Solver(M, N, gpu_params(R=R, d=float(R)))
        s.set_image(_cuda(f), _cuda(p))
        s.step(7)
        ref = s.phi().cpu().numpy()
        got = r["phi"].cpu().numpy()
        assert rel_l2(got, ref) <= 1e-6
        E, _ = s.energy()
        assert abs(r["energy"] - E) <= 1e-6 * abs(E)


C4_SIZES = [(128, 128, 3), (256, 256, 4), (512, 512, 5), (256, 512, 3), (512, 1024, 4)]


def _c4_instance(M, N, R, seed):
    """One instance of the batched workload's generator at a given size:
    ellipses with shape count and axes scaled to the area."""
    area = M * N / (1024.0 * 1024.0)
    n = max(1, int(round(12 * area)))
    sc = area ** 0.5
    lo = min(max(30.0 * sc, 8.0), 0.3 * min(M, N))
    hi = min(max(120.0 * sc, 8.0), 0.3 * min(M, N))
    return synth.ellipses(M, N, seed=seed, n_shapes=n, axis_lo=lo, axis_hi=hi)


@pytest.mark.parametrize("k", [2, 9])
def test_batch_against_oracle(sr, k):
    """Per instance, teacher-forced through sr_solve_batch: one instance of
    every size of the batched workload (128^2 ... 512 x 1024, R 3-5) solved
    together for k iterations (final phi, w, b returned) and again for k + 1;
    the last iteration of the second call starts from the first call's state
    (the batch is deterministic), so it is compared with one oracle iteration
    from that state by the element-wise bars (phi; w and b gate-aware)."""
    _note(f"batch vs oracle, teacher forced at k={k}")
    from tests.parity import check_phi, check_w_b, phi_tol
    inst = [(M, N, R) + tuple(_c4_instance(M, N, R, 4100 + i)) for i, (M, N, R) in enumerate(C4_SIZES)]

    def run(n):
        items = [dict(f=_cuda(f), phi0=_cuda(p), max_iter=n, params=gpu_params(R=R, d=float(R)), want_state=True)
                 for (M, N, R, f, p) in inst]
        rc, res = sr.solve_batch(items)
        assert rc == 0 and all(r["iters"] == n for r in res)
        return [(r["phi"].cpu().numpy(), r["w"].cpu().numpy(), r["b"].cpu().numpy()) for r in res]

    before, after = run(k), run(k + 1)
    for (M, N, R, f, p), (phi, w, b), (gphi, gw, gb) in zip(inst, before, after):
        P = oracle_params(R=R, d=float(R))
        g = O.edge_map(as64(f), P.sigma, P.rho, P.s_exp)
        start = O.State(as64(phi), as64(w[0]), as64(w[1]), as64(b[0]), as64(b[1]), k)
        ref, _ = O.sb_iteration(start, g, P)
        ratio = check_phi(gphi, ref.phi, start.phi, what=f"{M}x{N} R{R}")
        B1, B2, t = O.shrink_input(ref.phi, start.w1, start.w2, start.b1, start.b2, g, P)
        flips = check_w_b([gw[0], gw[1]], [gb[0], gb[1]], [ref.w1, ref.w2], [ref.b1, ref.b2],
                          [start.b1, start.b2], [B1, B2], t, P.zero_tol, g, O.dirac(ref.phi, P.eps),
                          np.pi / (2 * P.eps ** 2), P.gamma / P.mu, phi_tol(ref.phi, start.phi))
        _note(f"  {M}x{N} R{R}: worst phi error {ratio:.3f} of the bar, {int(flips.sum())} gate flips")


def test_batch_stratified_subset_against_oracle(sr):
    """32 instances of the 256-instance batched workload itself (7, 7, 6, 6, 6
    of the five sizes, R 3-5, the workload's seeds), solved together for 5
    iterations and for 6; each instance's sixth iteration is compared with
    one oracle iteration from its state after 5 (teacher forcing through the
    batch) by the element-wise bars."""
    _note("batch stratified 32-instance subset vs oracle")
    from tests.parity import check_phi, check_w_b, phi_tol
    sizes = synth.batch_sizes(256)
    sub = synth.batch_subset(32)
    inst = [sizes[k] + tuple(synth.batch_instance(k, sizes[k][0], sizes[k][1])) for k in sub]
    k = 5

    def run(n):
        items = [dict(f=_cuda(f), phi0=_cuda(p), max_iter=n, params=gpu_params(R=R, d=float(R)), want_state=True)
                 for (M, N, R, f, p) in inst]
        rc, res = sr.solve_batch(items)
        assert rc == 0 and all(r["iters"] == n for r in res)
        return [(r["phi"].cpu().numpy(), r["w"].cpu().numpy(), r["b"].cpu().numpy()) for r in res]

    before, after = run(k), run(k + 1)
    worst, flips_total = 0.0, 0
    for (M, N, R, f, p), (phi, w, b), (gphi, gw, gb) in zip(inst, before, after):
        P = oracle_params(R=R, d=float(R))
        g = O.edge_map(as64(f), P.sigma, P.rho, P.s_exp)
        start = O.State(as64(phi), as64(w[0]), as64(w[1]), as64(b[0]), as64(b[1]), k)
        ref, _ = O.sb_iteration(start, g, P)
        worst = max(worst, check_phi(gphi, ref.phi, start.phi, what=f"{M}x{N} R{R}"))
        B1, B2, t = O.shrink_input(ref.phi, start.w1, start.w2, start.b1, start.b2, g, P)
        flips = check_w_b([gw[0], gw[1]], [gb[0], gb[1]], [ref.w1, ref.w2], [ref.b1, ref.b2],
                          [start.b1, start.b2], [B1, B2], t, P.zero_tol, g, O.dirac(ref.phi, P.eps),
                          np.pi / (2 * P.eps ** 2), P.gamma / P.mu, phi_tol(ref.phi, start.phi))
        flips_total += int(flips.sum())
    _note(f"  32 instances: worst phi error {worst:.3f} of the bar, {flips_total} gate flips in all")


def test_batch_tolerance_and_caps(sr):
    _note("batch tolerance")
    inst = _instances()
    items = []
    for k, (M, N, R, f, p) in enumerate(inst):
        params = gpu_params(R=R, d=float(R), tol_outer=3e-3 if k % 2 == 0 else 0.0, min_iter=4)
        items.append(dict(f=_cuda(f), phi0=_cuda(p), max_iter=25 + k, params=params))
    rc, res = sr.solve_batch(items)
    for k, r in enumerate(res):
        if k % 2 == 0:
            assert r["status"] in (0, 1)
            if r["status"] == 0:
                assert r["r_last"] < 3e-3 and 4 <= r["iters"] <= 25 + k
            else:
                assert r["iters"] == 25 + k
        else:
            assert r["status"] == 0 and r["iters"] == 25 + k
    # the same instance solved alone for the reported iteration count agrees
    M, N, R, f, p = inst[0]
    s = sr.Solver(M, N, gpu_params(R=R, d=float(R)))
    s.set_image(_cuda(f), _cuda(p))
    s.step(res[0]["iters"])
    assert rel_l2(res[0]["phi"].cpu().numpy(), s.phi().cpu().numpy()) <= 1e-6


def test_batch_nonfinite_instance_isolated(sr):
    _note("batch nonfinite")
    inst = _instances()[:3]
    items = [dict(f=_cuda(f), phi0=_cuda(p), max_iter=5, params=gpu_params(R=R, d=float(R)))
             for (M, N, R, f, p) in inst]
    bad = inst[1][3].copy()
    bad[3, 3] = np.nan
    items[1]["f"] = _cuda(bad)
    rc, res = sr.solve_batch(items)
    assert res[1]["status"] == sr.SR_ENONFINITE
    assert res[0]["status"] == 0 and res[0]["iters"] == 5
    assert res[2]["status"] == 0 and res[2]["iters"] == 5


def test_autotune_leaves_state_and_results_unchanged(sr):
    """The tuner times the rhs kernel on the live state: the iterate is
    untouched, and the per-pixel arithmetic does not depend on the tile
    height, so every later iterate is bitwise the same."""
    _note("autotune")
    import os
    f, p = synth.ellipses(256, 256, seed=7, n_shapes=3, axis_lo=10.0, axis_hi=30.0, inset=8)
    kw = gpu_params(R=4, d=4.0)
    ref = sr.Solver(256, 256, kw)
    ref.set_image(_cuda(f), _cuda(p))
    ref.step(5)
    want = ref.phi().cpu().numpy()
    s = sr.Solver(256, 256, kw)
    s.set_image(_cuda(f), _cuda(p))
    before = s.phi().cpu().numpy()
    th, us = s.autotune(3)
    _note(f"  chose {th} rows; mean us per candidate {us}")
    assert th in (8, 16, 32) and all(v > 0 for v in us.values())
    assert np.array_equal(s.phi().cpu().numpy(), before)
    s.step(5)
    assert np.array_equal(s.phi().cpu().numpy(), want)
    for forced in ("8", "32"):
        os.environ["SR_TILE_TH"] = forced
        try:
            t = sr.Solver(256, 256, kw)
        finally:
            del os.environ["SR_TILE_TH"]
        t.set_image(_cuda(f), _cuda(p))
        t.step(5)
        assert np.array_equal(t.phi().cpu().numpy(), want), forced


def test_component_operators_leave_solver_state_unchanged(sr):
    """The component operators (edge map, repulsion field, implicit solve)
    called with host arrays stage them in the context's free planes: the
    phi plane of the pair that does not hold phi^k, the spare inner
    iterate, the free w / b halves.  Called at an odd and at an even
    iteration count, they leave the state (phi, w, b, k) bitwise unchanged,
    and the solve then continues bitwise like one that never called them."""
    _note("component operators with host staging mid-solve")
    M, N = 128, 256
    f, p = synth.ellipses(M, N, seed=21, n_shapes=3, axis_lo=10.0, axis_hi=30.0, inset=8)
    kw = gpu_params(R=3, d=4.0)
    ref = sr.Solver(M, N, kw)
    ref.set_image(_cuda(f), _cuda(p))
    ref.step(7)
    want = [t.cpu().numpy() for t in ref.get_state()[:3]]
    s = sr.Solver(M, N, kw)
    s.set_image(_cuda(f), _cuda(p))
    rng = np.random.default_rng(3)
    host = lambda *shape: rng.normal(size=shape).astype(np.float32)
    for k in (3, 6):   # operators at an odd, then an even iteration count
        s.step(3)
        before = [t.cpu().numpy() for t in s.get_state()[:3]]
        g = sr.sr_edge_map(s.ctx, host(M, N), np.empty((M, N), np.float32))
        v = sr.sr_repulsion(s.ctx, host(2, M, N), host(M, N), np.empty((2, M, N), np.float32))
        u = sr.sr_implicit_solve(s.ctx, host(M, N), np.empty((M, N), np.float32))
        assert all(np.isfinite(x).all() for x in (g, v, u))
        after = s.get_state()
        assert after[3] == k
        for a, b in zip(before, after[:3]):
            assert np.array_equal(a, b.cpu().numpy())
    s.step(1)
    got = s.get_state()
    assert got[3] == 7
    for a, b in zip(want, got[:3]):
        assert np.array_equal(a, b.cpu().numpy())


def test_fixed_point_w_batch_matches_single(sr):
    """17 instances of 512^2 with the fixed-point w solver (3 sweeps): the
    batch (above 4 Mpx per launch: 64x16 w-step tiles on 256 threads) gives
    bitwise the results of single solves (64x32 tiles on 512 threads), whose
    sweeps the teacher-forced tests check against the oracle."""
    _note("fixed-point w: batch vs single")
    kw = gpu_params(w_solver=1, w_sweeps=3)
    inst = [synth.ellipses(512, 512, seed=900 + i, n_shapes=3, axis_lo=15.0, axis_hi=60.0, inset=16)
            for i in range(17)]
    items = [dict(f=_cuda(f), phi0=_cuda(p), max_iter=3, params=kw) for (f, p) in inst]
    rc, res = sr.solve_batch(items)
    assert rc == 0
    for (f, p), r in zip(inst[:4] + inst[-2:], res[:4] + res[-2:]):
        assert r["iters"] == 3 and r["status"] == 0
        s = sr.Solver(512, 512, kw)
        s.set_image(_cuda(f), _cuda(p))
        s.step(3)
        assert np.array_equal(r["phi"].cpu().numpy(), s.phi().cpu().numpy())


@pytest.mark.parametrize("kernel", ["gather", "slide"])
def test_aos_batch_matches_single(sr, kernel, monkeypatch):
    """Uneven instances with the AOS phi solver: the batched solve gives
    bitwise the single solves' results."""
    monkeypatch.setenv("SR_AOS_KERNEL", kernel)
    _note(f"AOS: batch vs single ({kernel})")
    kw = gpu_params(phi_solver=1)
    inst = _instances()[:5]
    items = [dict(f=_cuda(f), phi0=_cuda(p), max_iter=4, params=gpu_params(phi_solver=1, R=R, d=float(R)))
             for (M, N, R, f, p) in inst]
    rc, res = sr.solve_batch(items)
    assert rc == 0
    for (M, N, R, f, p), r in zip(inst, res):
        s = sr.Solver(M, N, gpu_params(phi_solver=1, R=R, d=float(R)))
        s.set_image(_cuda(f), _cuda(p))
        s.step(4)
        assert np.array_equal(r["phi"].cpu().numpy(), s.phi().cpu().numpy())


@pytest.mark.parametrize("phi_solver", [0, 1])
def test_neumann_batch_matches_single(sr, phi_solver):
    """Neumann boundaries: the batched solve gives bitwise the single solves'
    results."""
    _note(f"Neumann: batch vs single (phi_solver={phi_solver})")
    inst = _instances()[:5]
    items = [dict(f=_cuda(f), phi0=_cuda(p), max_iter=4,
                  params=gpu_params(bc=1, phi_solver=phi_solver, R=R, d=float(R)))
             for (M, N, R, f, p) in inst]
    rc, res = sr.solve_batch(items)
    assert rc == 0
    for (M, N, R, f, p), r in zip(inst, res):
        s = sr.Solver(M, N, gpu_params(bc=1, phi_solver=phi_solver, R=R, d=float(R)))
        s.set_image(_cuda(f), _cuda(p))
        s.step(4)
        assert np.array_equal(r["phi"].cpu().numpy(), s.phi().cpu().numpy())
