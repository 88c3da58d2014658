"""Benchmark of the Split Bregman SR solver on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload ellipses-1024|annuli-4096]

A step is one outer iteration of Algorithm 1 (S inner FFT solves with the
fused repulsion window, then shrink / projection / Bregman) over one
synthetic image, with the inputs resident in HBM.  Prints one JSON line with
the throughput in megapixel-iterations per second, the roofline position of
the dominant kernel (HIP-event timing of each kernel kind on the solver's
stream, algorithmic bytes per launch), and the FP64 oracle timed on the host
on a bounded sample of the same workload.

    python bench.py --copy-probe 256

runs a plain 256 MiB device-to-device copy ten times and exits; profiled
with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE it calibrates those counters.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic (compulsory) bytes per pixel per launch of each kernel kind, FP32
# planes.  One inner step moves 40 B/px: read phi_s, w (2), g, D = 20 and
# write the half spectrum 4 (the rhs fused into the forward row FFT), the
# column solve reads and writes the spectrum (8), the inverse row FFT reads
# it and writes phi (8); the w step reads phi, w (2), b (2), g = 24 and writes
# w (2), b (2), D = 20.  Per outer iteration 40 S + 44 = 164 B/px at S = 3.
# With the rhs and the forward row FFT as separate launches the rhs kind is
# charged the reads (20) and the row FFT the spectrum write (4): the rhs
# plane they pass between them is not compulsory traffic.
BYTES_PER_PX = {"rhs_row_fft_fwd": 24, "rhs_repulsion": 20, "row_fft_fwd": 4, "col_fft_solve": 8,
                "row_fft_inv": 8, "w_step": 44}
# a fixed-point w sweep before the last one: reads phi (4), w (8), b (8), g (4), writes w (8)
BYTES_PER_PX_W_SWEEP = 32
# the AOS phi solve (one launch in place of the three FFT passes): reads r and phi_s, writes phi
BYTES_PER_PX_AOS = 12

# The paper's two-circles weights (alpha = gamma = 4, beta = 0.2, mu = 8,
# tau = 0.1, l = 1, d = 5, S = 3) with each workload's eps / R.
WORKLOADS = {
    "ellipses-1024": dict(M=1024, N=1024, R=3, eps=1.5, d=5.0, S=3, default_steps=2000,
                          text="ellipses-1024x1024: 12 ellipses with 2-6 px gaps, bias 0.2, noise 0.15; "
                               "rectangle phi0; R=3, eps=1.5, d=5, S=3, paper two-circles weights"),
    "annuli-4096": dict(M=4096, N=4096, R=5, eps=2.0, d=5.0, S=3, default_steps=300,
                        text="annuli-4096x4096: 64 annuli / holed ellipses, 10% crossed by bars, noise 0.2; "
                             "rectangle phi0; R=5, eps=2, d=5, S=3, paper two-circles weights"),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.txt")


def params_kw(wl):
    kw = dict(gamma=4.0, alpha=4.0, beta=0.2, mu=8.0, tau=0.1, eps=wl["eps"], band_l=1.0,
              d=wl["d"], R=wl["R"], sigma=1.5, rho=1000.0, s_exp=2, S=wl["S"],
              tol_inner=0.0, zero_tol=1e-3)
    if wl.get("w_sweeps"):   # the fixed-point w solver of eqs 38-40
        kw.update(w_solver=1, w_sweeps=wl["w_sweeps"])
    if wl.get("phi_solver") == "aos":   # AOS with constant A_l (end of Sec. 4)
        # at tau mu = 0.8 the AOS average under-damps modes that oscillate along
        # one axis (steady-state response up to 1 + 8 tau mu times the exact
        # one) and the Bregman update amplifies that: the iteration diverges;
        # tau = 0.04 (tau mu = 0.32) keeps it stable
        kw.update(phi_solver=1, tau=0.04)
    if wl.get("bc") == "neumann":   # zero normal derivative (eqs 17, 27)
        kw.update(bc=1)
    return kw


def make_input(name):
    from paper_2003_12693_amd import synth
    if name == "ellipses-1024":
        return synth.ellipses(1024, 1024, seed=2)
    return synth.annuli(4096, 4096, seed=3)


def build_source_id():
    """Digest of the sources in this tree, as the build script computes it
    (compared with the loaded library's sr_build_id)."""
    from paper_2003_12693_amd import build
    return build.source_id()


def measured_traffic(workload, kernel, tile_rows, build_id):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None if it was taken on a library built from other sources.  The
    separate right-hand-side kernel's traffic depends on its tile height
    (halo rows), so it is listed per height ("rhs_repulsion@16").  A 3-D
    kind that runs several kernels is listed as the mean over its launches
    of one outer iteration."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    key = f"{kernel}@{tile_rows}" if kernel == "rhs_repulsion" else kernel
    for line in open(TRAFFIC_FILE):
        parts = line.split("#", 1)[0].split()
        if len(parts) == 4 and parts[0] == workload and parts[1] == key and parts[3] == build_id:
            return int(parts[2])
    return None


def _oracle_run(f, phi0, kw, iters):
    """Seconds for `iters` outer iterations of the FP64 oracle (edge map and
    initialisation excluded); run in this process or in a worker."""
    from oracle import sr_oracle as O
    P = O.Params(**kw)
    g = O.edge_map(f, P.sigma, P.rho, P.s_exp)
    st = O.initial_state(phi0)
    t1 = time.perf_counter()
    for _ in range(iters):
        st, _ = O.sb_iteration(st, g, P)
    return time.perf_counter() - t1


def host_cpu():
    """(usable cores, capped at 16 -- the host share of one GPU -- and the CPU model)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return min(int(n or 1), 16), model


def cpu_baseline(f, phi0, wl, iters, all_cores=True):
    """The FP64 oracle as it stands (one NumPy process is single-threaded)
    timed on the host: one process, and one process per usable core running
    the same sample concurrently (the host's aggregate oracle throughput)."""
    M, N = f.shape
    kw = params_kw(wl)
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    t1 = _oracle_run(f, phi0, kw, iters)
    one = M * N * iters / 1e6 / t1
    cores, model = host_cpu()
    out = {"value": one, "unit": "MPix-it/s", "cores": 1, "kind": "oracle",
           "sample": f"{iters} outer iterations of the FP64 NumPy oracle on the same {M}x{N} input "
                     f"({t1:.1f} s; edge map and initialisation excluded)",
           "cpu": model, "nproc": cores}
    if all_cores and cores > 1:
        import multiprocessing as mp
        ctx = mp.get_context("spawn")
        t0 = time.perf_counter()
        with ctx.Pool(cores) as pool:
            secs = pool.starmap(_oracle_run, [(f, phi0, kw, iters)] * cores)
        wall = time.perf_counter() - t0
        slowest = max(secs)
        out.update(value=cores * M * N * iters / 1e6 / slowest, cores=cores,
                   sample=out["sample"] + f"; {cores} concurrent single-threaded oracle processes, aggregate over "
                                          f"the slowest ({slowest:.1f} s; {wall:.1f} s with start-up)",
                   single_core={"value": one, "cores": 1})
    return out


# The paper's 3-D (mandible) weights with a 5 x 5 x 5 window.
PARAMS_3D = dict(gamma=5.0, alpha=4.0, beta=0.2, mu=3.0, tau=0.05, eps=1.0, band_l=1.0, d=4.0, R=2, S=5,
                 sigma=1.5, rho=1000.0, s_exp=2, tol_inner=0.0, zero_tol=1e-3)
# algorithmic bytes per voxel per launch of each 3-D kernel kind (FP32):
#   window: the k pass reads w (12) and phi (4) and writes 3 components
#           (12); the j and i passes read and write 3 components (24): mean of 3
#   The spectrum holds k frequencies 0..P/2: h = 8 (P/2 + 1) / P bytes per voxel.
#   rhs (with the forward k transform): reads phi, w, g, v, D (4 + 12 + 4 +
#        12 + 4), writes the spectrum (h); the first of the S = 5 inner steps
#        reads b (12) and writes D (4) instead of reading D: + 12 / 5
#   fft: three passes read and write h each; the last reads h + phi_s 4,
#        writes 4: mean of 4
#   w step: reads phi, b, g, v (4 + 12 + 4 + 12), writes w and b (24)
BYTES_PER_VOX_3D = {"window": (28 + 2 * 24) / 3, "w_step": 56}


def bytes_per_vox_3d(kind, P):
    h = 8.0 * (P // 2 + 1) / P
    if kind == "rhs":
        return 36 + h + 12 / 5
    if kind == "fft":
        return (3 * 2 * h + h + 8) / 4
    return BYTES_PER_VOX_3D[kind]


def volume_bench(S, steps, warmup, cpu):
    """3-D solver on an S^3 volume of touching balls: throughput in
    megavoxel-iterations per second, per-kernel-kind timing, roofline."""
    import torch
    from paper_2003_12693_amd import sr, synth
    f, phi0 = synth.balls3d(S, S, S)
    s = sr.Solver3D(S, S, S, sr.sr_params_default(**PARAMS_3D))
    s.set_image(torch.from_numpy(f).cuda(), torch.from_numpy(phi0).cuda())
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    t1 = time.perf_counter()
    value = S ** 3 * steps / 1e6 / (t1 - t0)
    prof = sr.sr3_profile(s.ctx, 3)
    per_iter_ms = {k: v[0] * v[1] / 3 for k, v in prof.items()}
    dom = max(per_iter_ms, key=per_iter_ms.get)
    achieved = bytes_per_vox_3d(dom, S) * S ** 3 / (prof[dom][0] * 1e-3) / 1e9
    build_id = sr.sr_build_id()
    traffic = measured_traffic(f"balls3d-{S}", dom, None, build_id)
    out = {"metric": f"3-D SB megavoxel-iters/s at {S}^3", "value": round(value, 2), "unit": "MVox-it/s",
           "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round((t1 - t0) * 1e3 / steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"balls3d-{S}: touching balls, bias 0.2, noise 0.15, box phi0; the paper's 3-D "
                                  "weights (gamma 5, alpha 4, beta 0.2, mu 3, tau 0.05, eps 1, l 1, d 4, 5^3 window, "
                                  "S 5)"},
           "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                        "alg_bytes_per_launch": bytes_per_vox_3d(dom, S) * S ** 3},
           "kernels_ms": {k: round(v[0], 5) for k, v in prof.items()},
           "iteration_ms_sum_of_kernels": round(sum(per_iter_ms.values()), 4),
           "build_id": build_id}
    if traffic is not None:   # bytes the counters saw move, over the same duration
        out["roofline"]["achieved_by_counters"] = round(traffic / (prof[dom][0] * 1e-3) / 1e9, 1)
        out["roofline"]["frac_by_counters"] = round(out["roofline"]["achieved_by_counters"] / HBM_PEAK_GBS, 4)
    if cpu:
        from oracle import sr_oracle as O
        from oracle import sr_oracle3d as O3
        n = 96
        fc, pc = synth.balls3d(n, n, n)
        P = O.Params(**{k: v for k, v in PARAMS_3D.items() if k in O.Params.__dataclass_fields__})
        g = O3.edge_map(fc.astype(np.float64), P.sigma, P.rho, P.s_exp)
        st = O3.initial_state(pc.astype(np.float64))
        c0 = time.perf_counter()
        O3.sb_iteration(st, g, P)
        c1 = time.perf_counter()
        out["cpu_baseline"] = {"value": round(n ** 3 / 1e6 / (c1 - c0), 4), "unit": "MVox-it/s", "cores": 1,
                               "kind": "oracle", "sample": f"1 outer iteration of the FP64 NumPy 3-D oracle on a "
                                                           f"{n}^3 volume of the same kind ({c1 - c0:.1f} s)"}
    return out


def converge_bench(name, tol, cap, min_iter, check_every):
    """Time-to-converge of one workload under Algorithm 1's stop rule read as
    the relative phi change r_k < tol (after min_iter), checked every
    check_every iterations, capped at cap: set_image (edge map, initial
    state) plus the iterations, with f and phi0 already in HBM."""
    import torch
    from paper_2003_12693_amd import sr
    wl = dict(WORKLOADS[name])
    M, N = wl["M"], wl["N"]
    f, phi0 = make_input(name)
    kw = dict(params_kw(wl), tol_outer=tol, min_iter=min_iter, check_every=check_every)
    s = sr.Solver(M, N, device="cuda:0", **kw)
    ft = torch.from_numpy(f.astype(np.float32)).cuda()
    pt = torch.from_numpy(phi0.astype(np.float32)).cuda()
    s.set_image(ft, pt)          # warm-up: code objects and graphs, then a busy GPU
    s.prepare()
    s.step(check_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_image(ft, pt)
    info = s.step(cap)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    E, _ = s.energy()
    return {"metric": f"time-to-converge at {M}x{N} (r_k < {tol} after {min_iter}, checked every {check_every}, "
                      f"cap {cap})", "value": round(t, 4), "unit": "s", "higher_is_better": False,
            "iterations": info["k"], "converged": info["converged"], "r_last": info["r_last"],
            "ms_per_iteration": round(t * 1e3 / max(info["k"], 1), 4), "energy": E,
            "n_gpus": 1, "dtype": "f32", "data": "synthetic", "config": {"workload": wl["text"]}}


def batch_bench(count, cap, tol, cpu):
    """Time-to-converge of `count` uneven instances: one sr_solve_batch call
    against sequential plain solves (sr_step with the same stop rule).  With
    the CPU leg, a size-stratified 32-instance subset is also run 5 and 6
    iterations by the batch (final w, b returned) and the FP64 oracle times
    one iteration from each instance's state after 5: its throughput is the
    CPU baseline, and the batch's sixth iteration is compared with it per
    pixel (|phi_gpu - phi_ora| against 4 ulp32 + 1e-5 of the update; w gate
    decisions)."""
    import torch
    from paper_2003_12693_amd import sr, synth
    insts = synth.batch_items(count=count)
    dev = []
    for (M, N, R, f, phi0) in insts:
        kw = dict(params_kw(dict(eps=1.5, d=float(R), R=R, S=3)), tol_outer=tol, min_iter=20, check_every=10)
        dev.append((M, N, R, torch.from_numpy(f.astype(np.float32)).cuda(),
                    torch.from_numpy(phi0.astype(np.float32)).cuda(), kw))
    items = [dict(f=f, phi0=p, max_iter=cap, params=sr.sr_params_default(**kw)) for (M, N, R, f, p, kw) in dev]
    sr.solve_batch(items[:4])          # warm-up: code objects, graph machinery
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, res = sr.solve_batch(items)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    # sequential plain solves of the same instances
    t_plain = 0.0
    agree = []
    px_it = 0
    for (M, N, R, f, p, kw), r in zip(dev, res):
        s = sr.Solver(M, N, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_image(f, p)
        info = s.step(cap)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        px_it += M * N * r["iters"]
        same_iters = info["k"] == r["iters"]
        rel = float(torch.linalg.norm(s.phi() - r["phi"]) / torch.linalg.norm(s.phi()))
        agree.append((same_iters, rel))
        s.close()
    conv = sum(1 for r in res if r["status"] == 0)
    out = {
        "metric": f"time-to-converge, {count} uneven instances (sizes 128^2..512x1024, R 3-5, cap {cap}, r_k<{tol})",
        "value": round(t_batch, 4), "unit": "s", "higher_is_better": False,
        "plain_sequential_s": round(t_plain, 4), "speedup_vs_plain": round(t_plain / t_batch, 2),
        "batched_mpix_it_per_s": round(px_it / 1e6 / t_batch, 1),
        "converged": conv, "instances": count,
        "iters_equal_to_plain": sum(1 for a in agree if a[0]),
        "max_rel_phi_diff_vs_plain_when_iters_equal": max([a[1] for a in agree if a[0]] or [0.0]),
        "n_gpus": 1, "dtype": "f32", "data": "synthetic",
    }
    if cpu:
        out["cpu_baseline"] = batch_oracle_leg(sr)
    return out


def batch_oracle_leg(sr, k=5, n=32):
    """The oracle on the stratified subset: one iteration per instance from
    the batch's state after k iterations, timed; agreement of the batch's
    iteration k + 1 with it."""
    import torch
    from oracle import sr_oracle as O
    from paper_2003_12693_amd import synth
    sizes = synth.batch_sizes(256)
    sub = synth.batch_subset(n)
    inst = [sizes[i] + tuple(synth.batch_instance(i, sizes[i][0], sizes[i][1])) for i in sub]

    def run(iters):
        items = [dict(f=torch.from_numpy(f.astype(np.float32)).cuda(), phi0=torch.from_numpy(p.astype(np.float32)).cuda(),
                      max_iter=iters, want_state=True,
                      params=sr.sr_params_default(**params_kw(dict(eps=1.5, d=float(R), R=R, S=3))))
                 for (M, N, R, f, p) in inst]
        _, res = sr.solve_batch(items)
        return [(r["phi"].cpu().numpy().astype(np.float64), r["w"].cpu().numpy().astype(np.float64),
                 r["b"].cpu().numpy().astype(np.float64)) for r in res]

    before, after = run(k), run(k + 1)
    t_or, px, worst, gate_diff = 0.0, 0, 0.0, 0
    for (M, N, R, f, p), (phi, w, b), (gphi, gw, gb) in zip(inst, before, after):
        P = O.Params(**params_kw(dict(eps=1.5, d=float(R), R=R, S=3)))
        g = O.edge_map(f.astype(np.float32).astype(np.float64), P.sigma, P.rho, P.s_exp)
        st = O.State(phi, w[0], w[1], b[0], b[1], k)
        c0 = time.perf_counter()
        ref, _ = O.sb_iteration(st, g, P)
        t_or += time.perf_counter() - c0
        px += M * N
        ulp = np.spacing(np.abs(ref.phi).astype(np.float32)).astype(np.float64)
        bar = 4 * ulp + 1e-5 * np.abs(ref.phi - phi).max()
        worst = max(worst, float((np.abs(gphi - ref.phi) / bar).max()))
        gate_diff += int(np.count_nonzero((np.hypot(gw[0], gw[1]) > 0.5) != (np.hypot(ref.w1, ref.w2) > 0.5)))
    return {"value": round(px / 1e6 / t_or, 4), "unit": "MPix-it/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 NumPy oracle iteration on each of a size-stratified {n}-instance subset "
                      f"({t_or:.1f} s), from the batch's state after {k} iterations",
            "agreement": {"instances": n, "teacher_forced_at_k": k,
                          "worst_phi_error_over_bar": round(worst, 4), "w_gate_decisions_differing": gate_diff,
                          "bar": "|phi_gpu - phi_oracle| <= 4 ulp32(phi) + 1e-5 max|update| per pixel"}}


MFMA_BF16_PEAK_TFLOPS = 2500.0


def cnn_bench(batch, H, steps, warmup, train_batch, cpu):
    """Warm-start network throughput on H x H inputs: inference (forward on
    `batch` images) and training (forward + backward + Adam on `train_batch`
    images), with inputs resident in HBM; MFMA utilisation against the dense
    BF16 peak."""
    import torch
    from paper_2003_12693_amd import cnn
    rng = np.random.default_rng(0)

    def inputs(n):
        f = torch.from_numpy(rng.uniform(0, 1, (n, H, H)).astype(np.float32)).cuda()
        g = torch.from_numpy(rng.uniform(0.05, 1, (n, H, H)).astype(np.float32)).cuda()
        p = torch.from_numpy(rng.normal(0, 6, (n, H, H)).astype(np.float32)).cuda()
        return f, g, p

    params = cnn.he_init(1)
    res = {}
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # inference
    net = cnn.Network(batch, H, H, params)
    f, g, p = inputs(batch)
    out = torch.empty_like(f)
    for _ in range(warmup):
        cnn.cnn_forward(net.ctx, f, g, p, batch, 8.0, out)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        cnn.cnn_forward(net.ctx, f, g, p, batch, 8.0, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1) / steps
    fl_fwd, _ = cnn.flops(batch, H, H)
    net.close()
    del net
    # training
    net = cnn.Network(train_batch, H, H, params)
    f, g, p = inputs(train_batch)
    t = torch.from_numpy(rng.normal(0, 6, (train_batch, H, H)).astype(np.float32)).cuda()
    for _ in range(warmup):
        cnn.cnn_forward(net.ctx, f, g, p, train_batch, 8.0)
        cnn.cnn_backward(net.ctx, t, 8.0, want_loss=False)
        cnn.cnn_adam_step(net.ctx, 1e-4)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        cnn.cnn_forward(net.ctx, f, g, p, train_batch, 8.0)
        cnn.cnn_backward(net.ctx, t, 8.0, want_loss=False)
        cnn.cnn_adam_step(net.ctx, 1e-4)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_train = e0.elapsed_time(e1) / steps
    _, fl_train = cnn.flops(train_batch, H, H)
    net.close()
    tf_fwd = fl_fwd / (ms_fwd * 1e-3) / 1e12
    tf_train = fl_train / (ms_train * 1e-3) / 1e12
    out = {
        "metric": f"CNN warm-start inference images/s at {H}^2",
        "value": round(batch / (ms_fwd * 1e-3), 2), "unit": "images/s", "higher_is_better": True,
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(ms_fwd, 4),
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"warm-start encoder-decoder (3x3 convs 16-32-64-128, BF16 storage, FP32 "
                               f"accumulate) on {batch} x 3 x {H}x{H} inputs",
                   "gflop_per_image_forward": round(fl_fwd / batch / 1e9, 3),
                   "gflop_per_image_train_step": round(fl_train / train_batch / 1e9, 3)},
        "roofline": {"bound": "mfma", "kernel": "whole forward pass", "achieved": round(tf_fwd, 2),
                     "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf_fwd / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None},
        "training": {"batch": train_batch, "ms_per_step": round(ms_train, 3),
                     "images_per_s": round(train_batch / (ms_train * 1e-3), 2),
                     "tflops": round(tf_train, 2), "frac": round(tf_train / MFMA_BF16_PEAK_TFLOPS, 4)},
    }
    if cpu:
        from oracle import cnn_reference as R
        from paper_2003_12693_amd.cnn import he_init
        pr = R.unflatten(he_init(1).astype(np.float64))
        hs = 256
        x = rng.normal(size=(1, hs, hs, 3))
        t0 = time.perf_counter()
        R.forward(pr, x)
        dt = time.perf_counter() - t0
        fl, _ = cnn.flops(1, hs, hs)
        out["cpu_baseline"] = {"value": round(fl / dt / (fl_fwd / batch), 4), "unit": "images/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"FP64 NumPy reference forward of one {hs}x{hs} image ({dt:.1f} s), "
                                         f"scaled to {H}x{H} by the FLOP count"}
    return out


def warmstart_bench(n):
    """Time-to-solve on n held-out 512^2 instances: the plain solver's
    fixed-budget solve against the committed warm-start network's start
    refined by Split Bregman to the same energy (inference, refinement and
    fallbacks included)."""
    from paper_2003_12693_amd import warmstart as W
    params = np.load(W.WEIGHTS)
    W.evaluate(params, [W.EVAL_SEED0 + 999], k_plain=200, log=lambda m: None)     # warm-up
    summary, rows = W.evaluate(params, list(range(W.EVAL_SEED0, W.EVAL_SEED0 + n)), log=lambda m: None)
    return {
        "metric": f"time-to-solve at {W.SIZE}^2, plain ({W.K_PLAIN} iterations) vs CNN warm start",
        "value": round(summary["mean_s_warm_incl_inference_and_fallback"], 5), "unit": "s",
        "higher_is_better": False, "plain_s": round(summary["mean_s_plain"], 5),
        "speedup_vs_plain": round(summary["mean_s_plain"] / summary["mean_s_warm_incl_inference_and_fallback"], 2),
        "iters_saved_frac": round(summary["iters_saved_frac"], 4), "accepted": summary["accepted"],
        "instances": summary["instances"], "fallback_rate": summary["fallback_rate"],
        "within_window": summary["within_window"], "max_abs_rel_dE_accepted": summary["max_abs_rel_dE_accepted"],
        "n_gpus": 1, "dtype": "f32 solver, bf16 network", "data": "synthetic",
        "config": {"workload": f"{n} held-out 512^2 ellipse images (3 ellipses, semi-axes 15-60 px, noise 0.15, "
                               f"bias 0.2), rectangle phi0, paper two-circles weights, R=3, eps=1.5"},
    }


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_mib": mib, "bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="ellipses-1024", choices=sorted(WORKLOADS))
    ap.add_argument("--profile-iters", type=int, default=20)
    ap.add_argument("--tile-rows", type=int, default=0, choices=[0, 8, 16, 32],
                    help="stencil tile height (default: chosen by the autotuner)")
    ap.add_argument("--cpu-iters", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--w-sweeps", type=int, default=0, metavar="R",
                    help="use the fixed-point w solver (eqs 38-40) with R sweeps instead of soft thresholding")
    ap.add_argument("--phi-solver", default="fft", choices=["fft", "aos"],
                    help="phi sub-problem solver: the FFT solve (eq 37) or AOS with constant A_l")
    ap.add_argument("--bc", default="periodic", choices=["periodic", "neumann"],
                    help="boundaries: periodic, or Neumann (mirror ghosts; the FFT solve then runs on the "
                         "2M x 2N mirror extension)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    ap.add_argument("--converge", action="store_true",
                    help="time-to-converge of the workload: r_k < 1e-4 after 20 iterations, cap 2000")
    ap.add_argument("--batch", type=int, default=0, metavar="COUNT",
                    help="time-to-converge of COUNT uneven instances, batched vs plain")
    ap.add_argument("--cnn", type=int, default=0, metavar="BATCH",
                    help="warm-start network throughput: inference on BATCH images, training on --train-batch")
    ap.add_argument("--train-batch", type=int, default=16)
    ap.add_argument("--warmstart", type=int, default=0, metavar="N",
                    help="time-to-solve of N held-out instances, plain vs CNN warm start")
    ap.add_argument("--cnn-size", type=int, default=512)
    ap.add_argument("--volume", type=int, default=0, metavar="S",
                    help="3-D solver throughput on an S^3 volume (S a power of two, 8..256)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the solver runs on a single "
              "device; see the sharding notes in the design document)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.converge:
        print(json.dumps(converge_bench(args.workload, 1e-4, 2000, 20, 10)), flush=True)
        return
    if args.batch:
        print(json.dumps(batch_bench(args.batch, 500, 1e-4, not args.no_cpu_baseline)), flush=True)
        return
    if args.volume:
        steps = args.steps if args.steps is not None else 20
        print(json.dumps(volume_bench(args.volume, steps, min(args.warmup, 3), not args.no_cpu_baseline)),
              flush=True)
        return
    if args.warmstart:
        print(json.dumps(warmstart_bench(args.warmstart)), flush=True)
        return
    if args.cnn:
        steps = args.steps if args.steps is not None else 20
        print(json.dumps(cnn_bench(args.cnn, args.cnn_size, steps, min(args.warmup, 5), args.train_batch,
                                   not args.no_cpu_baseline)), flush=True)
        return

    import torch
    from paper_2003_12693_amd import sr

    wl = dict(WORKLOADS[args.workload])
    if args.w_sweeps:
        wl["w_sweeps"] = args.w_sweeps
        wl["text"] += f"; fixed-point w solver, {args.w_sweeps} sweeps"
    if args.phi_solver == "aos":
        wl["phi_solver"] = "aos"
        wl["text"] += "; AOS phi solver, tau=0.04"
    if args.bc == "neumann":
        wl["bc"] = "neumann"
        wl["text"] += "; Neumann boundaries" + ("" if args.phi_solver == "aos" else " (DCT-II solve on the grid)")
    steps = args.steps if args.steps is not None else wl["default_steps"]
    M, N = wl["M"], wl["N"]
    f, phi0 = make_input(args.workload)
    if args.tile_rows:
        os.environ["SR_TILE_TH"] = str(args.tile_rows)
    s = sr.Solver(M, N, device="cuda:0", **params_kw(wl))
    ft = torch.from_numpy(f.astype(np.float32)).cuda()
    pt = torch.from_numpy(phi0.astype(np.float32)).cuda()
    s.set_image(ft, pt)
    tile_th = args.tile_rows or s.autotune(20)[0]
    s.prepare()   # every graph sr_step replays is instantiated before the timed region
    s.step(args.warmup)   # after the host-side graph set-up, so the GPU enters the timed region busy
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    rc, info = sr.sr_step(s.ctx, steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = max(e0.elapsed_time(e1), (t1 - t0) * 1e3)
    value = M * N * steps / 1e6 / (ms / 1e3)

    E, terms = s.energy()
    # per-kernel timing: further outer iterations from where the timed run ended,
    # launched without a graph, every iteration kernel with its own HIP events
    # (recorded at the kernel's start and end, on the solver's stream)
    prof = sr.sr_profile_kernels(s.ctx, args.profile_iters)
    if args.phi_solver == "aos":   # the phi solve is timed in the column-solve slot
        prof = {("aos_solve" if k == "col_fft_solve" else k): v for k, v in prof.items()
                if k not in ("row_fft_fwd", "row_fft_inv")}
    elif prof["row_fft_fwd"][1] == 0:   # the rhs fused into the forward row FFT
        prof = {("rhs_row_fft_fwd" if k == "rhs_repulsion" else k): v for k, v in prof.items()
                if k != "row_fft_fwd"}
    per_iter = {k: prof[k][1] / args.profile_iters for k in prof}      # launches per outer iteration
    per_iter_ms = {k: prof[k][0] * per_iter[k] for k in prof}
    dom = max(per_iter_ms, key=per_iter_ms.get)
    dom_ms = prof[dom][0]
    bytes_px = dict(BYTES_PER_PX, aos_solve=BYTES_PER_PX_AOS)
    if args.w_sweeps > 1:   # w_step launches average the sweeps and the full step
        bytes_px["w_step"] = (BYTES_PER_PX["w_step"] + BYTES_PER_PX_W_SWEEP * (args.w_sweeps - 1)) / args.w_sweeps
    alg_bytes = bytes_px[dom] * M * N
    achieved = alg_bytes / (dom_ms * 1e-3) / 1e9
    build_id = sr.sr_build_id()
    traffic = (None if args.w_sweeps or args.phi_solver != "fft" or args.bc != "periodic"
               else measured_traffic(args.workload, dom, tile_th, build_id))

    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes}
    if traffic is not None:   # bytes the counters saw move, over the same duration
        roof["achieved_by_counters"] = round(traffic / (dom_ms * 1e-3) / 1e9, 1)
        roof["frac_by_counters"] = round(roof["achieved_by_counters"] / HBM_PEAK_GBS, 4)
    out = {
        "metric": f"SB megapixel-iters/s at {M}^2" if M == N else f"SB megapixel-iters/s at {M}x{N}",
        "value": round(value, 2),
        "unit": "MPix-it/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["text"], "M": M, "N": N, "R": wl["R"], "S": wl["S"],
                   "tile_rows": None if "rhs_row_fft_fwd" in prof else tile_th,
                   "bytes_per_px_iter": sum(bytes_px[k] * per_iter[k] for k in prof),
                   "launches_per_iter": sum(per_iter.values()),
                   "w_solver": "fixed-point" if args.w_sweeps else "shrink", "w_sweeps": args.w_sweeps or None,
                   "phi_solver": args.phi_solver, "bc": args.bc},
        "roofline": roof,
        "kernels_ms": {k: round(v[0], 5) for k, v in prof.items()},
        "iteration_ms_sum_of_kernels": round(sum(per_iter_ms.values()), 5),
        "energy_after": E,
        "r_last": info.r_last,
        "build_id": build_id,
        "build_matches_tree": build_id == build_source_id(),
    }
    if not args.no_cpu_baseline:
        iters = args.cpu_iters if args.cpu_iters is not None else (5 if M * N <= 1 << 20 else 1)
        out["cpu_baseline"] = cpu_baseline(f, phi0, wl, iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
