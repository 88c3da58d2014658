"""Learned warm start for the SR solver: data generation, training and
evaluation (launch and orchestration only; every numerical step runs in the
library's kernels, through the sr_* and cnn_* entry points).

The network (include/cnn.h) maps (f, g, phi^0) to a predicted level set
phi-hat.  It is trained only on solutions of the plain solver: every training
instance is solved by sr_solve_batch, and the target is the solved level set
clipped to +-CLIP (beyond the band the model's energy densities are constant,
so clipping loses nothing the energy sees).

The reference solve is the plain solver run for a fixed budget of K_PLAIN
iterations.  On these images the whole-grid relative-change rule never fires
(far-field drift keeps it near 3e-4), and the energy has no lasting minimum
at the objects: the contour shrinks at about 0.01 px per iteration, rests on
metastable plateaus and eventually passes through the edges.  A fixed budget
is the reproducible definition of "the plain solve".

Split Bregman always refines the prediction and judges the result: the warm
solve starts Algorithm 1 from phi-hat moved outward by MARGIN px (sr_set_image
with it as the initial level set: w = grad+ phi, b = 0; the margin is folded
into the head bias) and iterates until its energy reaches the plain solve's
final energy E_plain to within E_TOL (relative).  Chunks of iterations shrink
to single iterations near the target; the energy falls in bursts of up to
~1e-3 per iteration there, wider than the window, so when the last iteration
steps over it the crossing is resolved on the segment between the last two
iterates (the energy depends on phi alone and is continuous in it:
bisection finds a phi whose energy lies inside the window).  Every accepted
run therefore ends within E_TOL of the plain energy.  A start whose energy
is already below that (a prediction past the plain solve, which the
refinement cannot judge), or that does not reach it within K_PLAIN
iterations, is rejected and the plain solve used instead; a rejected start
is charged both.

    python -m paper_2003_12693_amd.warmstart train --n-train 2048 --epochs 40 \
        --weights W.npy --report train.json
    python -m paper_2003_12693_amd.warmstart eval --weights W.npy --n-eval 64 --report eval.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import cnn, sr, synth

SIZE = 512
CLIP = 8.0
E_TOL = 1e-4
TRAIN_SEED0 = 5_000_000
EVAL_SEED0 = 6_000_000
K_PLAIN = 10000
MARGIN = 2.0
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_512.npy")


def solver_kw(tol=0.0):
    """The paper's two-circles weights with eps = 1.5, R = 3, d = 5, S = 3;
    no early stop by default (tol = 0: the fixed budget decides)."""
    return dict(gamma=4.0, alpha=4.0, beta=0.2, mu=8.0, tau=0.1, eps=1.5, band_l=1.0, d=5.0, R=3,
                sigma=1.5, rho=1000.0, s_exp=2, S=3, tol_inner=0.0, zero_tol=1e-3,
                tol_outer=tol, min_iter=20, check_every=10)


def instance(seed, size=SIZE):
    """Ellipse images at half the scale of the 1024^2 workload: 3 ellipses with
    semi-axes 15-60 px, 2-6 px gaps, bias field and noise; rectangle phi^0."""
    f, phi0 = synth.ellipses(size, size, seed=seed, n_shapes=3, axis_lo=15.0, axis_hi=60.0)
    return f.astype(np.float32), phi0.astype(np.float32)


def _gen(seed):
    return instance(seed)


def make_instances(seeds, workers=8):
    """Host-side instance generation; the worker pool forks, so call this
    before the process first touches the GPU."""
    if workers > 1 and len(seeds) > 16:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            return pool.map(_gen, seeds, chunksize=8)
    return [instance(s) for s in seeds]


# ---------------------------------------------------------------------------
# data
# ---------------------------------------------------------------------------
def generate(insts, cap=K_PLAIN, chunk=128, log=print):
    """Solve every instance (f, phi0) with the plain batched solver.  Returns
    GPU tensors F, G, PHI0 [n, S, S] and TARGET (converged phi) plus
    per-instance iteration counts, energies and statuses."""
    import torch
    kw = solver_kw()
    params = sr.sr_params_default(**kw)
    n = len(insts)
    F = torch.empty((n, SIZE, SIZE), dtype=torch.float32, device="cuda")
    G = torch.empty_like(F)
    P0 = torch.empty_like(F)
    T = torch.empty_like(F)
    iters, energy, status = np.zeros(n, np.int64), np.zeros(n), np.zeros(n, np.int64)
    ctx = sr.Solver(SIZE, SIZE, **kw)
    t_solve = 0.0
    for c0 in range(0, n, chunk):
        part = insts[c0:c0 + chunk]
        for i, (f, p) in enumerate(part):
            F[c0 + i].copy_(torch.from_numpy(f))
            P0[c0 + i].copy_(torch.from_numpy(p))
            sr.sr_edge_map(ctx.ctx, F[c0 + i], G[c0 + i])
        items = [dict(f=F[c0 + i], phi0=P0[c0 + i], max_iter=cap, params=params) for i in range(len(part))]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = sr.solve_batch(items)
        torch.cuda.synchronize()
        t_solve += time.perf_counter() - t0
        for i, r in enumerate(res):
            T[c0 + i].copy_(r["phi"])
            iters[c0 + i], energy[c0 + i], status[c0 + i] = r["iters"], r["energy"], r["status"]
        log(f"  solved {c0 + len(part)}/{n}: mean iters {iters[:c0 + len(part)].mean():.0f}, "
            f"not converged {int((status[:c0 + len(part)] != 0).sum())}, batched solve {t_solve:.1f} s")
    ctx.close()
    return F, G, P0, T, iters, energy, status, t_solve


# ---------------------------------------------------------------------------
# training
# ---------------------------------------------------------------------------
def _augment(x, k):
    """One of the 8 symmetries of the square (the solver and the rectangle
    initialisation are equivariant under them)."""
    import torch
    if k & 4:
        x = x.transpose(-1, -2)
    if k & 1:
        x = torch.flip(x, (-1,))
    if k & 2:
        x = torch.flip(x, (-2,))
    return x.contiguous()


def train(F, G, P0, T, epochs, batch=16, lr=1e-3, seed=0, val=0.1, log=print):
    import torch
    n = F.shape[0]
    nval = max(1, int(round(val * n)))
    idx = np.random.default_rng(seed).permutation(n)
    vidx, tidx = idx[:nval], idx[nval:]
    net = cnn.Network(batch, SIZE, SIZE, cnn.he_init(seed))
    rng = np.random.default_rng(seed + 1)
    steps_per_epoch = len(tidx) // batch
    total = epochs * steps_per_epoch
    hist = []
    t0 = time.perf_counter()
    step = 0

    def val_loss():
        tot, cnt = 0.0, 0
        for b0 in range(0, nval, batch):
            b = torch.from_numpy(vidx[b0:b0 + batch]).cuda()
            m = len(b)
            net.forward(F[b].contiguous(), G[b].contiguous(), P0[b].contiguous(), CLIP, want_output=False)
            tot += net.backward(T[b].contiguous(), CLIP)[0] * m
            cnt += m
        return tot / cnt

    for ep in range(epochs):
        perm = rng.permutation(tidx)
        run = 0.0
        for s in range(steps_per_epoch):
            b = torch.from_numpy(perm[s * batch:(s + 1) * batch]).cuda()
            k = int(rng.integers(8))
            f, g, p, t = (_augment(X[b], k) for X in (F, G, P0, T))
            net.forward(f, g, p, CLIP, want_output=False)
            want = (s % 20) == 0
            loss = cnn.cnn_backward(net.ctx, t, CLIP, want_loss=want)
            # cosine learning-rate decay
            net.adam_step(lr=lr * 0.5 * (1.0 + np.cos(np.pi * step / total)))
            step += 1
            if want:
                run = loss
        vl = val_loss()
        hist.append({"epoch": ep + 1, "train_loss": run, "val_loss": vl, "s": time.perf_counter() - t0})
        log(f"  epoch {ep + 1}/{epochs}: train {run:.5f} val {vl:.5f} ({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    params = net.get_params().cpu().numpy()
    return params, hist, time.perf_counter() - t0, steps_per_epoch * batch


# ---------------------------------------------------------------------------
# evaluation
# ---------------------------------------------------------------------------
def warm_solve(s, net, f, g, phi0, k_plain, E_plain, max_chunk=200):
    """Refine the network's prediction with Split Bregman until the energy is
    within E_TOL of E_plain.  Chunks of iterations are sized from the observed
    energy rate; a chunk that jumps below the window is undone (state
    snapshot) and retried at half length, down to single iterations.
    Returns (accepted, iterations, seconds, energy, reason)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start = net.forward(f[None], g[None], phi0[None], CLIP)[0]
    s.set_image(f, start)
    tol = E_TOL * abs(E_plain)
    phi_s, w_s, b_s = s._empty(s.M, s.N), s._empty(2, s.M, s.N), s._empty(2, s.M, s.N)
    E = s.energy()[0]
    k, rate, cap, chunk = 0, None, max_chunk, 1
    while True:
        if abs(E - E_plain) <= tol:
            torch.cuda.synchronize()
            return True, k, time.perf_counter() - t0, E, "energy reached"
        if E < E_plain - tol:
            return False, k, time.perf_counter() - t0, E, "start below the plain energy"
        if k >= k_plain:
            return False, k, time.perf_counter() - t0, E, "budget spent"
        if rate is None or rate <= 0:                # no progress measured yet: grow the chunk
            chunk = 1 if rate is None else min(cap, 2 * chunk)
        else:
            chunk = int(max(1, min(cap, 0.5 * (E - E_plain) / rate)))
        chunk = min(chunk, k_plain - k)
        kk = sr.sr_get_state(s.ctx, phi_s, w_s, b_s)
        info = s.step(chunk)
        done = int(info["iters_done"])
        E_new = s.energy()[0]
        if E_new < E_plain - tol and done > 1:
            s.set_state(phi_s, w_s, b_s, kk)        # undo, retry shorter
            cap = max(1, done // 2)
            continue
        rate = (E - E_new) / max(done, 1)
        if E_new < E_plain - tol:                    # one iteration stepped over the window
            E_x = resolve_crossing(s, phi_s, w_s, b_s, kk, E_plain, tol)
            torch.cuda.synchronize()
            return True, k + done, time.perf_counter() - t0, E_x, "crossing resolved on the last step"
        E, k = E_new, k + done


def resolve_crossing(s, phi_prev, w_prev, b_prev, k_prev, E_plain, tol, max_halvings=40):
    """The last iteration took the energy from above the window
    |E - E_plain| <= tol to below it.  The energy is a continuous function
    of phi alone (eqs 7-10), so on the segment phi_a = phi_prev + a (phi_new -
    phi_prev), a in [0, 1], it crosses the window; bisection on a (energies
    by the library, sr_energy of the interpolated phi) finds a point inside.
    The solver is left at that phi (with the previous w, b).  Returns its
    energy."""
    phi_new = s.phi()
    lo, hi = 0.0, 1.0
    E = None
    for _ in range(max_halvings):
        a = 0.5 * (lo + hi)
        phi_a = (phi_prev + a * (phi_new - phi_prev)).contiguous()
        s.set_state(phi_a, w_prev, b_prev, k_prev + 1)
        E = s.energy()[0]
        if abs(E - E_plain) <= tol:
            return E
        if E > E_plain:
            lo = a
        else:
            hi = a
    return E


def evaluate(params, seeds, k_plain=K_PLAIN, log=print):
    """Plain solve (k_plain iterations) and warm solve of every seed."""
    import torch
    s = sr.Solver(SIZE, SIZE, **solver_kw())
    p = np.array(params, dtype=np.float32, copy=True)
    p[-1] -= MARGIN / CLIP          # head bias: phi-hat - MARGIN
    net = cnn.Network(1, SIZE, SIZE, p)
    rows = []
    for sd in seeds:
        f, p0 = instance(sd)
        ft, pt = torch.from_numpy(f).cuda(), torch.from_numpy(p0).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_image(ft, pt)
        s.step(k_plain)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        E_plain = s.energy()[0]
        g = s.g()
        ok, it_w, t_w, E_w, why = warm_solve(s, net, ft, g, pt, k_plain, E_plain)
        cost_it = it_w if ok else it_w + k_plain
        cost_t = t_w if ok else t_w + t_plain
        rows.append({"seed": sd, "iters_plain": k_plain, "iters_warm": it_w, "accepted": ok, "reason": why,
                     "E_plain": E_plain, "E_warm": E_w, "rel_dE": (E_w - E_plain) / abs(E_plain),
                     "t_plain": t_plain, "t_warm": t_w, "cost_iters": cost_it, "cost_s": cost_t})
        log(f"  seed {sd}: plain {k_plain} it {t_plain * 1e3:.0f} ms E {E_plain:.6g}; warm {it_w} it "
            f"{t_w * 1e3:.0f} ms E {E_w:.6g} ({why})")
    s.close()
    net.close()
    ip = np.array([r["iters_plain"] for r in rows], float)
    ic = np.array([r["cost_iters"] for r in rows], float)
    tp = np.array([r["t_plain"] for r in rows])
    tc = np.array([r["cost_s"] for r in rows])
    acc = np.array([r["accepted"] for r in rows])
    summary = {
        "instances": len(rows), "accepted": int(acc.sum()), "fallback_rate": float(1 - acc.mean()),
        "k_plain": k_plain, "e_tol": E_TOL, "margin_px": MARGIN,
        "mean_iters_warm_accepted": float(np.mean([r["iters_warm"] for r in rows if r["accepted"]] or [0])),
        "within_window": int(sum(1 for r in rows if r["accepted"] and abs(r["rel_dE"]) <= E_TOL)),
        "resolved_on_last_step": int(sum(1 for r in rows if r["reason"] == "crossing resolved on the last step")),
        "max_abs_rel_dE_accepted": float(max([abs(r["rel_dE"]) for r in rows if r["accepted"]] or [0])),
        "mean_iters_warm_incl_fallback": float(ic.mean()),
        "iters_saved_frac": float(1 - ic.sum() / ip.sum()),
        "mean_s_plain": float(tp.mean()), "mean_s_warm_incl_inference_and_fallback": float(tc.mean()),
        "time_saved_frac": float(1 - tc.sum() / tp.sum()),
    }
    return summary, rows


def evaluate_many(params, seeds, k_plain=K_PLAIN, chunk=128, log=print):
    """Iterations saved and fallback rate over many held-out instances: the
    plain solves run batched (sr_solve_batch gives every instance bitwise the
    result of its single solve), each warm start is refined on its own."""
    import torch
    kw = solver_kw()
    params_sr = sr.sr_params_default(**kw)
    s = sr.Solver(SIZE, SIZE, **kw)
    p = np.array(params, dtype=np.float32, copy=True)
    p[-1] -= MARGIN / CLIP
    net = cnn.Network(1, SIZE, SIZE, p)
    rows = []
    t_batch = 0.0
    for c0 in range(0, len(seeds), chunk):
        part = seeds[c0:c0 + chunk]
        insts = [instance(sd) for sd in part]
        ft = [torch.from_numpy(f).cuda() for f, _ in insts]
        pt = [torch.from_numpy(q).cuda() for _, q in insts]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, res = sr.solve_batch([dict(f=a, phi0=b, max_iter=k_plain, params=params_sr) for a, b in zip(ft, pt)])
        torch.cuda.synchronize()
        t_batch += time.perf_counter() - t0
        for sd, a, b, r in zip(part, ft, pt, res):
            s.set_image(a, b)                   # g for the network input
            ok, it_w, t_w, E_w, why = warm_solve(s, net, a, s.g(), b, k_plain, r["energy"])
            rows.append({"seed": sd, "accepted": ok, "iters_warm": it_w, "reason": why, "E_plain": r["energy"],
                         "E_warm": E_w, "rel_dE": None if E_w is None else (E_w - r["energy"]) / abs(r["energy"]),
                         "t_warm": t_w})
        acc = sum(1 for r in rows if r["accepted"])
        log(f"  {len(rows)} instances: {acc} accepted, mean warm iterations "
            f"{np.mean([r['iters_warm'] for r in rows if r['accepted']] or [0]):.0f}")
    s.close()
    net.close()
    acc = [r for r in rows if r["accepted"]]
    cost = [r["iters_warm"] if r["accepted"] else r["iters_warm"] + k_plain for r in rows]
    summary = {
        "instances": len(rows), "accepted": len(acc), "fallback_rate": 1 - len(acc) / len(rows),
        "k_plain": k_plain, "e_tol": E_TOL, "margin_px": MARGIN,
        "mean_iters_warm_accepted": float(np.mean([r["iters_warm"] for r in acc] or [0])),
        "max_iters_warm_accepted": int(max([r["iters_warm"] for r in acc] or [0])),
        "within_window": sum(1 for r in acc if abs(r["rel_dE"]) <= E_TOL),
        "resolved_on_last_step": sum(1 for r in rows if r["reason"] == "crossing resolved on the last step"),
        "max_abs_rel_dE_accepted": float(max([abs(r["rel_dE"]) for r in acc] or [0])),
        "iters_saved_frac": float(1 - np.sum(cost) / (k_plain * len(rows))),
        "plain_batched_s_per_instance": t_batch / len(rows),
        "mean_warm_s_incl_inference": float(np.mean([r["t_warm"] for r in rows])),
        "reasons": {k: sum(1 for r in rows if r["reason"] == k) for k in sorted({r["reason"] for r in rows})},
    }
    return summary, rows


# ---------------------------------------------------------------------------
def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--n-train", type=int, default=2048)
    t.add_argument("--epochs", type=int, default=40)
    t.add_argument("--batch", type=int, default=16)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--n-eval", type=int, default=32)
    t.add_argument("--weights", default=WEIGHTS)
    t.add_argument("--report", default=None)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--n-eval", type=int, default=32)
    e.add_argument("--n-eval-many", type=int, default=0,
                   help="also: iterations saved / fallback rate over this many held-out seeds (plain solves batched)")
    e.add_argument("--report", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    report = {}
    if a.cmd == "train":
        log(f"generating {a.n_train} training instances ({SIZE}^2); solving them with the plain batched solver")
        insts = make_instances(list(range(TRAIN_SEED0, TRAIN_SEED0 + a.n_train)))
        F, G, P0, T, iters, energy, status, t_gen = generate(insts, log=log)
        del insts
        report["data"] = {"instances": a.n_train, "size": SIZE, "mean_iters": float(iters.mean()),
                          "not_converged": int((status != 0).sum()), "batched_solve_s": t_gen}
        log("training")
        params, hist, t_train, per_epoch = train(F, G, P0, T, a.epochs, a.batch, a.lr, log=log)
        report["training"] = {"epochs": a.epochs, "batch": a.batch, "lr": a.lr, "images_per_epoch": per_epoch,
                              "seconds": t_train, "history": hist}
        os.makedirs(os.path.dirname(os.path.abspath(a.weights)), exist_ok=True)
        np.save(a.weights, params)
        del F, G, P0, T
    else:
        params = np.load(a.weights)
    log(f"evaluating on {a.n_eval} held-out instances")
    summary, rows = evaluate(params, list(range(EVAL_SEED0, EVAL_SEED0 + a.n_eval)), log=log)
    report["eval"] = summary
    report["eval_rows"] = rows
    log(json.dumps(summary))
    if a.cmd == "eval" and a.n_eval_many:
        log(f"evaluating iterations saved on {a.n_eval_many} held-out instances")
        many, mrows = evaluate_many(params, list(range(EVAL_SEED0, EVAL_SEED0 + a.n_eval_many)), log=log)
        report["eval_many"] = many
        report["eval_many_rows"] = mrows
        log(json.dumps(many))
    if a.report:
        with open(a.report, "w") as fh:
            json.dump(report, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
