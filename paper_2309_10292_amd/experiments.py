"""Measurement runs of the growth directions on one MI355X, each printing one
JSON record (and writing it to --out):

  precision  L=1024 cube, F=0.03, k=0.06, 200 steps, no noise: throughput of
             FP64 / FP32 / BF16 / FP16 storage (their errors against the FP64
             oracle are measured by the GPU tests).
  batched    256 independent simulations (F ~ U[0.01, 0.06], k ~ U[0.04,
             0.07], L ~ U{32, 48, ..., 192}), cube start, 500 steps, FP64:
             one persistent batched sweep (default and autotuned, graph
             replay) against the same simulations run one after another.
  small      the L=64 parity workload (FP64, 100 steps): eager launches
             against one captured HIP graph replayed. Its 8 MB of state stay
             in the caches, so this is launch and latency cost, not an HBM
             figure.
  surrogate  the 16-step surrogate trained on stencil trajectories at L=128
             and run with the stencil-fallback controller, against the plain
             FP64 stencil on the same GPU.

    python -m paper_2309_10292_amd.experiments precision|batched|small|surrogate [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _timed(torch, fn):
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1)


def precision(args):
    """Throughput of each storage type on the L=1024 workload (200 steps).
    Their errors against the FP64 oracle are measured by
    tests/test_gpu_precision.py."""
    import torch
    from paper_2309_10292_amd import gs
    from synth import workload
    p = workload("precision_l1024")
    L, n, side = p["L"], p["steps"], p["cube_side"]
    kw = {k: p[k] for k in ("Du", "Dv", "F", "k", "dt", "noise")}
    out = dict(experiment="precision", workload=f"periodic {L}^3, F={p['F']}, k={p['k']}, {n} steps, noise 0",
               storage={})
    for storage in args.storages.split(","):
        with gs.Sim(L, L, L, storage=storage, cube_side=side, **kw) as s:
            if args.tune:
                s.tune(reps=1)
            s.step(2)
            ms = _timed(torch, lambda: s.step(n))
            cfg = s.config()
            d = s.diagnostics(allow_nonfinite=True)
        bpc = {"f64": 32, "f32": 16, "bf16": 8, "f16": 8}[storage]
        rec = dict(gcells=round(L ** 3 * n / (ms * 1e-3) / 1e9, 2), ms_per_step=round(ms / n, 4), launch=cfg,
                   algorithmic_gbs=round(bpc * L ** 3 * n / (ms * 1e-3) / 1e9, 1),
                   sum_u=d["sum_u"], sum_v=d["sum_v"], nonfinite=d["nonfinite"])
        out["storage"][storage] = rec
        print(json.dumps({storage: rec}), flush=True)
    return out


def small(args):
    """The L=64 parity workload: 100 FP64 steps launched one by one, and
    the same steps replayed from one captured HIP graph (median of 20 runs
    each, after a warm-up)."""
    import torch
    from paper_2309_10292_amd import gs
    from synth import workload
    p = workload("small_l64")
    L, n, side = p["L"], p["steps"], p["cube_side"]
    kw = {k: p[k] for k in ("Du", "Dv", "F", "k", "dt", "noise")}
    out = dict(experiment="small", workload=f"periodic {L}^3, FP64, {n} steps, noise 0", steps=n)
    with gs.Sim(L, L, L, storage="f64", cube_side=side, **kw) as s:
        if args.tune:
            s.tune(reps=3)
        out["launch"] = s.config()
        launches = -(-n // out["launch"]["tblock"])
        for mode, fn in (("eager", lambda: s.step(n)), ("graph", lambda: s.step_graph(n))):
            fn()
            t = sorted(_timed(torch, fn) for _ in range(20))
            ms = t[len(t) // 2]
            out[mode] = dict(ms=round(ms, 4), us_per_step=round(ms * 1e3 / n, 2),
                             gcells=round(L ** 3 * n / (ms * 1e-3) / 1e9, 2))
        out["launches_per_run"] = launches
        print(json.dumps(out), flush=True)
    return out


def batched(args):
    import torch
    from paper_2309_10292_amd import gs
    from synth import batch_sweep
    sims = batch_sweep(args.n_sims)
    n = args.steps
    base = dict(Du=0.2, Dv=0.1, dt=1.0, cube_side=12, storage="f64")
    cells = sum(s["L"] ** 3 for s in sims)
    out = dict(experiment="batched", n_sims=len(sims), steps=n, cells=cells,
               sizes=sorted({s["L"] for s in sims}))
    with gs.Batch(sims, **base) as b:
        b.step(3)  # warm-up (lists uploaded at init)
        ms = _timed(torch, lambda: b.step(n))
        out["batch_default"] = dict(ms=round(ms, 2), gcells=round(cells * n / (ms * 1e-3) / 1e9, 2),
                                    config=b.config(0))
        t0 = time.perf_counter()
        table = b.tune(reps=2)
        out["tune_seconds"] = round(time.perf_counter() - t0, 2)
        out["tune_table"] = table
        b.step_graph(n)  # capture
        ms = _timed(torch, lambda: b.step_graph(n))
        out["batch_tuned_graph"] = dict(ms=round(ms, 2), gcells=round(cells * n / (ms * 1e-3) / 1e9, 2))
        ms = _timed(torch, lambda: b.step(n))
        out["batch_tuned"] = dict(ms=round(ms, 2), gcells=round(cells * n / (ms * 1e-3) / 1e9, 2))
    # the same simulations, each alone with the single-grid path: with the
    # library defaults, and with the configuration gs_tune picks for that size
    tuned = {}
    for L in sorted({s["L"] for s in sims}):
        with gs.Sim(L, L, L, F=0.03, k=0.055, **base) as one:
            cfg, _ = one.tune(reps=2)
            tuned[L] = cfg
    out["alone_tuned_configs"] = {str(L): c for L, c in tuned.items()}
    for label, use_tuned in (("each_alone_default", False), ("each_alone_tuned", True)):
        total = 0.0
        for s in sims:
            with gs.Sim(s["L"], s["L"], s["L"], F=s["F"], k=s["k"], **base) as one:
                if use_tuned:
                    c = tuned[s["L"]]
                    one.set_config(c["tile"], c["tblock"], c["zchunk"])
                one.step(2)
                total += _timed(torch, lambda: one.step_graph(n) if use_tuned else one.step(n))
        out[label] = dict(ms=round(total, 2), gcells=round(cells * n / (total * 1e-3) / 1e9, 2))
    out["speedup_batched_vs_alone_tuned"] = round(out["each_alone_tuned"]["ms"] / out["batch_tuned_graph"]["ms"], 2)
    out["speedup_batched_vs_alone_default"] = round(out["each_alone_default"]["ms"] / out["batch_tuned_graph"]["ms"], 2)
    return out


def surrogate(args):
    """Train on args.trajectories stencil trajectories at L (chunks of
    args.chunk trajectories generated by the batched FP32 stencil, pairs 16
    steps apart), then run the controller on held-out trajectories."""
    import torch
    from paper_2309_10292_amd import gs
    from paper_2309_10292_amd.surrogate import JUMP, Surrogate, generate_pairs, run_controlled, train
    from synth import random_blobs, surrogate_init
    L = args.L
    out = dict(experiment="surrogate", L=L, trajectories=args.trajectories, steps_per_trajectory=args.traj_steps,
               pairs_per_trajectory=len(range(args.warm, args.traj_steps - JUMP + 1, args.pair_every)),
               batch=args.batch, lr=args.lr)
    blobs = random_blobs(args.trajectories + args.held_out, L, seed=230910292, side_range=(6, 24))
    train_blobs, test_blobs = blobs[:args.trajectories], blobs[args.trajectories:]
    hist, curve = [], []
    t_gen = t_train = 0.0
    with Surrogate(L, L, L, max_batch=args.batch, params=surrogate_init(0)) as m:
        for c0 in range(0, len(train_blobs), args.chunk):
            t0 = time.perf_counter()
            data = generate_pairs(L, train_blobs[c0:c0 + args.chunk], args.traj_steps, args.pair_every, warm=args.warm)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            iters = max(1, int(round(data[0].shape[0] * args.epochs / args.batch)))
            frac = c0 / len(train_blobs)
            lr = args.lr * (0.1 ** frac)  # decays tenfold over the run
            hist += train(m, data, iters, args.batch, lr=lr, seed=c0)
            torch.cuda.synchronize()
            t_gen += t1 - t0
            t_train += time.perf_counter() - t1
            last_data = data
            del data
            curve.append((len(hist), float(np.mean(hist[-20:]))))
            print(json.dumps(dict(chunk=c0 // args.chunk, iters=len(hist), loss=float(np.mean(hist[-20:])),
                                  gen_s=round(t_gen, 1), train_s=round(t_train, 1))), flush=True)
        out["train"] = dict(iters=len(hist), loss_first=float(np.mean(hist[:20])), loss_last=float(np.mean(hist[-50:])),
                            generate_seconds=round(t_gen, 1), train_seconds=round(t_train, 1), curve=curve)
        # one jump on pairs of the last training chunk: network against
        # persistence (no change), to tell under- from over-fitting
        u, v, ut, vt, Fd, kd = last_data
        pu_, pv_ = torch.empty_like(u[0]), torch.empty_like(v[0])
        fit = []
        for i in range(0, u.shape[0], max(1, u.shape[0] // 16)):
            m.predict(u[i], v[i], float(Fd[i]), float(kd[i]), pu_, pv_)
            n2 = 2 * u[i].numel()
            fit.append(dict(net=((gs.sqdiff(pu_, ut[i]) + gs.sqdiff(pv_, vt[i])) / n2) ** 0.5,
                            persistence=((gs.sqdiff(u[i], ut[i]) + gs.sqdiff(v[i], vt[i])) / n2) ** 0.5))
        out["train"]["one_jump_rms_last_chunk"] = dict(net_mean=float(np.mean([x["net"] for x in fit])),
                                                      persistence_mean=float(np.mean([x["persistence"] for x in fit])))
        del last_data
        params = m.params()
        if args.save:
            np.save(args.save, params)
        # timing of one jump against 16 FP64 stencil steps (L^3, one sample)
        b = test_blobs[0]
        with gs.Sim(L, L, L, init="none", u0=np.ones((L,) * 3), v0=np.zeros((L,) * 3), F=b["F"], k=b["k"]) as s:
            s.fill_cube(b["x0"], b["y0"], b["z0"], b["side"])
            s.step(args.warm)
            s.tune(reps=2)  # the stencil side gets its autotuned configuration
            u, v, _ = s.current()
            pu, pv = torch.empty_like(u), torch.empty_like(v)
            m.predict(u, v, b["F"], b["k"], pu, pv)
            ms_jump = _timed(torch, lambda: [m.predict(u, v, b["F"], b["k"], pu, pv) for _ in range(10)]) / 10
            s.step(JUMP)
            ms_stencil = _timed(torch, lambda: s.step(10 * JUMP)) / 10
            cfg = s.config()
        out["timing"] = dict(ms_surrogate_jump=round(ms_jump, 4), ms_stencil_16_steps_f64=round(ms_stencil, 4),
                             stencil_config=cfg, surrogate_cell_steps_per_s=round(L ** 3 * JUMP / (ms_jump * 1e-3) / 1e9, 2),
                             stencil_cell_steps_per_s=round(L ** 3 * JUMP / (ms_stencil * 1e-3) / 1e9, 2))
        # one jump from stencil states of held-out trajectories: the network
        # against persistence (no change over 16 steps), both against the
        # FP64 stencil
        one = []
        for b in test_blobs:
            with gs.Sim(L, L, L, init="none", u0=np.ones((L,) * 3), v0=np.zeros((L,) * 3), F=b["F"], k=b["k"]) as s:
                s.fill_cube(b["x0"], b["y0"], b["z0"], b["side"])
                s.step(args.warm)
                for j in range(4):
                    u, v, _ = s.current()
                    u0, v0 = u.clone(), v.clone()
                    m.predict(u0, v0, b["F"], b["k"], pu, pv)
                    s.step(JUMP)
                    u1, v1, _ = s.current()
                    n2 = 2 * u1.numel()
                    one.append(dict(net=((gs.sqdiff(pu, u1) + gs.sqdiff(pv, v1)) / n2) ** 0.5,
                                    persistence=((gs.sqdiff(u0, u1) + gs.sqdiff(v0, v1)) / n2) ** 0.5))
        out["one_jump_rms"] = dict(net_mean=float(np.mean([x["net"] for x in one])),
                                   persistence_mean=float(np.mean([x["persistence"] for x in one])), samples=one)
        # controller on held-out trajectories, with the BF16-storage stencil on
        # the same trajectory as a second reference point
        runs = []
        for b in test_blobs:
            with gs.Sim(L, L, L, init="none", u0=np.ones((L,) * 3), v0=np.zeros((L,) * 3), F=b["F"], k=b["k"]) as s:
                s.fill_cube(b["x0"], b["y0"], b["z0"], b["side"])
                s.step(args.warm)
                r = run_controlled(m, s, b["F"], b["k"], jumps=args.jumps, check_every=4, tol=args.tol)
                ut, vt, _ = s.current()
                # the same trajectory with the plain stencil
                with gs.Sim(L, L, L, init="none", u0=np.ones((L,) * 3), v0=np.zeros((L,) * 3), F=b["F"], k=b["k"]) as ref:
                    ref.fill_cube(b["x0"], b["y0"], b["z0"], b["side"])
                    ref.step(args.warm + args.jumps * JUMP)
                    ur, vr, _ = ref.current()
                    rms_end = ((gs.sqdiff(ut, ur) + gs.sqdiff(vt, vr)) / (2 * ur.numel())) ** 0.5
                    u16 = np.ones((L,) * 3)
                    with gs.Sim(L, L, L, storage="bf16", init="none", u0=u16, v0=np.zeros((L,) * 3), F=b["F"],
                                k=b["k"]) as lo:
                        lo.fill_cube(b["x0"], b["y0"], b["z0"], b["side"])
                        lo.step(args.warm + args.jumps * JUMP)
                        ul, vl = lo.read()
                        uh, vh = ref.read()
                        rms_bf16 = float(np.sqrt((np.sum((ul - uh) ** 2) + np.sum((vl - vh) ** 2)) / (2 * uh.size)))
                runs.append(dict(F=b["F"], k=b["k"], checks=r["checks"], fallbacks=r["fallbacks"],
                                 rms_at_checks=[round(x, 6) for x in r["rms"]], rms_end_vs_stencil=rms_end,
                                 rms_end_bf16_stencil=rms_bf16, seconds=round(r["seconds"], 4)))
        out["controller"] = dict(tol=args.tol, check_every=4, jumps=args.jumps, runs=runs,
                                 fallback_rate=sum(x["fallbacks"] for x in runs) / max(1, sum(x["checks"] for x in runs)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["precision", "batched", "small", "surrogate"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--storages", default="f64,f32,bf16,f16")
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--n-sims", type=int, default=256)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--trajectories", type=int, default=2000)
    ap.add_argument("--held-out", type=int, default=4)
    ap.add_argument("--chunk", type=int, default=40)
    ap.add_argument("--traj-steps", type=int, default=1024)
    ap.add_argument("--pair-every", type=int, default=64)
    ap.add_argument("--warm", type=int, default=64)
    ap.add_argument("--epochs", type=float, default=1.0)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--jumps", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--save", default=None, help="save the trained parameters (.npy)")
    a = ap.parse_args(argv)
    res = {"precision": precision, "batched": batched, "small": small, "surrogate": surrogate}[a.which](a)
    s = json.dumps(res)
    print(s)
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            f.write(s + "\n")


if __name__ == "__main__":
    main()
