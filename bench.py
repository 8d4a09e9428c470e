#!/usr/bin/env python3
"""Throughput of the fused Gray-Scott step on one MI355X.

Workload (default): one GPU's weak-scaling share at L=512 (periodic 512^3
cells), Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1, noise 1e-7 (Philox-keyed),
cube initial state, FP64 storage. A "step" is one time step of the whole
grid: neighbour gather, Laplacian, reaction/feed/kill, noise, Euler update
and the ping-pong; the default launch fuses three steps per pass over HBM.
Inputs are resident in HBM before timing starts.

Prints ONE JSON line: metric/value (G cell-updates/s), roofline of the step
kernel (algorithmic bytes per launch, 32 B per cell-update in FP64, over the
average launch time from HIP events on the kernel's stream; the measured HBM
bytes per launch when a counter profile of the current kernel source exists),
the FP32/BF16/FP16 storage variants at the same workload, and the CPU oracle
timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
BYTES_PER_CELL = {"f64": 32, "f32": 16, "bf16": 8, "f16": 8}  # read u,v + write u,v once per step
# Vector issue peak of MI355X: 256 CUs x 4 SIMDs, one wave64 instruction per
# SIMD every 4 cycles (64 lanes) at 2.4 GHz = 39.3 T lane-instructions/s.
VALU_PEAK_TOPS = 256 * 4 * 64 / 4 * 2.4e9 / 1e12
# Vector instructions the method itself needs per FP64 cell-update: 36 FP64
# operations (two Laplacians with the exact division by 6, the reaction, the
# Euler update) and, with noise, 12 more (a Philox4x32-10 block per 4 cells:
# 10 rounds of two 32x32->64-bit products and two three-input XORs, then the
# word's conversion and the fused noise term).


def alu_ops_per_cell_update(storage, noise):
    return 36 + (12 if noise else 0) if storage == "f64" else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f64", choices=list(BYTES_PER_CELL))
    ap.add_argument("--L", type=int, default=512)
    ap.add_argument("--tile", type=int, default=0, help="0 = library choice")
    ap.add_argument("--tblock", type=int, default=0, help="fused steps per sweep, 0 = library choice")
    ap.add_argument("--zchunk", type=int, default=0, help="planes per workgroup chunk, 0 = library choice")
    ap.add_argument("--tune", action="store_true", help="autotune the launch configuration first")
    ap.add_argument("--variants", default="f32,bf16,f16", help="other storage types to time, or 'none'")
    ap.add_argument("--variant-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the oracle sample")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "traffic.json"))
    return ap.parse_args()


def time_steps(torch, sim, steps, warmup):
    """Times `steps` steps with HIP events on the stream the library launches
    on (torch's current stream, bound at init). Returns (ms per step, ms per
    launch of the full-depth sweeps, launches timed)."""
    cfg = sim.config()
    T = cfg["tblock"]
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    full = (steps // T) * T
    ev[0].record(st)
    sim.step(full)
    ev[1].record(st)
    sim.step(steps - full)
    ev[2].record(st)
    ev[2].synchronize()
    torch.cuda.synchronize()
    total = ev[0].elapsed_time(ev[2])
    per_launch = ev[0].elapsed_time(ev[1]) / max(1, full // T)
    return total / steps, per_launch, full // T


KERNEL_SOURCES = ["paper_2309_10292_amd/csrc/gs_tblock.hip", "paper_2309_10292_amd/csrc/gs_device.hpp"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(path, kernel_key):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), or
    None when there is no measurement or the kernel sources changed since."""
    try:
        with open(path) as f:
            t = json.load(f).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not t or t.get("source_sha256") != kernel_source_hash():
        return None
    return t["bytes"]


def cpu_baseline(L, p, budget_s):
    """The FP64 oracle on the host cores: whole-grid steps of the same
    workload until the time budget is used (at least one step)."""
    from oracle import oracle as O
    threads = O.max_threads()
    u, v = O.init_cube(L=L)
    done, t0 = 0, time.perf_counter()
    while True:
        u, v = O.run(u, v, 1, step0=done, **p)
        done += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return dict(value=round(L ** 3 * done / el / 1e9, 4), unit="Gcell-updates/s", cores=threads, kind="oracle",
                cpu_model=model,
                sample=f"{done} whole-grid FP64 steps of the {L}^3 noisy workload, {el:.1f} s on {threads} threads")


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {a.gpus} is not supported "
              "(the step runs on one MI355X; multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2309_10292_amd import gs
    from synth import workload
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    gs.load()
    wl = workload("weak_share_l512")
    L = a.L
    p = {k: wl[k] for k in ("Du", "Dv", "F", "k", "dt", "noise", "seed")}

    want_err = a.storage == "f64" and a.variants != "none"

    def measure(storage, steps, warmup, main=False, fields=False):
        kw = dict(tile=a.tile, tblock=a.tblock, zchunk=a.zchunk) if main else {}
        with gs.Sim(L, L, L, storage=storage, cube_side=wl["cube_side"], **kw, **p) as s:
            if main and a.tune:
                s.tune(reps=2)
            cfg = s.config()
            ms, per_launch, launches = time_steps(torch, s, steps, warmup)
            d = s.diagnostics(allow_nonfinite=True)
            uv = s.read() if fields else None  # FP64 host copies of the final state
        return ms, per_launch, launches, cfg, d, uv

    ms, per_launch, launches, cfg, diag, ref = measure(a.storage, a.steps, a.warmup, main=True, fields=want_err)
    cells = L ** 3
    value = cells / (ms * 1e-3) / 1e9
    bpc = BYTES_PER_CELL[a.storage]
    T = cfg["tblock"]
    # Algorithmic HBM bytes per cell-update: both fields read once and written
    # once (32 B in FP64, 16 B in FP32). A launch that fuses T steps performs T
    # cell-updates per cell, so its algorithmic figure is T passes' worth of
    # bytes and can exceed the HBM peak; `traffic` holds what the counters
    # measured for one launch, and `per_pass` the rate of a single read and
    # write of both fields per launch.
    updates = T * cells
    achieved = bpc * updates / (per_launch * 1e-3) / 1e9
    per_pass = bpc * cells / (per_launch * 1e-3) / 1e9
    kname = "stencil_tb" if cfg["tile"] > 4 else "stencil_tile"
    kernel_key = f"{kname}_{a.storage}_T{T}_L{L}"
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic_for(a.traffic_file, kernel_key),
                kernel=f"{kname} ({T} fused steps per launch)", bytes_per_cell_update=bpc,
                cell_updates_per_launch=updates, algorithmic_bytes_per_launch=bpc * updates,
                launches_timed=launches, ms_per_launch=round(per_launch, 5),
                per_pass=dict(bytes=bpc * cells, gbs=round(per_pass, 1), frac=round(per_pass / HBM_PEAK_GBS, 4)))
    # The secondary roof, vector issue: the method's own instructions per
    # cell-update against the VALU peak (the kernel issues more: the halo
    # rows of the fused levels and address arithmetic).
    ops = alu_ops_per_cell_update(a.storage, p["noise"] != 0.0)
    if ops is not None:
        alu = ops * updates / (per_launch * 1e-3) / 1e12
        roof["alu"] = dict(ops_per_cell_update=ops, achieved=round(alu, 2), peak=round(VALU_PEAK_TOPS, 2),
                           unit="T lane-instructions/s", frac=round(alu / VALU_PEAK_TOPS, 4))

    # Reduced-precision storage: timed over the last variant_steps of the same
    # number of steps as the FP64 run, then compared with the FP64 state (which
    # is bitwise the FP64 definition's) field by field.
    variants = {}
    for sv in [x for x in a.variants.split(",") if x and x not in (a.storage, "none")]:
        total = a.warmup + a.steps
        vsteps = min(a.variant_steps, total)
        vms, _, _, vcfg, vd, vuv = measure(sv, vsteps, total - vsteps, fields=want_err)
        vach = BYTES_PER_CELL[sv] * cells / (vms * 1e-3) / 1e9
        variants[sv] = dict(value=round(cells / (vms * 1e-3) / 1e9, 3), ms_per_step=round(vms, 5),
                            algorithmic_gbs=round(vach, 1), frac=round(vach / HBM_PEAK_GBS, 4), steps_timed=vsteps,
                            bytes_per_cell=BYTES_PER_CELL[sv], launch_config=vcfg)
        if want_err:
            err = {}
            for name, x, y in (("u", vuv[0], ref[0]), ("v", vuv[1], ref[1])):
                dlt = x - y
                err[f"{name}_maxabs"] = float(abs(dlt).max())
                err[f"{name}_rms"] = float(math.sqrt(float((dlt * dlt).mean())))
            variants[sv]["error_vs_f64"] = dict(after_steps=total, **{k: float(f"{v:.3e}") for k, v in err.items()})
            del vuv

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(L, p, a.cpu_seconds)

    out = {
        "metric": "Gcell-updates/s + HBM GB/s vs peak, FP64 vs FP32/BF16 at stated error",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.storage,
        "data": "synthetic (cube initial state, Philox noise)",
        "config": {"workload": f"gray-scott periodic {L}^3, noise 1e-7, {a.storage} storage (one GPU's weak-scaling share)",
                   "L": L, "Du": p["Du"], "Dv": p["Dv"], "F": p["F"], "k": p["k"], "dt": p["dt"],
                   "noise": p["noise"], "launch": cfg},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
        "diagnostics_after": {k: diag[k] for k in ("sum_u", "sum_v", "min_u", "max_u", "min_v", "max_v", "nonfinite")},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
