#!/usr/bin/env python3
"""Throughput of the fused Gray-Scott step on one MI355X.

Workload (default): one GPU's weak-scaling share at L=512 (periodic 512^3
cells), Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1, noise 1e-7 (Philox-keyed),
cube initial state, FP64 storage. A "step" is one time step of the whole
grid: neighbour gather, Laplacian, reaction/feed/kill, noise, Euler update
and the ping-pong; the default launch fuses three steps per pass over HBM.
Inputs are resident in HBM before timing starts.

Timing: after the warm-up steps, blocks of exactly --steps steps are timed
with HIP events on the stream the library launches on, each block bracketed by
device synchronisations; at least five blocks, and more until half a second
of GPU time is covered. `value` is the median block's rate; the spread of the
blocks is reported beside it.

Prints ONE JSON line: metric/value (G cell-updates/s), the roofline of the
step kernel, the FP32/BF16/FP16 storage variants and BF16 with u stored as
1 - u ("bf16c") at the same workload (timed the same way, with their error
against the FP64 state), and the CPU oracle
timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
BYTES_PER_CELL = {"f64": 32, "f32": 16, "bf16": 8, "f16": 8, "bf16c": 8}  # read u,v + write u,v once per step
# Vector issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock at
# 2.4 GHz = 39.3 T lane-instructions/s; FP64 add/mul/fma issue at that rate
# (78.6 TFLOP/s counting an fma as two).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Lanes of the temporally blocked tiles (tile index -> workgroup size).
TB_LANES = {5: 256, 6: 512, 7: 512, 8: 768, 9: 1024}
# Kernel sources whose change invalidates counter measurements.
KERNEL_SOURCES = ["paper_2309_10292_amd/csrc/gs_tblock.hip", "paper_2309_10292_amd/csrc/gs_step.hip",
                  "paper_2309_10292_amd/csrc/gs_device.hpp", "paper_2309_10292_amd/csrc/gs_launch.hpp",
                  "paper_2309_10292_amd/csrc/gs_tblock_common.hpp", "paper_2309_10292_amd/csrc/gs_api.cpp",
                  "paper_2309_10292_amd/csrc/gs_internal.hpp"]
MIN_BLOCKS = 5
MIN_TIMED_SECONDS = 0.5
MAX_BLOCKS = 2000
ERR_STEPS = 1000  # run length of the L=512 workload, at which the variants' error is taken


def alu_ops_per_cell_update(storage, noise):
    """Vector instructions the FP64 step needs per cell-update on this
    hardware: per field, the Laplacian is 5 adds, the product 6c, the
    subtraction and the division by 6 (4 operations for the correctly rounded
    quotient: a product, two fmas and the shift-or that picks the multiplier),
    11 in all; the reaction, feed and kill terms and the Euler update (dt = 1)
    take 13 more. With noise, one Philox4x32-10 block per 4 cells (10 rounds
    of two 32x32->64-bit products and two three-input XORs) plus the word's
    conversion, the fused noise term and its addition: 13."""
    if storage != "f64":
        return None
    return 2 * 11 + 13 + (13 if noise else 0)


def kernel_name(cfg, storage, noise):
    ctype = {"f64": "double", "f32": "float", "bf16": "bf16", "f16": "f16", "bf16c": "bf16c"}[storage]
    tile = cfg["tile"]
    if tile in TB_LANES:
        return (f"stencil_tb<{ctype}, {cfg['tx'] // 4}, {cfg['ty']}, {cfg['tblock']}, {TB_LANES[tile]}, "
                f"{'true' if noise else 'false'}>")
    return f"stencil_tile<{ctype}> (tile {tile})"


def traffic_key(kname, L, zchunk):
    return f"{kname} L={L} zchunk={zchunk}"


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_for(path, key):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), or
    None when there is no measurement for this kernel instantiation, grid and
    z-chunk, or the kernel sources changed since."""
    try:
        with open(path) as f:
            t = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not t or t.get("source_sha256") != kernel_source_hash():
        return None
    return t["bytes"]


def roofline(storage, noise, cells, T, ms_per_launch, traffic):
    """Roof of the step kernel: the larger of the HBM time of one pass
    (both fields read and written once per launch, the least a launch can
    move) and the vector time of the method's instructions for the launch's
    T cell-updates per cell; `frac` is that time over the measured launch
    time, so it cannot exceed 1. The Eq. 5a-style figure (bytes per
    cell-update times cell-updates, which counts fused steps that never reach
    HBM) is kept as `effective`."""
    t = ms_per_launch * 1e-3
    bpc = BYTES_PER_CELL[storage]
    pass_bytes = bpc * cells
    hbm_gbs = pass_bytes / t / 1e9
    hbm = dict(bytes_per_launch=pass_bytes, achieved=round(hbm_gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(hbm_gbs / HBM_PEAK_GBS, 4))
    ops = alu_ops_per_cell_update(storage, noise)
    alu = None
    if ops is not None:
        tops = ops * T * cells / t / 1e12
        alu = dict(ops_per_cell_update=ops, ops_per_launch=ops * T * cells, achieved=round(tops, 2),
                   peak=round(VALU_PEAK_TOPS, 2), unit="T lane-instructions/s", frac=round(tops / VALU_PEAK_TOPS, 4))
    eff = bpc * T * cells / t / 1e9
    out = dict(effective=dict(bytes_per_cell_update=bpc, cell_updates_per_launch=T * cells, gbs=round(eff, 1),
                              frac_of_peak=round(eff / HBM_PEAK_GBS, 4)),
               hbm=hbm, alu=alu, ms_per_launch=round(ms_per_launch, 5), traffic=traffic)
    if traffic:
        out["measured"] = dict(bytes_per_launch=traffic, gbs=round(traffic / t / 1e9, 1),
                               frac=round(traffic / t / 1e9 / HBM_PEAK_GBS, 4),
                               ratio_to_one_pass=round(traffic / pass_bytes, 3))
    if alu is not None and alu["frac"] > hbm["frac"]:
        out.update(bound="alu", achieved=alu["achieved"], peak=alu["peak"], unit=alu["unit"], frac=alu["frac"])
    else:
        out.update(bound="hbm", achieved=hbm["achieved"], peak=hbm["peak"], unit=hbm["unit"], frac=hbm["frac"])
    return out


def parse(argv=None):
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
    ap.add_argument("--variants", default="f32,bf16,f16,bf16c", help="other storage types to time, or 'none'")
    ap.add_argument("--blocks", type=int, default=0, help="timed blocks (0: at least 5, until 0.5 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="budget of the all-thread oracle sample")
    ap.add_argument("--cpu1-seconds", type=float, default=4.0, help="budget of the one-thread oracle sample")
    ap.add_argument("--traffic-file", default=os.path.join(ROOT, "profiles", "traffic.json"))
    return ap.parse_args(argv)


def time_blocks(torch, sim, steps, warmup, blocks=0):
    """Warm-up, then timed blocks of exactly `steps` steps (HIP events on the
    stream the library launches on, torch's current stream, bound at init;
    device synchronisation around every block). Returns per-block ms per
    step, per-block ms per full-depth launch, and launches per block."""
    cfg = sim.config()
    T = cfg["tblock"]
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    full = (steps // T) * T
    per_step, per_launch = [], []
    total = 0.0
    while True:
        torch.cuda.synchronize()
        ev[0].record(st)
        sim.step(full)
        ev[1].record(st)
        sim.step(steps - full)
        ev[2].record(st)
        ev[2].synchronize()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[2])
        per_step.append(ms / steps)
        if full:
            per_launch.append(ev[0].elapsed_time(ev[1]) / (full // T))
        total += ms * 1e-3
        n = len(per_step)
        if blocks:
            if n >= blocks:
                break
        elif (n >= MIN_BLOCKS and total >= MIN_TIMED_SECONDS) or n >= MAX_BLOCKS:
            break
    return per_step, per_launch, full // T


def run_fields(gs, storage, L, wl, p, steps):
    """Both fields, widened to FP64 on the host, after `steps` steps of the
    workload from the cube state in the library's default launch configuration."""
    with gs.Sim(L, L, L, storage=storage, cube_side=wl["cube_side"], **p) as s:
        s.step(steps)
        return s.read()


def spread(xs):
    return dict(median=round(statistics.median(xs), 5), min=round(min(xs), 5), max=round(max(xs), 5), n=len(xs))


def cpu_baseline(L, p, budget_s, budget1_s):
    """The FP64 oracle on the host cores: whole-grid steps of the same
    workload until the time budget is used (at least one step), on every
    thread, and on one thread for a 256^3 grid of the same workload."""
    import numpy as np  # noqa: F401
    from oracle import oracle as O

    def rate(Lc, budget):
        u, v = O.init_cube(L=Lc)
        done, t0 = 0, time.perf_counter()
        while True:
            u, v = O.run(u, v, 1, step0=done, **p)
            done += 1
            el = time.perf_counter() - t0
            if el >= budget:
                return Lc ** 3 * done / el / 1e9, done, el

    threads = O.max_threads()
    v_all, n_all, el_all = rate(L, budget_s)
    L1 = min(L, 256)
    O.set_threads(1)
    try:
        v_one, n_one, el_one = rate(L1, budget1_s)
    finally:
        O.set_threads(threads)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return dict(value=round(v_all, 4), unit="Gcell-updates/s", cores=threads, kind="oracle", cpu_model=model,
                sample=f"{n_all} whole-grid FP64 steps of the {L}^3 noisy workload, {el_all:.1f} s on {threads} threads",
                one_thread=dict(value=round(v_one, 4), unit="Gcell-updates/s", cores=1,
                                sample=f"{n_one} whole-grid FP64 steps of the same workload at {L1}^3, "
                                       f"{el_one:.1f} s on 1 thread"))


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
    noisy = p["noise"] != 0.0
    cells = L ** 3
    want_err = a.storage == "f64" and a.variants != "none"

    def measure(storage, blocks, main=False):
        kw = dict(tile=a.tile, tblock=a.tblock, zchunk=a.zchunk) if main else {}
        with gs.Sim(L, L, L, storage=storage, cube_side=wl["cube_side"], **kw, **p) as s:
            if main and a.tune:
                s.tune(reps=2)
            cfg = s.config()
            tx, ty = gs.tile_info(cfg["tile"], storage, cfg["tblock"])
            cfg.update(tx=tx, ty=ty)
            per_step, per_launch, launches = time_blocks(torch, s, a.steps, a.warmup, blocks)
            d = s.diagnostics(allow_nonfinite=True)
        return dict(per_step=per_step, per_launch=per_launch, launches=launches, cfg=cfg, diag=d)

    m = measure(a.storage, a.blocks, main=True)
    cfg = m["cfg"]
    blocks = len(m["per_step"])
    ms = statistics.median(m["per_step"])
    value = cells / (ms * 1e-3) / 1e9
    T = cfg["tblock"]
    kname = kernel_name(cfg, a.storage, noisy)
    ms_launch = statistics.median(m["per_launch"]) if m["per_launch"] else ms * T
    traffic = traffic_for(a.traffic_file, traffic_key(kname, L, cfg["zchunk"]))
    roof = roofline(a.storage, noisy, cells, T, ms_launch, traffic)
    roof.update(kernel=kname, launch={k: cfg[k] for k in ("tile", "tblock", "zchunk")},
                launches_timed=m["launches"] * blocks,
                ms_per_launch_spread=spread(m["per_launch"]) if m["per_launch"] else None)

    # Reduced-precision storage, timed the same way (same warm-up, block length
    # and number of blocks). Its error is measured on the workload's own run
    # length, ERR_STEPS steps from the cube state, field by field against the
    # FP64 state after as many steps, which is bitwise the FP64 definition's
    # (the FP64 parity tests pin it against the oracle).
    variants = {}
    ref = None
    for sv in [x for x in a.variants.split(",") if x and x not in (a.storage, "none")]:
        vm = measure(sv, blocks)
        vms = statistics.median(vm["per_step"])
        vach = BYTES_PER_CELL[sv] * cells / (vms * 1e-3) / 1e9
        variants[sv] = dict(value=round(cells / (vms * 1e-3) / 1e9, 3), ms_per_step=spread(vm["per_step"]),
                            algorithmic_gbs=round(vach, 1), frac=round(vach / HBM_PEAK_GBS, 4),
                            bytes_per_cell=BYTES_PER_CELL[sv], launch_config=vm["cfg"])
        if want_err:
            if ref is None:
                ref = run_fields(gs, a.storage, L, wl, p, ERR_STEPS)
            got = run_fields(gs, sv, L, wl, p, ERR_STEPS)
            err = {}
            for name, x, y in (("u", got[0], ref[0]), ("v", got[1], ref[1])):
                dlt = x - y
                err[f"{name}_maxabs"] = float(abs(dlt).max())
                err[f"{name}_rms"] = float(math.sqrt(float((dlt * dlt).mean())))
            variants[sv]["error_vs_f64"] = dict(after_steps=ERR_STEPS, **{k: float(f"{v:.3e}") for k, v in err.items()})
            del got
        del vm
    del ref

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(L, p, a.cpu_seconds, a.cpu1_seconds)

    out = {
        "metric": "Gcell-updates/s + HBM GB/s vs peak, FP64 vs FP32/BF16 at stated error",
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 5),
        "timed_blocks": dict(spread(m["per_step"]), steps_per_block=a.steps,
                             gcells_min=round(cells / (max(m["per_step"]) * 1e-3) / 1e9, 3),
                             gcells_max=round(cells / (min(m["per_step"]) * 1e-3) / 1e9, 3)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.storage,
        "data": "synthetic (cube initial state, Philox noise)",
        "config": {"workload": f"gray-scott periodic {L}^3, noise 1e-7, {a.storage} storage (one GPU's weak-scaling share)",
                   "L": L, "Du": p["Du"], "Dv": p["Dv"], "F": p["F"], "k": p["k"], "dt": p["dt"],
                   "noise": p["noise"], "launch": {k: cfg[k] for k in ("tile", "tblock", "zchunk")}},
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
        "diagnostics_after": {k: m["diag"][k] for k in ("sum_u", "sum_v", "min_u", "max_u", "min_v", "max_v", "nonfinite")},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
