"""Calibration runs on one MI355X: the achievable streaming bandwidth (the
library's copy kernel) and the single-field FP64 7-point Laplacian, the
analogue of the paper's single-variable rows (Section 5.1, Tables 2 and 3).

Bandwidths use the periodic form of the paper's effective-bytes model
(Eq. 4a/4b, 5a): every cell is read once and written once, 16 bytes per
cell for the FP64 Laplacian, 2 x bytes for a copy.

    python -m paper_2309_10292_amd.calibrate [--L 1024] [--reps 20]
"""
from __future__ import annotations

import argparse
import json

HBM_PEAK_GBS = 8000.0


def _time(torch, fn, reps, warmup=3):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--copy-gib", type=float, default=4.0)
    a = ap.parse_args(argv)
    import torch
    from paper_2309_10292_amd import gs
    out = {}
    nbytes = int(a.copy_gib * (1 << 30)) // 16 * 16
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    ms = _time(torch, lambda: gs.copy(src, dst), a.reps)
    bw = 2 * nbytes / (ms * 1e-3) / 1e9
    out["copy"] = dict(bytes=nbytes, ms=round(ms, 4), gbs=round(bw, 1), frac=round(bw / HBM_PEAK_GBS, 4))
    ms_t = _time(torch, lambda: dst.copy_(src), a.reps)
    bw_t = 2 * nbytes / (ms_t * 1e-3) / 1e9
    out["torch_copy"] = dict(ms=round(ms_t, 4), gbs=round(bw_t, 1), frac=round(bw_t / HBM_PEAK_GBS, 4))
    del src, dst
    L = a.L
    f = torch.rand((L, L, L), dtype=torch.float64, device="cuda")
    o = torch.empty_like(f)
    ms = _time(torch, lambda: gs.laplacian7(f, o), a.reps)
    cells = L ** 3
    bw = 16 * cells / (ms * 1e-3) / 1e9
    out["laplacian7_f64"] = dict(L=L, ms=round(ms, 4), gcells=round(cells / (ms * 1e-3) / 1e9, 2), gbs=round(bw, 1),
                                 frac=round(bw / HBM_PEAK_GBS, 4))
    print(json.dumps(out))
    return out


if __name__ == "__main__":
    main()
