"""The learned 16-step surrogate: binding of gs_surrogate_* (include/gs.h),
training-data generation with the batched stencil, the training loop and the
inference controller that falls back to the stencil.

Argument marshalling and control flow only: the network's forward and
backward passes, the optimiser, the stencil steps, initial states and the
error checks all run in libgs's kernels.
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np

from . import gs

NPARAMS = 60578
JUMP = 16  # steps replaced by one surrogate evaluation


class Surrogate:
    def __init__(self, nx, ny, nz, max_batch=1, params=None, device="cuda", stream=None):
        import torch
        lib = gs.load()
        self.shape = (int(nz), int(ny), int(nx))
        self.max_batch = int(max_batch)
        wsb = int(lib.gs_surrogate_workspace_bytes(nx, ny, nz, max_batch))
        if wsb == 0:
            raise gs.GSError(gs.GS_ERR_UNSUPPORTED, f"surrogate grid {nx}x{ny}x{nz} unsupported")
        self.workspace = torch.empty(wsb, dtype=torch.uint8, device=torch.device(device))
        self.stream = gs._stream_handle(stream)
        if params is None:
            from synth import surrogate_init
            params = surrogate_init(0)
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == NPARAMS
        h = ctypes.c_void_p()
        gs.check(lib.gs_surrogate_init(nx, ny, nz, max_batch, p.ctypes.data, self.workspace.data_ptr(), wsb,
                                       self.stream, ctypes.byref(h)))
        self.h = h

    def params(self) -> np.ndarray:
        out = np.empty(NPARAMS, dtype=np.float32)
        gs.check(gs.load().gs_surrogate_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        gs.check(gs.load().gs_surrogate_set_params(self.h, p.ctypes.data))

    @staticmethod
    def _fk(F, k, n):
        F = np.ascontiguousarray(np.broadcast_to(np.asarray(F, dtype=np.float64), (n,)))
        k = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.float64), (n,)))
        return F, k

    def predict(self, u, v, F, k, u_out=None, v_out=None):
        """u, v: CUDA tensors (nsamp, nz, ny, nx) or (nz, ny, nx), float64 or float32."""
        import torch
        single = u.dim() == 3
        n = 1 if single else u.shape[0]
        io = {torch.float64: gs.DTYPES["f64"], torch.float32: gs.DTYPES["f32"]}[u.dtype]
        assert u.is_contiguous() and v.is_contiguous() and u.dtype == v.dtype
        u_out = torch.empty_like(u) if u_out is None else u_out
        v_out = torch.empty_like(v) if v_out is None else v_out
        Fa, ka = self._fk(F, k, n)
        gs.check(gs.load().gs_surrogate_predict(self.h, n, io, u.data_ptr(), v.data_ptr(), Fa.ctypes.data,
                                                ka.ctypes.data, u_out.data_ptr(), v_out.data_ptr()))
        return u_out, v_out

    def loss_grad(self, u, v, ut, vt, F, k, want_grad=False):
        """FP32 CUDA tensors (nsamp, nz, ny, nx). Returns (loss, grad or None)."""
        n = u.shape[0]
        Fa, ka = self._fk(F, k, n)
        loss = ctypes.c_double()
        g = np.empty(NPARAMS, dtype=np.float32) if want_grad else None
        gs.check(gs.load().gs_surrogate_loss_grad(self.h, n, u.data_ptr(), v.data_ptr(), ut.data_ptr(), vt.data_ptr(),
                                                  Fa.ctypes.data, ka.ctypes.data, ctypes.byref(loss),
                                                  g.ctypes.data if want_grad else None))
        return loss.value, g

    # gs_surr_tensor values (include/gs.h)
    INPUT, PRE, ACT, PRED, DOUT, DPRE = range(6)
    _CHANNELS = {INPUT: 8, PRE: 32, ACT: 32, DOUT: 8, DPRE: 32}

    def read_tensor(self, tensor, layer, nsamp):
        """A stored tensor of the last forward/backward pass of nsamp samples:
        BF16 tensors as float32 arrays (nsamp, nz, ny, nx, channels); the
        prediction as float32 (2, nsamp, nz, ny, nx)."""
        rows = nsamp * int(np.prod(self.shape))
        if tensor == self.PRED:
            out = np.empty(2 * rows, dtype=np.float32)
            gs.check(gs.load().gs_surrogate_read_tensor(self.h, tensor, layer, out.ctypes.data, out.nbytes))
            return out.reshape((2, nsamp) + self.shape)
        c = self._CHANNELS[tensor]
        raw = np.empty(rows * c, dtype=np.uint16)
        gs.check(gs.load().gs_surrogate_read_tensor(self.h, tensor, layer, raw.ctypes.data, raw.nbytes))
        return (raw.astype(np.uint32) << 16).view(np.float32).reshape((nsamp,) + self.shape + (c,))

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        gs.check(gs.load().gs_surrogate_adam(self.h, float(lr), float(beta1), float(beta2), float(eps)))

    def close(self):
        if self.h is not None and self.h.value:
            gs.check(gs.load().gs_surrogate_destroy(self.h))
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def generate_pairs(L, blobs, steps_total, pair_every, warm=0, storage="f32", device="cuda"):
    """Training pairs from stencil trajectories (batched persistent sweeps).

    `blobs` (synth.random_blobs) gives one trajectory each: a random cube of
    (0.25, 0.33) in a (1, 0) background and its own (F, k). After `warm`
    steps, every `pair_every` steps the state and the state JUMP steps later
    form one pair. Returns FP32 tensors (N, L, L, L) u, v, ut, vt and numpy F, k.
    """
    import torch
    sims = [dict(L=L, F=b["F"], k=b["k"]) for b in blobs]
    us, vs, uts, vts, Fs, ks = [], [], [], [], [], []
    with gs.Batch(sims, storage=storage, init="none", Du=0.2, Dv=0.1, dt=1.0, device=device) as bt:
        for i, b in enumerate(blobs):
            bt.fill_cube(i, b["x0"], b["y0"], b["z0"], b["side"])
        bt.step(warm)
        t = warm
        while t + JUMP <= steps_total:
            cur = [_field_views(bt, i, L) for i in range(len(blobs))]
            snap = [(u.clone(), v.clone()) for u, v in cur]
            bt.step(JUMP)
            for i, b in enumerate(blobs):
                u1, v1 = _field_views(bt, i, L)
                us.append(snap[i][0]); vs.append(snap[i][1])
                uts.append(u1.clone()); vts.append(v1.clone())
                Fs.append(b["F"]); ks.append(b["k"])
            extra = pair_every - JUMP
            if extra > 0:
                bt.step(extra)
            t += max(pair_every, JUMP)
        bt.sync()
    stack = lambda xs: torch.stack(xs).contiguous()
    return stack(us), stack(vs), stack(uts), stack(vts), np.array(Fs), np.array(ks)


def _field_views(bt, i, L):
    import torch
    pu, pv, _ = bt.current_ptrs(i)
    # views of the batch arena at the simulation's current buffers
    base = bt.arena.data_ptr()
    n = L ** 3
    es = bt.arena.element_size()
    dt = {0: torch.float64, 1: torch.float32, 2: torch.bfloat16, 3: torch.float16}[bt.params.storage]
    item = torch.tensor([], dtype=dt).element_size()
    u = bt.arena[(pu - base) // es:(pu - base) // es + n * item].view(dt).view(L, L, L)
    v = bt.arena[(pv - base) // es:(pv - base) // es + n * item].view(dt).view(L, L, L)
    return u, v


def train(model: Surrogate, data, iters, batch, lr=1e-3, seed=0, log_every=0, lr_final=None):
    """Adam on random minibatches of `data` (generate_pairs output). Returns the loss history."""
    u, v, ut, vt, F, k = data
    rng = np.random.default_rng(seed)
    hist = []
    for it in range(iters):
        idx = rng.choice(u.shape[0], size=batch, replace=False)
        import torch
        ii = torch.as_tensor(idx, device=u.device)
        loss, _ = model.loss_grad(u[ii].contiguous(), v[ii].contiguous(), ut[ii].contiguous(), vt[ii].contiguous(),
                                  F[idx], k[idx])
        step_lr = lr if lr_final is None else lr * (lr_final / lr) ** (it / max(1, iters - 1))
        model.adam(step_lr)
        hist.append(loss)
        if log_every and it % log_every == 0:
            print(f"iter {it} loss {loss:.4e}", flush=True)
    return hist


def run_controlled(model: Surrogate, sim, F, k, jumps, check_every=4, tol=1e-3):
    """Advances `sim` (a gs.Sim) by jumps x JUMP steps with surrogate jumps in
    windows of `check_every` jumps. The last jump of every window is computed
    by the stencil, and the surrogate's prediction of the same jump (from the
    same state) is compared with it: the check bounds the error of that one
    jump, not the drift the window's earlier, unchecked jumps accumulated. If
    the RMS difference over both fields is within `tol`, the stencil's result
    of that jump is kept; otherwise (or if it is not finite) the whole window
    is rolled back to its verified starting state and recomputed with the
    stencil (a fallback). Returns counts, the RMS of every check and the wall
    time."""
    import torch
    st = torch.cuda.current_stream()
    fallbacks, checks, errors = 0, 0, []
    u, v, _ = sim.current()
    pu, pv = torch.empty_like(u), torch.empty_like(v)
    snap_u, snap_v = torch.empty_like(u), torch.empty_like(v)
    t0 = time.perf_counter()
    j = 0
    while j < jumps:
        w = min(check_every, jumps - j)
        u, v, step0 = sim.current()
        gs.copy(u, snap_u)
        gs.copy(v, snap_v)
        for i in range(w):
            u, v, _ = sim.current()
            model.predict(u, v, F, k, pu, pv)
            if i < w - 1 or w < check_every:
                # unchecked jump: the prediction becomes the state
                gs.copy(pu, u)
                gs.copy(pv, v)
                sim.advance_index(JUMP)
                continue
            checks += 1
            sim.step(JUMP)
            su, sv, _ = sim.current()
            rms = ((gs.sqdiff(pu, su) + gs.sqdiff(pv, sv)) / (2 * su.numel())) ** 0.5
            errors.append(rms)
            if not (math.isfinite(rms) and rms <= tol):
                fallbacks += 1
                u, v, _ = sim.current()
                gs.copy(snap_u, u)
                gs.copy(snap_v, v)
                sim.set_index(step0)
                sim.step(w * JUMP)
        j += w
    st.synchronize()
    el = time.perf_counter() - t0
    return dict(jumps=jumps, checks=checks, fallbacks=fallbacks, rms=errors, seconds=el)
