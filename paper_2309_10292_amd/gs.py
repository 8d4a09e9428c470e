"""ctypes binding of libgs.so (include/gs.h), same names as the C ABI.

Argument marshalling only: PyTorch provides device memory (four field
buffers and the workspace) and the HIP stream; every step of the path runs in
the library's kernels. Importing this module does not touch the GPU. Calls
fail loudly (RuntimeError) when the library is missing or returns an error.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libgs.so")

GS_OK, GS_ERR_INVALID_ARG, GS_ERR_UNSUPPORTED, GS_ERR_HIP, GS_ERR_NONFINITE, GS_ERR_STATE = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "GS_OK", -1: "GS_ERR_INVALID_ARG", -2: "GS_ERR_UNSUPPORTED", -3: "GS_ERR_HIP",
                -4: "GS_ERR_NONFINITE", -5: "GS_ERR_STATE"}
# "bf16c": BF16 storage whose u buffers hold 1 - u (GS_BF16C)
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "bf16c": 4}
INIT_NONE, INIT_CUBE = 0, 1
MAX_TBLOCK = 4


class gs_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("storage", ctypes.c_int32),
                ("Du", ctypes.c_double), ("Dv", ctypes.c_double), ("F", ctypes.c_double),
                ("k", ctypes.c_double), ("dt", ctypes.c_double), ("noise", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("step0", ctypes.c_uint64),
                ("init_mode", ctypes.c_int32), ("cube_side", ctypes.c_int32),
                ("cube_u", ctypes.c_double), ("cube_v", ctypes.c_double),
                ("tblock", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("zchunk", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class gs_diag(ctypes.Structure):
    _fields_ = [("sum_u", ctypes.c_double), ("sum_v", ctypes.c_double),
                ("min_u", ctypes.c_double), ("max_u", ctypes.c_double),
                ("min_v", ctypes.c_double), ("max_v", ctypes.c_double),
                ("nonfinite", ctypes.c_int64)]


class gs_tune_entry(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("tblock", ctypes.c_int32), ("zchunk", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("ms_per_step", ctypes.c_double)]


class gs_batch_tune_entry(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("n_sims", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("tblock", ctypes.c_int32), ("zchunk", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("ms_per_step", ctypes.c_double), ("gcells", ctypes.c_double)]


class GSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

# (name, restype, argtypes) of every entry point the header declares.
_VP, _DP, _I32, _I64, _SZ = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_PP = ctypes.POINTER(gs_params)
_SIM = ctypes.c_void_p
SIGNATURES = [
    ("gs_version", ctypes.c_char_p, []),
    ("gs_last_error", ctypes.c_char_p, []),
    ("gs_workspace_bytes", _SZ, [_PP]),
    ("gs_num_tiles", _I32, []),
    ("gs_tile_info", _I32, [_I32, _I32, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    ("gs_init", _I32, [_PP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(_SIM)]),
    ("gs_step", _I32, [_SIM, _I64]),
    ("gs_read", _I32, [_SIM, _DP, _DP]),
    ("gs_write", _I32, [_SIM, _DP, _DP]),
    ("gs_current", _I32, [_SIM, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_uint64)]),
    ("gs_diagnostics", _I32, [_SIM, ctypes.POINTER(gs_diag)]),
    ("gs_sync", _I32, [_SIM]),
    ("gs_destroy", _I32, [_SIM]),
    ("gs_set_config", _I32, [_SIM, _I32, _I32, _I32]),
    ("gs_get_config", _I32, [_SIM, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    ("gs_tune", _I32, [_SIM, _I32, ctypes.c_void_p, _I32, ctypes.POINTER(_I32)]),
    ("gs_step_graph", _I32, [_SIM, _I64]),
    ("gs_batch_arena_bytes", _SZ, [_I32, _I32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("gs_batch_workspace_bytes", _SZ, [_I32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("gs_batch_init", _I32, [_PP, _I32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p, _VP, _SZ, _VP, _SZ, _VP, ctypes.POINTER(_SIM)]),
    ("gs_batch_step", _I32, [_SIM, _I64]),
    ("gs_batch_step_graph", _I32, [_SIM, _I64]),
    ("gs_batch_set_config", _I32, [_SIM, _I32, _I32, _I32, _I32]),
    ("gs_batch_get_config", _I32, [_SIM, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    ("gs_batch_tune", _I32, [_SIM, _I32, ctypes.c_void_p, _I32, ctypes.POINTER(_I32)]),
    ("gs_batch_max_tblock", _I32, [_I32, _I32]),
    ("gs_batch_current", _I32, [_SIM, _I32, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_uint64)]),
    ("gs_batch_read", _I32, [_SIM, _I32, _DP, _DP]),
    ("gs_batch_write", _I32, [_SIM, _I32, _DP, _DP]),
    ("gs_batch_diagnostics", _I32, [_SIM, _I32, ctypes.POINTER(gs_diag)]),
    ("gs_batch_sync", _I32, [_SIM]),
    ("gs_batch_destroy", _I32, [_SIM]),
    ("gs_surrogate_workspace_bytes", _SZ, [_I32, _I32, _I32, _I32]),
    ("gs_surrogate_init", _I32, [_I32, _I32, _I32, _I32, ctypes.c_void_p, _VP, _SZ, _VP, ctypes.POINTER(_SIM)]),
    ("gs_surrogate_set_params", _I32, [_SIM, ctypes.c_void_p]),
    ("gs_surrogate_get_params", _I32, [_SIM, ctypes.c_void_p]),
    ("gs_surrogate_predict", _I32, [_SIM, _I32, _I32, _VP, _VP, ctypes.c_void_p, ctypes.c_void_p, _VP, _VP]),
    ("gs_surrogate_loss_grad", _I32, [_SIM, _I32, _VP, _VP, _VP, _VP, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    ("gs_surrogate_adam", _I32, [_SIM, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    ("gs_surrogate_read_tensor", _I32, [_SIM, _I32, _I32, ctypes.c_void_p, _SZ]),
    ("gs_surrogate_destroy", _I32, [_SIM]),
    ("gs_set_step", _I32, [_SIM, ctypes.c_uint64]),
    ("gs_fill_cube", _I32, [_SIM, _I32, _I32, _I32, _I32, ctypes.c_double, ctypes.c_double]),
    ("gs_batch_fill_cube", _I32, [_SIM, _I32, _I32, _I32, _I32, _I32, ctypes.c_double, ctypes.c_double]),
    ("gs_sqdiff_workspace_bytes", _SZ, []),
    ("gs_sqdiff", _I32, [_VP, _VP, _SZ, _I32, _VP, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("gs_sqdiff_noalloc", _I32, [_VP, _VP, _SZ, _I32, _VP, ctypes.POINTER(ctypes.c_double)]),
    ("gs_laplacian7", _I32, [_VP, _VP, _I32, _I32, _I32, _VP]),
    ("gs_copy", _I32, [_VP, _VP, _SZ, _VP]),
]


def load(path: str = LIB_PATH):
    """Load libgs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"libgs.so not found at {path}: build it with python paper_2309_10292_amd/build.py "
                               "(the HIP library is required; there is no fallback)")
        L = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return load().gs_last_error().decode()


def check(status: int):
    if status != GS_OK:
        raise GSError(status, last_error())


def make_params(nx, ny, nz, *, storage="f64", Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1.0, noise=0.0,
                seed=0, step0=0, init="cube", cube_side=12, cube_u=0.25, cube_v=0.33, tblock=0, tile=0, zchunk=0):
    p = gs_params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.storage = DTYPES[storage] if isinstance(storage, str) else int(storage)
    p.Du, p.Dv, p.F, p.k, p.dt, p.noise = float(Du), float(Dv), float(F), float(k), float(dt), float(noise)
    p.seed, p.step0 = int(seed), int(step0)
    p.init_mode = INIT_CUBE if init == "cube" else INIT_NONE
    p.cube_side, p.cube_u, p.cube_v = int(cube_side), float(cube_u), float(cube_v)
    p.tblock, p.tile, p.zchunk = int(tblock), int(tile), int(zchunk)
    return p


def workspace_bytes(p: gs_params) -> int:
    return int(load().gs_workspace_bytes(ctypes.byref(p)))


def _torch_dtype(storage):
    import torch
    return {0: torch.float64, 1: torch.float32, 2: torch.bfloat16, 3: torch.float16, 4: torch.bfloat16}[storage]


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def max_tblock(tile: int, storage="f64", batch: bool = False) -> int:
    """Largest fused depth `tile` accepts for a storage type (0: not available)."""
    st = DTYPES[storage] if isinstance(storage, str) else int(storage)
    L = load()
    if batch:
        return int(L.gs_batch_max_tblock(int(tile), st))
    mt = ctypes.c_int32()
    if L.gs_tile_info(int(tile), st, 1, None, None, ctypes.byref(mt)) != GS_OK:
        return 0
    return int(mt.value)


def tile_info(tile: int, storage="f64", tblock: int = 1):
    """Output tile (tx cells, ty rows) of `tile` for a storage type and depth."""
    st = DTYPES[storage] if isinstance(storage, str) else int(storage)
    tx, ty = ctypes.c_int32(), ctypes.c_int32()
    check(load().gs_tile_info(int(tile), st, int(tblock), ctypes.byref(tx), ctypes.byref(ty), None))
    return tx.value, ty.value


def tblock_tiles():
    """Tile indices of the temporally blocked kernel (the first four tiles
    select the single-step kernel)."""
    return list(range(5, int(load().gs_num_tiles()) + 1))


class Sim:
    """One Gray-Scott simulation bound to four torch-allocated device buffers.

    Keyword arguments are those of gs_params (see make_params); `init` is
    "cube" or "none" (then pass u0, v0 as float64 numpy arrays, written with
    gs_write).
    """

    def __init__(self, nx, ny, nz, *, device="cuda", stream=None, u0=None, v0=None, **kw):
        import torch
        lib = load()
        if u0 is not None:
            kw["init"] = "none"
        self.params = make_params(nx, ny, nz, **kw)
        self.shape = (int(nz), int(ny), int(nx))
        n = int(nx) * int(ny) * int(nz)
        dt = _torch_dtype(self.params.storage)
        dev = torch.device(device)
        self.buffers = [torch.empty(n, dtype=dt, device=dev) for _ in range(4)]
        wsb = workspace_bytes(self.params)
        if wsb == 0:
            # invalid params: let gs_init report why
            wsb = 256
        self.workspace = torch.empty(wsb, dtype=torch.uint8, device=dev)
        self._stream_obj = stream
        self.stream = _stream_handle(stream)
        h = ctypes.c_void_p()
        check(lib.gs_init(ctypes.byref(self.params), *[b.data_ptr() for b in self.buffers],
                          self.workspace.data_ptr(), self.stream, ctypes.byref(h)))
        self.h = h
        if u0 is not None:
            self.write(u0, v0)

    def step(self, n: int = 1):
        check(load().gs_step(self.h, int(n)))

    def step_graph(self, n: int):
        """Same as step(n), replayed from a captured HIP graph."""
        check(load().gs_step_graph(self.h, int(n)))

    def set_config(self, tile: int, tblock: int, zchunk: int):
        check(load().gs_set_config(self.h, int(tile), int(tblock), int(zchunk)))

    def config(self):
        t, b, z = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(load().gs_get_config(self.h, ctypes.byref(t), ctypes.byref(b), ctypes.byref(z)))
        return dict(tile=t.value, tblock=b.value, zchunk=z.value)

    def tune(self, reps: int = 3):
        """Autotune the launch configuration on this grid (state unchanged).
        Returns (chosen config, list of measured candidates)."""
        cap = 256
        table = (gs_tune_entry * cap)()
        n = ctypes.c_int32()
        check(load().gs_tune(self.h, int(reps), ctypes.cast(table, ctypes.c_void_p), cap, ctypes.byref(n)))
        rows = [dict(tile=e.tile, tblock=e.tblock, zchunk=e.zchunk, ms_per_step=e.ms_per_step)
                for e in table[:min(n.value, cap)]]
        return self.config(), rows

    def read(self):
        u = np.empty(self.shape, dtype=np.float64)
        v = np.empty(self.shape, dtype=np.float64)
        check(load().gs_read(self.h, u.ctypes.data_as(_DP), v.ctypes.data_as(_DP)))
        return u, v

    def write(self, u=None, v=None):
        def prep(a):
            if a is None:
                return None, None
            a = np.ascontiguousarray(a, dtype=np.float64)
            assert a.shape == self.shape, (a.shape, self.shape)
            return a, a.ctypes.data_as(_DP)
        ua, up = prep(u)
        va, vp = prep(v)
        check(load().gs_write(self.h, up, vp))

    def current(self):
        """(u_tensor, v_tensor, step): views of the buffers holding the current state."""
        pu, pv, st = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_uint64()
        check(load().gs_current(self.h, ctypes.byref(pu), ctypes.byref(pv), ctypes.byref(st)))
        by_ptr = {b.data_ptr(): b for b in self.buffers}
        return by_ptr[pu.value].view(self.shape), by_ptr[pv.value].view(self.shape), int(st.value)

    def diagnostics(self, allow_nonfinite=False):
        d = gs_diag()
        s = load().gs_diagnostics(self.h, ctypes.byref(d))
        if s != GS_OK and not (allow_nonfinite and s == GS_ERR_NONFINITE):
            check(s)
        return dict(sum_u=d.sum_u, sum_v=d.sum_v, min_u=d.min_u, max_u=d.max_u, min_v=d.min_v,
                    max_v=d.max_v, nonfinite=int(d.nonfinite))

    def set_index(self, step: int):
        """Set the global step index of the current state (gs_set_step)."""
        check(load().gs_set_step(self.h, int(step)))

    def advance_index(self, n: int):
        """Advance the step index by n without computing steps (the state was
        replaced by other means)."""
        _, _, st = self.current()
        check(load().gs_set_step(self.h, st + int(n)))

    def fill_cube(self, x0, y0, z0, side, cu=0.25, cv=0.33):
        check(load().gs_fill_cube(self.h, int(x0), int(y0), int(z0), int(side), float(cu), float(cv)))

    def sync(self):
        check(load().gs_sync(self.h))

    def close(self):
        if self.h is not None and self.h.value:
            check(load().gs_destroy(self.h))
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Many independent simulations advanced by persistent launches.

    `sims` is a list of dicts {nx, ny, nz, F, k} (or {L, F, k} for cubes);
    the remaining keyword arguments are the shared gs_params (storage, Du, Dv,
    dt, noise, seed, init, cube_side, ...). One torch allocation holds all
    fields (the arena) and one the workspace.
    """

    def __init__(self, sims, *, device="cuda", stream=None, **kw):
        import torch
        lib = load()
        n = len(sims)
        dims = [(int(d.get("nx", d.get("L"))), int(d.get("ny", d.get("L"))), int(d.get("nz", d.get("L"))))
                for d in sims]
        self.n = n
        self.shapes = [(nz, ny, nx) for (nx, ny, nz) in dims]
        self.nx = (ctypes.c_int32 * n)(*[d[0] for d in dims])
        self.ny = (ctypes.c_int32 * n)(*[d[1] for d in dims])
        self.nz = (ctypes.c_int32 * n)(*[d[2] for d in dims])
        F = (ctypes.c_double * n)(*[float(d["F"]) for d in sims])
        k = (ctypes.c_double * n)(*[float(d["k"]) for d in sims])
        self.params = make_params(8, 8, 8, **kw)
        arena_b = int(lib.gs_batch_arena_bytes(self.params.storage, n, self.nx, self.ny, self.nz))
        ws_b = int(lib.gs_batch_workspace_bytes(n, self.nx, self.ny, self.nz))
        if arena_b == 0 or ws_b == 0:
            raise GSError(GS_ERR_INVALID_ARG, "invalid batch grid sizes or storage type")
        dev = torch.device(device)
        self.arena = torch.empty(arena_b, dtype=torch.uint8, device=dev)
        self.workspace = torch.empty(ws_b, dtype=torch.uint8, device=dev)
        self.stream = _stream_handle(stream)
        h = ctypes.c_void_p()
        check(lib.gs_batch_init(ctypes.byref(self.params), n, self.nx, self.ny, self.nz, F, k,
                                self.arena.data_ptr(), arena_b, self.workspace.data_ptr(), ws_b, self.stream,
                                ctypes.byref(h)))
        self.h = h

    def step(self, n: int = 1):
        check(load().gs_batch_step(self.h, int(n)))

    def step_graph(self, n: int):
        check(load().gs_batch_step_graph(self.h, int(n)))

    def set_config(self, tile, tblock, zchunk, sim=-1):
        check(load().gs_batch_set_config(self.h, int(sim), int(tile), int(tblock), int(zchunk)))

    def config(self, sim):
        t, b, z = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(load().gs_batch_get_config(self.h, int(sim), ctypes.byref(t), ctypes.byref(b), ctypes.byref(z)))
        return dict(tile=t.value, tblock=b.value, zchunk=z.value)

    def tune(self, reps: int = 2):
        cap = 1024
        table = (gs_batch_tune_entry * cap)()
        n = ctypes.c_int32()
        check(load().gs_batch_tune(self.h, int(reps), ctypes.cast(table, ctypes.c_void_p), cap, ctypes.byref(n)))
        return [dict(nx=e.nx, ny=e.ny, nz=e.nz, n_sims=e.n_sims, tile=e.tile, tblock=e.tblock, zchunk=e.zchunk,
                     ms_per_step=e.ms_per_step, gcells=e.gcells) for e in table[:min(n.value, cap)]]

    def current_ptrs(self, sim):
        pu, pv, st = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_uint64()
        check(load().gs_batch_current(self.h, int(sim), ctypes.byref(pu), ctypes.byref(pv), ctypes.byref(st)))
        return pu.value, pv.value, int(st.value)

    def read(self, sim):
        shape = self.shapes[sim]
        u = np.empty(shape, dtype=np.float64)
        v = np.empty(shape, dtype=np.float64)
        check(load().gs_batch_read(self.h, int(sim), u.ctypes.data_as(_DP), v.ctypes.data_as(_DP)))
        return u, v

    def write(self, sim, u, v):
        shape = self.shapes[sim]
        u = np.ascontiguousarray(u, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert u.shape == shape and v.shape == shape
        check(load().gs_batch_write(self.h, int(sim), u.ctypes.data_as(_DP), v.ctypes.data_as(_DP)))

    def diagnostics(self, sim):
        d = gs_diag()
        check(load().gs_batch_diagnostics(self.h, int(sim), ctypes.byref(d)))
        return dict(sum_u=d.sum_u, sum_v=d.sum_v, min_u=d.min_u, max_u=d.max_u, min_v=d.min_v,
                    max_v=d.max_v, nonfinite=int(d.nonfinite))

    def fill_cube(self, sim, x0, y0, z0, side, cu=0.25, cv=0.33):
        check(load().gs_batch_fill_cube(self.h, int(sim), int(x0), int(y0), int(z0), int(side), float(cu), float(cv)))

    def sync(self):
        check(load().gs_batch_sync(self.h))

    def close(self):
        if self.h is not None and self.h.value:
            check(load().gs_batch_destroy(self.h))
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


_sqdiff_ws = {}


def sqdiff(a, b, stream=None):
    """Sum of (a - b)^2 in FP64 over two equal CUDA tensors (library kernel)."""
    import torch
    assert a.is_cuda and b.is_cuda and a.dtype == b.dtype and a.numel() == b.numel()
    assert a.is_contiguous() and b.is_contiguous()
    storage = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2, torch.float16: 3}[a.dtype]
    dev = a.device
    if dev not in _sqdiff_ws:
        _sqdiff_ws[dev] = torch.empty(int(load().gs_sqdiff_workspace_bytes()), dtype=torch.uint8, device=dev)
    out = ctypes.c_double()
    check(load().gs_sqdiff(a.data_ptr(), b.data_ptr(), a.numel(), storage, _sqdiff_ws[dev].data_ptr(),
                           _stream_handle(stream), ctypes.byref(out)))
    return out.value


def sqdiff_noalloc(a, b, stream=None):
    """As sqdiff, through gs_sqdiff_noalloc (the library's static scratch; no workspace)."""
    import torch
    assert a.is_cuda and b.is_cuda and a.dtype == b.dtype and a.numel() == b.numel()
    assert a.is_contiguous() and b.is_contiguous()
    storage = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2, torch.float16: 3}[a.dtype]
    out = ctypes.c_double()
    check(load().gs_sqdiff_noalloc(a.data_ptr(), b.data_ptr(), a.numel(), storage, _stream_handle(stream),
                                   ctypes.byref(out)))
    return out.value


def laplacian7(f, out=None, stream=None):
    """Single-field FP64 Laplacian of a (nz, ny, nx) float64 CUDA tensor."""
    import torch
    assert f.dtype == torch.float64 and f.is_cuda and f.is_contiguous() and f.dim() == 3
    if out is None:
        out = torch.empty_like(f)
    nz, ny, nx = f.shape
    check(load().gs_laplacian7(f.data_ptr(), out.data_ptr(), nx, ny, nz, _stream_handle(stream)))
    return out


def copy(src, dst, stream=None):
    """Device copy with the library's streaming kernel (bandwidth reference)."""
    assert src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= nbytes
    check(load().gs_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream_handle(stream)))
