"""Python access to the FP64 Gray-Scott oracle (gs_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the HIP library or its binding.

Arrays are numpy float64, shape (nz, ny, nx), C-contiguous, so that the flat
index is idx = x + nx (y + ny z), the layout the paper's problem is read in.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "libgs_oracle.so")

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile gs_oracle.c with gcc (plain C, no contraction). Returns the .so path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class OracleLib:
    """ctypes view of one build of gs_oracle.c (the default build, or a test's
    deliberately mutated copy)."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i, d, u64, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_int64
        sig = {
            "gso_philox4x32_10": ([u32p, u32p, u32p], None),
            "gso_noise_r": ([u64, u64, u64], d),
            "gso_noise_field": ([u64, u64, i64, dp], None),
            "gso_init_cube": ([i, i, i, i, d, d, dp, dp], None),
            "gso_laplacian": ([i, i, i, dp, dp], None),
            "gso_step": ([i, i, i, d, d, d, d, d, d, u64, u64, dp, dp, dp, dp], None),
            "gso_run": ([i, i, i, d, d, d, d, d, d, u64, u64, i64, dp, dp], ctypes.c_int),
            "gso_run_window": ([i, i, i, i, i, i, i, d, d, d, d, d, d, u64, u64, i64, dp, dp], ctypes.c_int),
            "gso_set_threads": ([i], None),
            "gso_max_threads": ([], i),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        self.L = L

    def __getattr__(self, name):
        return getattr(self.L, name)


def build_from(src: str, out: str) -> str:
    """Compile another copy of the oracle source (used by mutation tests)."""
    subprocess.run(["gcc", *CFLAGS, src, "-o", out, "-lm"], check=True)
    return out


_lib = None


def lib(override: "OracleLib | None" = None) -> OracleLib:
    if override is not None:
        return override
    global _lib
    if _lib is None:
        _lib = OracleLib(build())
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n: int) -> None:
    lib().gso_set_threads(int(n))


def max_threads() -> int:
    return int(lib().gso_max_threads())


def philox4x32_10(counter, key, impl=None):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in counter])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib(impl).gso_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def noise_r(seed: int, t: int, idx: int, impl=None) -> float:
    return float(lib(impl).gso_noise_r(seed, t, idx))


def noise_field(seed: int, t: int, shape, impl=None) -> np.ndarray:
    n = int(np.prod(shape))
    r = np.empty(n, dtype=np.float64)
    lib(impl).gso_noise_field(seed, t, n, _dp(r))
    return r.reshape(shape)


def init_cube(L=None, side=12, cu=0.25, cv=0.33, shape=None, impl=None):
    """Initial state: u=1, v=0, plus a centred cube of side `side` at (cu, cv)."""
    if shape is None:
        shape = (L, L, L)
    nz, ny, nx = shape
    u = np.empty(shape, dtype=np.float64)
    v = np.empty(shape, dtype=np.float64)
    lib(impl).gso_init_cube(nx, ny, nz, side, cu, cv, _dp(u), _dp(v))
    return u, v


def laplacian(f: np.ndarray, impl=None) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    out = np.empty_like(f)
    lib(impl).gso_laplacian(nx, ny, nz, _dp(f), _dp(out))
    return out


def step(u, v, *, Du, Dv, F, k, dt, noise=0.0, seed=0, t=0, impl=None):
    """One step; returns new (u, v) arrays."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    nz, ny, nx = u.shape
    un, vn = np.empty_like(u), np.empty_like(v)
    lib(impl).gso_step(nx, ny, nz, Du, Dv, F, k, dt, noise, seed, t, _dp(u), _dp(v), _dp(un), _dp(vn))
    return un, vn


def run(u, v, n_steps, *, Du, Dv, F, k, dt, noise=0.0, seed=0, step0=0, impl=None, **_ignored):
    """n_steps steps from global step step0; returns new (u, v) arrays."""
    u = np.array(u, dtype=np.float64, order="C", copy=True)
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    nz, ny, nx = u.shape
    rc = lib(impl).gso_run(nx, ny, nz, Du, Dv, F, k, dt, noise, seed, step0, int(n_steps), _dp(u), _dp(v))
    if rc != 0:
        raise MemoryError("oracle scratch allocation failed")
    return u, v


def extract_window(f: np.ndarray, x0: int, y0: int, z0: int, w: int) -> np.ndarray:
    """w^3 periodic window of a (nz, ny, nx) field with lower corner (x0, y0, z0)."""
    nz, ny, nx = f.shape
    zi = (z0 + np.arange(w)) % nz
    yi = (y0 + np.arange(w)) % ny
    xi = (x0 + np.arange(w)) % nx
    return np.ascontiguousarray(f[np.ix_(zi, yi, xi)])


def run_window(uw, vw, grid_shape, corner, n_steps, *, Du, Dv, F, k, dt, noise=0.0, seed=0, step0=0,
               impl=None, **_ignored):
    """Advance a w^3 window (see gso_run_window); returns new (u, v) windows
    whose cells at least n_steps from every face are exact."""
    uw = np.array(uw, dtype=np.float64, order="C", copy=True)
    vw = np.array(vw, dtype=np.float64, order="C", copy=True)
    w = uw.shape[0]
    assert uw.shape == (w, w, w) == vw.shape
    nz, ny, nx = grid_shape
    x0, y0, z0 = corner
    rc = lib(impl).gso_run_window(nx, ny, nz, x0, y0, z0, w, Du, Dv, F, k, dt, noise, seed, step0,
                                  int(n_steps), _dp(uw), _dp(vw))
    if rc != 0:
        raise MemoryError("oracle scratch allocation failed")
    return uw, vw


def diagnostics(u: np.ndarray, v: np.ndarray) -> dict:
    """Exactly rounded sums (math.fsum), min/max and non-finite count."""
    uf, vf = u.ravel(), v.ravel()
    nonfinite = int(np.count_nonzero(~np.isfinite(uf)) + np.count_nonzero(~np.isfinite(vf)))
    return dict(sum_u=math.fsum(uf.tolist()), sum_v=math.fsum(vf.tolist()),
                min_u=float(np.min(uf)), max_u=float(np.max(uf)),
                min_v=float(np.min(vf)), max_v=float(np.max(vf)), nonfinite=nonfinite)
