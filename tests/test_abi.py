"""C ABI checks that need no GPU: the library loads, exports every entry point
include/gs.h declares, its structs have the header's layout, and argument
validation returns the documented status before any HIP call."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2309_10292_amd import gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(gs_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_and_library_exports_everything():
    L = gs.load()
    names = declared_functions()
    assert "gs_init" in names and "gs_step" in names and "gs_read" in names
    for n in names:
        assert hasattr(L, n), f"libgs.so does not export {n}"
    bound = {s[0] for s in gs.SIGNATURES}
    assert set(names) <= bound, f"binding misses {set(names) - bound}"


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    fields = [f[0] for f in gs.gs_params._fields_]
    dfields = [f[0] for f in gs.gs_diag._fields_]
    body = "\n".join(f'printf("p {f} %zu\\n", offsetof(gs_params, {f}));' for f in fields)
    body += "\n".join(f'printf("d {f} %zu\\n", offsetof(gs_diag, {f}));' for f in dfields)
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gs.h"\nint main(void){'
                    'printf("P %zu\\nD %zu\\n", sizeof(gs_params), sizeof(gs_diag));' + body + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I" + os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if not line:
            continue
        parts = line.split()
        got[tuple(parts[:-1])] = int(parts[-1])
    assert got[("P",)] == ctypes.sizeof(gs.gs_params)
    assert got[("D",)] == ctypes.sizeof(gs.gs_diag)
    for f in fields:
        assert got[("p", f)] == getattr(gs.gs_params, f).offset, f
    for f in dfields:
        assert got[("d", f)] == getattr(gs.gs_diag, f).offset, f


def _init_status(**kw):
    L = gs.load()
    shape = kw.pop("shape", (64, 64, 64))
    p = gs.make_params(*shape, **kw)
    h = ctypes.c_void_p(1234)
    st = L.gs_init(ctypes.byref(p), None, None, None, None, None, None, ctypes.byref(h))
    assert h.value is None, "out must be NULL on failure"
    return st, gs.last_error()


@pytest.mark.parametrize("kw,status", [
    (dict(shape=(63, 64, 64)), gs.GS_ERR_UNSUPPORTED),
    (dict(shape=(64, 3, 64)), gs.GS_ERR_UNSUPPORTED),
    (dict(shape=(64, 64, 2)), gs.GS_ERR_UNSUPPORTED),
    (dict(Du=float("nan")), gs.GS_ERR_INVALID_ARG),
    (dict(F=float("inf")), gs.GS_ERR_INVALID_ARG),
    (dict(dt=float("-inf")), gs.GS_ERR_INVALID_ARG),
    (dict(Dv=-0.1), gs.GS_ERR_INVALID_ARG),
    (dict(noise=-1e-7), gs.GS_ERR_INVALID_ARG),
    (dict(storage=7), gs.GS_ERR_INVALID_ARG),
    (dict(cube_side=0), gs.GS_ERR_INVALID_ARG),
    (dict(cube_side=65), gs.GS_ERR_INVALID_ARG),
    (dict(tblock=gs.MAX_TBLOCK + 1), gs.GS_ERR_INVALID_ARG),
    (dict(tile=99), gs.GS_ERR_INVALID_ARG),
    (dict(tile=1, tblock=2), gs.GS_ERR_INVALID_ARG),
    (dict(zchunk=-1), gs.GS_ERR_INVALID_ARG),
    (dict(), gs.GS_ERR_INVALID_ARG),  # valid params, NULL buffers
])
def test_init_validation(kw, status):
    st, msg = _init_status(**kw)
    assert st == status, msg
    assert msg


def test_misaligned_and_aliased_buffers():
    L = gs.load()
    p = gs.make_params(64, 64, 64)
    h = ctypes.c_void_p()
    st = L.gs_init(ctypes.byref(p), 4096 + 8, 8192, 12288, 16384, 20480, None, ctypes.byref(h))
    assert st == gs.GS_ERR_INVALID_ARG and "aligned" in gs.last_error()
    st = L.gs_init(ctypes.byref(p), 4096, 4096, 12288, 16384, 20480, None, ctypes.byref(h))
    assert st == gs.GS_ERR_INVALID_ARG and "aliases" in gs.last_error()


def test_null_handle_is_state_error():
    L = gs.load()
    assert L.gs_step(None, 1) == gs.GS_ERR_STATE
    assert L.gs_read(None, None, None) == gs.GS_ERR_STATE
    assert L.gs_write(None, None, None) == gs.GS_ERR_STATE
    assert L.gs_sync(None) == gs.GS_ERR_STATE
    assert L.gs_destroy(None) == gs.GS_ERR_STATE
    d = gs.gs_diag()
    assert L.gs_diagnostics(None, ctypes.byref(d)) == gs.GS_ERR_STATE
    assert L.gs_current(None, None, None, None) == gs.GS_ERR_STATE


def test_calibration_entry_points_validate():
    L = gs.load()
    assert L.gs_laplacian7(None, None, 64, 64, 64, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_laplacian7(4096, 8192, 60, 64, 64, None) == gs.GS_ERR_UNSUPPORTED
    assert gs.last_error() == "grid 60x64x64 unsupported (>= 4 each, nx % 8 == 0)"
    assert L.gs_laplacian7(4096, 4096, 64, 64, 64, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_copy(4096, 8192, 17, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_copy(None, 8192, 16, None) == gs.GS_ERR_INVALID_ARG


def test_workspace_and_tiles():
    p = gs.make_params(64, 64, 64)
    assert gs.workspace_bytes(p) > 0
    assert gs.workspace_bytes(gs.make_params(60, 64, 64)) == 0
    L = gs.load()
    n = L.gs_num_tiles()
    assert n >= 1
    for t in range(1, n + 1):
        for s in range(5):
            tx, ty, mt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            assert L.gs_tile_info(t, s, 1, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(mt)) == gs.GS_OK
            assert tx.value > 0 and ty.value > 0 and mt.value >= 1
            for T in range(1, mt.value + 1):
                assert L.gs_tile_info(t, s, T, ctypes.byref(tx), ctypes.byref(ty), None) == gs.GS_OK
                assert ty.value > 0
            assert L.gs_tile_info(t, s, mt.value + 1, None, None, None) == gs.GS_ERR_INVALID_ARG
    assert L.gs_tile_info(0, 0, 1, None, None, None) == gs.GS_ERR_INVALID_ARG


def test_batch_max_tblock():
    L = gs.load()
    n = L.gs_num_tiles()
    assert L.gs_batch_max_tblock(1, 0) == 0           # single-step tile
    assert L.gs_batch_max_tblock(n + 1, 0) == 0       # out of range
    assert L.gs_batch_max_tblock(5, 7) == 0           # unknown storage
    for t in range(5, n + 1):
        for s in range(4):
            mb = L.gs_batch_max_tblock(t, s)
            assert 0 <= mb <= gs.max_tblock(t, s) <= 4
    assert gs.max_tblock(6, "f64") == 4 and gs.max_tblock(6, "f64", batch=True) == 4
    # the complemented BF16 storage is for single grids only
    for t in range(5, n + 1):
        assert L.gs_batch_max_tblock(t, 4) == 0
        assert gs.max_tblock(t, "bf16c") == gs.max_tblock(t, "bf16")


def test_noise_below_bound_rejected():
    """Noise amplitudes in (0, 2^-990) would make the kernels' exactly scaled
    noise subnormal; gs_init rejects them before any HIP call."""
    import math
    L = gs.load()
    assert gs.workspace_bytes(gs.make_params(16, 16, 16, noise=math.ldexp(1.0, -990))) > 0
    p = gs.make_params(16, 16, 16, noise=math.ldexp(1.0, -1000))
    assert gs.workspace_bytes(p) == 0
    assert L.gs_init(ctypes.byref(p), None, None, None, None, None, None, ctypes.byref(ctypes.c_void_p())) == gs.GS_ERR_UNSUPPORTED


def test_tune_cache_lookup(tmp_path, monkeypatch):
    """gs_init takes a configuration recorded in the GS_TUNE_CACHE table for
    the same (storage, nx, ny, nz, noise on/off) when gs_params leaves the
    launch configuration to the library, and ignores entries for other keys,
    entries the library cannot run and malformed lines. (No HIP call: the
    state is not initialised and the handle is not destroyed.)"""
    L = gs.load()
    cache = tmp_path / "tune.jsonl"
    line = ('{{"kind":"{kind}","storage":{st},"nx":{nx},"ny":32,"nz":32,"noise":{nz},'
            '"tile":{t},"tblock":{T},"zchunk":{zc},"ms_per_step":0.1}}')
    cache.write_text("\n".join([
        "not json at all",
        line.format(kind="single", st=0, nx=64, nz=0, t=7, T=2, zc=8),    # used for the f64 64x32x32 grid
        line.format(kind="single", st=0, nx=64, nz=1, t=6, T=3, zc=16),   # same grid with noise
        line.format(kind="batch", st=0, nx=64, nz=0, t=5, T=1, zc=16),    # another kind
        line.format(kind="single", st=0, nx=32, nz=0, t=9, T=4, zc=8),    # tile 9 fuses at most 1 step in FP64
    ]) + "\n")
    monkeypatch.setenv("GS_TUNE_CACHE", str(cache))
    buf = ctypes.create_string_buffer(4096 + 256)
    base = (ctypes.addressof(buf) + 255) // 256 * 256
    ptrs = [ctypes.c_void_p(base + 256 * i) for i in range(5)]

    def config(nx, noise=0.0, tile=0):
        p = gs.make_params(nx, 32, 32, noise=noise, init="none", tile=tile)
        h = ctypes.c_void_p()
        assert L.gs_init(ctypes.byref(p), *ptrs[:4], ptrs[4], None, ctypes.byref(h)) == gs.GS_OK
        t, T, zc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert L.gs_get_config(h, ctypes.byref(t), ctypes.byref(T), ctypes.byref(zc)) == gs.GS_OK
        return t.value, T.value, zc.value

    assert config(64) == (7, 2, 8)
    assert config(64, noise=1e-7) == (6, 3, 16)
    default = config(48)                      # no entry
    assert config(32) == default              # unrunnable entry ignored
    assert config(64, tile=1)[0] == 1         # an explicit choice wins over the table
