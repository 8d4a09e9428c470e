"""GPU parity of the fused step (libgs through its C ABI) against the FP64
oracle. FP64 storage must match bit for bit (the contract is max-abs 1e-12
after 100 steps; the kernels follow the oracle's operation order, so the
expected difference is exactly zero)."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import random_state, subnormal_field, workload
from tests.gpu_util import max_abs, require_gpu, window_from_device

pytestmark = pytest.mark.gpu

P0 = {k: workload("small_l64")[k] for k in ("Du", "Dv", "F", "k", "dt")}


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def small_ref():
    p = workload("small_l64")
    u0, v0 = O.init_cube(L=p["L"], side=p["cube_side"], cu=p["cube_u"], cv=p["cube_v"])
    return O.run(u0, v0, p["steps"], **p)


def _sim(shape, **kw):
    from paper_2309_10292_amd import gs
    nz, ny, nx = shape
    return gs.Sim(nx, ny, nz, **kw)


def test_init_cube_matches_oracle(torch):
    for storage in ("f64",):
        with _sim((64, 64, 64), storage=storage, cube_side=12) as s:
            u, v = s.read()
        ue, ve = O.init_cube(L=64, side=12)
        assert np.array_equal(u, ue) and np.array_equal(v, ve)
    with _sim((20, 16, 24), cube_side=5, cube_u=0.4, cube_v=0.2) as s:
        u, v = s.read()
    ue, ve = O.init_cube(shape=(20, 16, 24), side=5, cu=0.4, cv=0.2)
    assert np.array_equal(u, ue) and np.array_equal(v, ve)


def test_small_l64_fp64_bitwise(torch, small_ref):
    p = workload("small_l64")
    from paper_2309_10292_amd import gs
    L = gs.load()
    for tile in range(0, L.gs_num_tiles() + 1):
        with _sim((64, 64, 64), storage="f64", tile=tile, **P0) as s:
            s.step(p["steps"])
            u, v = s.read()
        err = max(max_abs(u, small_ref[0]), max_abs(v, small_ref[1]))
        assert err <= 1e-12, f"tile {tile}: max-abs {err}"
        assert np.array_equal(u, small_ref[0]) and np.array_equal(v, small_ref[1]), f"tile {tile} not bitwise"


@pytest.mark.parametrize("shape", [(4, 4, 8), (20, 36, 40), (9, 13, 24), (6, 20, 136), (70, 5, 16)])
def test_ragged_shapes_with_noise_bitwise(torch, shape):
    from paper_2309_10292_amd import gs
    u0, v0 = random_state(shape, seed=sum(shape), lo_u=0.2, hi_u=1.0, lo_v=0.0, hi_v=0.5)
    p = dict(Du=0.19, Dv=0.11, F=0.029, k=0.055, dt=0.9, noise=0.01, seed=31337, step0=123)
    ue, ve = O.run(u0, v0, 5, **p)
    for tile in range(1, gs.load().gs_num_tiles() + 1):
        with _sim(shape, u0=u0, v0=v0, tile=tile, **p) as s:
            s.step(5)
            u, v = s.read()
        assert np.array_equal(u, ue) and np.array_equal(v, ve), f"shape {shape} tile {tile}: {max_abs(u, ue)}"


def test_noise_config_bitwise(torch):
    """The noisy workload's parameters (noise 1e-7) and a stronger noise on an
    L=64 grid from the cube state, 40 steps."""
    for noise in (1e-7, 0.05):
        p = dict(workload("weak_share_l512"))
        p.update(noise=noise)
        u0, v0 = O.init_cube(L=64)
        ue, ve = O.run(u0, v0, 40, **p)
        with _sim((64, 64, 64), **{k: p[k] for k in ("Du", "Dv", "F", "k", "dt", "noise", "seed")}) as s:
            s.step(40)
            u, v = s.read()
        assert np.array_equal(u, ue) and np.array_equal(v, ve), (noise, max_abs(u, ue))


def _bits_equal(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint64), np.ascontiguousarray(b).view(np.uint64))


@pytest.mark.parametrize("Dv,dt,noise", [(0.5, 1.0, 0.0), (1.0, 0.9, 0.0), (0.5, 1.0, 1e-200)])
def test_fp64_subnormal_states_bitwise(torch, Dv, dt, noise):
    """FP64 from states whose v is subnormal (m 2^-1074, m < 2^20, the decayed
    tails of a field), with u = 0 and with u random, and from a state whose u
    is subnormal too, in the single-step kernel and the blocked kernel with one
    and three fused steps, bit for bit against the oracle. About one in twelve
    such Laplacian numerators is an odd multiple of 3 2^-1074, whose quotient
    by 6 is a tie of the subnormal grid that only the true division rounds to
    even (Eq. 3 divides by 6). The case with noise (1e-200, added to u) runs
    the noise kernels too, among them the three-step one that prefetches
    through LDS."""
    from paper_2309_10292_amd import gs
    shape = (12, 20, 40)
    n = 7
    p = dict(Du=0.2, Dv=Dv, F=0.02, k=0.048, dt=dt, noise=noise, seed=31)
    tiles = [(1, 1)] + [(t, T) for t in gs.tblock_tiles() for T in (1, 3) if T <= gs.max_tblock(t, "f64")]
    v0 = subnormal_field(shape, seed=int(Dv * 10))
    u_rand, _ = random_state(shape, seed=5, lo_u=0.2, hi_u=1.0)
    for case, u0 in (("u=0", np.zeros(shape)), ("u random", u_rand),
                     ("u subnormal", subnormal_field(shape, seed=99))):
        ue, ve = O.run(u0, v0, n, **p)
        assert np.count_nonzero(ve) > 0  # the tails have not all flushed to zero
        for tile, T in tiles:
            with _sim(shape, u0=u0, v0=v0, tile=tile, tblock=T, **p) as s:
                s.step(n)
                u, v = s.read()
            assert _bits_equal(u, ue) and _bits_equal(v, ve), \
                f"{case} Dv={Dv} tile={tile} T={T}: {np.count_nonzero(u != ue)} u, {np.count_nonzero(v != ve)} v cells differ"


def test_resume_bitwise(torch):
    p = dict(P0, noise=0.02, seed=99)
    with _sim((32, 32, 32), cube_side=10, **p) as s:
        s.step(30)
        u_full, v_full = s.read()
    with _sim((32, 32, 32), cube_side=10, **p) as s:
        s.step(15)
        u_mid, v_mid = s.read()
        _, _, st = s.current()
        assert st == 15
    with _sim((32, 32, 32), u0=u_mid, v0=v_mid, step0=15, **p) as s:
        s.step(15)
        u2, v2 = s.read()
    assert np.array_equal(u_full, u2) and np.array_equal(v_full, v2)


def test_step_zero_and_split_calls(torch):
    """gs_step(0) is a no-op; gs_step(a) + gs_step(b) == gs_step(a + b)."""
    with _sim((24, 24, 32), noise=1e-3, seed=5, **P0) as s:
        s.step(0)
        s.step(3)
        s.step(4)
        a = s.read()
    with _sim((24, 24, 32), noise=1e-3, seed=5, **P0) as s:
        s.step(7)
        b = s.read()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_deterministic_repeat(torch):
    """Two runs give the same bits (a race in LDS staging would show here)."""
    outs = []
    for _ in range(2):
        with _sim((64, 96, 128), noise=1e-4, seed=3, cube_side=30, **P0) as s:
            s.step(25)
            outs.append(s.read())
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_fixed_point_all_storage_types(torch):
    for storage in ("f64", "f32", "bf16", "f16", "bf16c"):
        with _sim((16, 16, 16), storage=storage, cube_side=1, cube_u=1.0, cube_v=0.0, **P0) as s:
            s.step(10)
            u, v = s.read()
        assert np.all(u == 1.0) and np.all(v == 0.0), storage


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_16bit_rounding_ties_to_even(torch, storage):
    """16-bit storage rounds FP32 to nearest, ties to even, on the device:
    cube values exactly halfway between two neighbours of the format land on
    the one with the even significand, and a value just above a tie rounds
    up."""
    def rne(x):
        if storage == "f16":
            return float(np.float16(np.float32(x)))
        b = int(np.array([x], dtype=np.float32).view(np.uint32)[0])
        b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
        return float(np.array([b << 16], dtype=np.uint32).view(np.float32)[0])

    h = 2.0 ** -8 if storage == "bf16" else 2.0 ** -11  # half the spacing just above 1
    cases = [(1 + h, 1 + 3 * h),                  # ties: 1 and 1 + 4h
             (1 + h + 2.0 ** -20, 0.25 + h / 4)]  # just above a tie: 1 + 2h; a tie at 0.25: 0.25
    expect = [(1.0, 1 + 4 * h), (1 + 2 * h, 0.25)]
    for (cu, cv), (eu, ev) in zip(cases, expect):
        assert (rne(cu), rne(cv)) == (eu, ev)
        with _sim((16, 16, 16), storage=storage, cube_side=4, cube_u=cu, cube_v=cv) as s:
            u, v = s.read()
        c = slice(6, 10)
        assert np.all(u[c, c, c] == eu) and np.all(v[c, c, c] == ev), (storage, cu, cv)
        assert np.all(u[:6] == 1.0) and np.all(v[:6] == 0.0)


def test_bf16c_stores_the_complement_of_u(torch):
    """The complemented BF16 storage keeps 1 - u: u = 1 - 3 2^-12 (1 - u has
    two significant bits) survives the cube initialisation, a host write and
    read, and the diagnostics exactly, where plain BF16 (steps of 2^-9 below
    1) rounds it to 1; v is plain BF16."""
    cu, cv = 1.0 - 3 * 2.0 ** -12, 0.25
    with _sim((16, 16, 16), storage="bf16", cube_side=4, cube_u=cu, cube_v=cv) as s:
        u, _ = s.read()
    assert u[8, 8, 8] == 1.0
    with _sim((16, 16, 16), storage="bf16c", cube_side=4, cube_u=cu, cube_v=cv) as s:
        u, v = s.read()
        c = slice(6, 10)
        assert np.all(u[c, c, c] == cu) and np.all(v[c, c, c] == cv)
        assert np.all(u[:6] == 1.0) and np.all(v[:6] == 0.0)
        ut, vt, _ = s.current()  # the raw u buffer holds 1 - u
        raw = ut.float().cpu().numpy()
        assert np.all(raw[c, c, c] == 3 * 2.0 ** -12) and np.all(raw[:6] == 0.0)
        d = s.diagnostics()
        assert d["min_u"] == cu and d["max_u"] == 1.0 and d["max_v"] == cv
        assert d["sum_u"] == 16 ** 3 - 64 * 3 * 2.0 ** -12
        w = np.full((16, 16, 16), 1.0 - 5 * 2.0 ** -14)
        s.write(w, v)
        u2, v2 = s.read()
        assert np.array_equal(u2, w) and np.array_equal(v2, v)


def test_diagnostics_vs_oracle(torch, small_ref):
    p = workload("small_l64")
    with _sim((64, 64, 64), **P0) as s:
        s.step(p["steps"])
        d = s.diagnostics()
        u_t, v_t, _ = s.current()
        e = O.diagnostics(*small_ref)
        for key in ("sum_u", "sum_v"):
            assert abs(d[key] - e[key]) <= 1e-14 * abs(e[key]), key
        for key in ("min_u", "max_u", "min_v", "max_v"):
            assert d[key] == e[key], key
        assert d["nonfinite"] == 0
        # a non-finite value written by the caller is counted and reported
        u_t.view(-1)[12345] = float("nan")
        v_t.view(-1)[7] = float("inf")
        torch.cuda.synchronize()
        from paper_2309_10292_amd import gs
        with pytest.raises(gs.GSError) as ei:
            s.diagnostics()
        assert ei.value.status == gs.GS_ERR_NONFINITE
        d2 = s.diagnostics(allow_nonfinite=True)
        assert d2["nonfinite"] == 2


def test_reduced_precision_within_bars(torch, small_ref):
    """FP32 / FP16 / BF16 storage (FP32 arithmetic) on
    the L=64 workload, 100 steps, against the FP64 oracle."""
    bars = {"f32": 1e-5, "f16": 5e-3, "bf16": 5e-2, "bf16c": 5e-2}
    p = workload("small_l64")
    for storage, bar in bars.items():
        with _sim((64, 64, 64), storage=storage, **P0) as s:
            s.step(p["steps"])
            u, v = s.read()
        err = max(max_abs(u, small_ref[0]), max_abs(v, small_ref[1]))
        print(f"{storage}: max-abs {err:.3e}")
        assert err <= bar, (storage, err)


def test_reduced_precision_with_noise_l64(torch):
    """FP32 / FP16 / BF16 storage with the noise term on (n = 1e-3, Philox
    keyed as in FP64), L=64 cube state, 100 steps, against the FP64 oracle.
    The storage types round the noise like every other update: FP32 keeps it
    to about 1e-7 of u near 1, FP16 to half of 2^-10 and BF16 to half of 2^-7,
    so the bars are those of the noise-free L=64 run."""
    bars = {"f32": 1e-5, "f16": 5e-3, "bf16": 5e-2, "bf16c": 5e-2}
    p = dict(workload("small_l64"), noise=1e-3, seed=77)
    u0, v0 = O.init_cube(L=64)
    ue, ve = O.run(u0, v0, p["steps"], **p)
    kw = {k: p[k] for k in ("Du", "Dv", "F", "k", "dt", "noise", "seed")}
    for storage, bar in bars.items():
        with _sim((64, 64, 64), storage=storage, **kw) as s:
            s.step(p["steps"])
            u, v = s.read()
        err = max(max_abs(u, ue), max_abs(v, ve))
        print(f"{storage} with noise: max-abs {err:.3e}")
        assert err <= bar, (storage, err)


def test_laplacian7_bitwise(torch):
    from paper_2309_10292_amd import gs
    for shape in [(24, 40, 64), (5, 7, 16), (33, 17, 200)]:
        f = np.random.default_rng(len(shape)).uniform(-1, 1, size=shape)
        ft = torch.from_numpy(f).cuda()
        out = gs.laplacian7(ft)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), O.laplacian(f)), shape


def test_copy_kernel(torch):
    from paper_2309_10292_amd import gs
    a = torch.randint(0, 255, (1 << 20,), dtype=torch.uint8, device="cuda")
    b = torch.zeros_like(a)
    gs.copy(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def _sampled_windows(s_state_prev, s_state_now, shape, p, step_prev, n, corners, w=16):
    (up, vp), (un, vn) = s_state_prev, s_state_now
    p = {k: p[k] for k in ("Du", "Dv", "F", "k", "dt", "noise", "seed")}
    for corner in corners:
        uw = window_from_device(up, *corner, w)
        vw = window_from_device(vp, *corner, w)
        ue, ve = O.run_window(uw, vw, shape, corner, n, step0=step_prev, **p)
        inner = slice(n, w - n)
        ug = window_from_device(un, *corner, w)[inner, inner, inner]
        vg = window_from_device(vn, *corner, w)[inner, inner, inner]
        assert np.array_equal(ug, ue[inner, inner, inner]), (corner, max_abs(ug, ue[inner, inner, inner]))
        assert np.array_equal(vg, ve[inner, inner, inner]), corner


def test_full_size_l512_noise(torch):
    """One GPU's weak-scaling share, L=512, noise 1e-7, 1000 steps, in the
    launch configuration the benchmark times: the first two steps are
    compared over the whole field, the last five on sampled windows (cells
    evaluated one by one by the oracle from the GPU's own state at step 995,
    covering the cube's centre, its edge, quiet cells and the periodic seam)."""
    p = workload("weak_share_l512")
    L = p["L"]
    shape = (L, L, L)
    kw = {k: p[k] for k in ("Du", "Dv", "F", "k", "dt", "noise", "seed")}
    with _sim(shape, **kw) as s:
        s.step(2)
        u, v = s.read()
        u0, v0 = O.init_cube(L=L)
        ue, ve = O.run(u0, v0, 2, **p)
        assert np.array_equal(u, ue) and np.array_equal(v, ve), max_abs(u, ue)
        del u, v, ue, ve, u0, v0
        s.step(p["steps"] - 2 - 5)
        u_t, v_t, st = s.current()
        assert st == p["steps"] - 5
        prev = (u_t.clone(), v_t.clone())
        s.step(5)
        u_t, v_t, st = s.current()
        assert st == p["steps"]
        corners = [(248, 248, 248), (240, 250, 260), (0, 0, 0), (505, 505, 505), (100, 300, 200), (500, 3, 255)]
        _sampled_windows(prev, (u_t, v_t), shape, dict(p), p["steps"] - 5, 5, corners)


def test_full_size_l1024_fp64_sampled(torch):
    """The L=1024 precision workload in FP64 (F=0.03, k=0.06, 200 steps):
    sampled windows for the last four steps against the oracle."""
    p = workload("precision_l1024")
    L = p["L"]
    shape = (L, L, L)
    kw = {k: p[k] for k in ("Du", "Dv", "F", "k", "dt", "noise")}
    with _sim(shape, **kw) as s:
        s.step(p["steps"] - 4)
        u_t, v_t, _ = s.current()
        prev = (u_t.clone(), v_t.clone())
        s.step(4)
        u_t, v_t, st = s.current()
        assert st == p["steps"]
        c = (L - 12) // 2
        corners = [(c, c, c), (c - 8, c + 4, c - 2), (c + 10, c - 10, c + 5), (0, 0, 0), (1016, 1016, 1016)]
        _sampled_windows(prev, (u_t, v_t), shape, dict(p), p["steps"] - 4, 4, corners)
        del prev


def tb_tiles():
    from paper_2309_10292_amd import gs
    return gs.tblock_tiles()


def max_T(tile, storage):
    from paper_2309_10292_amd import gs
    return gs.max_tblock(tile, storage)


@pytest.mark.parametrize("zc", [3, 8, 16])
@pytest.mark.parametrize("T", [1, 2, 3, 4])
def test_tblock_bitwise_vs_oracle(torch, T, zc):
    """The temporally blocked kernel (T steps per pass, every shape) against the
    oracle on ragged periodic grids with noise; step counts that are not
    multiples of T exercise the remainder launch, and z-chunks shorter than
    T (3 planes) the wavefront's prologue and epilogue overlapping."""
    for shape in [(20, 36, 40), (9, 13, 24), (70, 5, 16), (4, 4, 8)]:
        u0, v0 = random_state(shape, seed=7 * T + sum(shape), lo_u=0.2, hi_u=1.0, lo_v=0.0, hi_v=0.5)
        p = dict(Du=0.19, Dv=0.11, F=0.029, k=0.055, dt=0.9, noise=0.01, seed=4242, step0=77)
        n = 2 * T + 1
        ue, ve = O.run(u0, v0, n, **p)
        for tile in tb_tiles():
            if T > max_T(tile, "f64"):
                continue
            with _sim(shape, u0=u0, v0=v0, tile=tile, tblock=T, zchunk=zc, **p) as s:
                s.step(n)
                u, v = s.read()
            assert np.array_equal(u, ue) and np.array_equal(v, ve), \
                f"T={T} zc={zc} tile={tile} shape={shape}: {max_abs(u, ue)} {max_abs(v, ve)}"


def test_tblock_small_l64_fp64_bitwise(torch, small_ref):
    p = workload("small_l64")
    for T in (1, 2, 4):
        for tile in tb_tiles():
            if T > max_T(tile, "f64"):
                continue
            with _sim((64, 64, 64), tile=tile, tblock=T, **P0) as s:
                s.step(p["steps"])
                u, v = s.read()
            assert np.array_equal(u, small_ref[0]) and np.array_equal(v, small_ref[1]), (T, tile)


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16", "bf16c"])
def test_tblock_reduced_precision_equals_single_step(torch, storage):
    """Reduced-precision storage: T fused steps round every intermediate level
    to the storage type, so they equal T single-step sweeps bit for bit."""
    shape = (24, 40, 48)
    p = dict(P0, noise=1e-3, seed=11)
    with _sim(shape, storage=storage, tile=1, cube_side=10, **p) as s:
        s.step(9)
        ref = s.current()
        ref = (ref[0].clone(), ref[1].clone())
    for tile in tb_tiles():
        for T in range(2, max_T(tile, storage) + 1):
            with _sim(shape, storage=storage, tile=tile, tblock=T, cube_side=10, **p) as s:
                s.step(9)
                u_t, v_t, st = s.current()
                assert st == 9
                assert torch.equal(u_t, ref[0]) and torch.equal(v_t, ref[1]), (storage, tile, T)


def test_tblock_full_size_l512_noise(torch):
    """The benchmarked configuration class at full size: L=512, noise 1e-7,
    T=2 temporally blocked sweeps; 10 steps compared over the whole field."""
    p = workload("weak_share_l512")
    L = p["L"]
    kw = {k: p[k] for k in ("Du", "Dv", "F", "k", "dt", "noise", "seed")}
    with _sim((L, L, L), tile=5, tblock=2, **kw) as s:
        s.step(10)
        u, v = s.read()
    u0, v0 = O.init_cube(L=L)
    ue, ve = O.run(u0, v0, 10, **p)
    assert np.array_equal(u, ue) and np.array_equal(v, ve), max_abs(u, ue)


def test_graph_replay_matches_eager(torch):
    """gs_step_graph: several replays of one captured graph, with eager work
    and synchronisations between them, each checked against eager stepping
    (noise on, so a wrong step index in a replay would show)."""
    shape = (32, 40, 48)
    p = dict(P0, noise=0.01, seed=8)
    for tile, T in ((1, 1), (6, 3), (5, 2)):
        with _sim(shape, tile=tile, tblock=T, cube_side=12, **p) as eager, \
                _sim(shape, tile=tile, tblock=T, cube_side=12, **p) as g:
            for rep in range(4):
                eager.step(7)
                g.step_graph(7)
                a, b = eager.current(), g.current()
                assert a[2] == b[2]
                assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), (tile, T, rep)
                # eager work on the graph's handle between replays
                g.step(1)
                eager.step(1)
                torch.cuda.synchronize()
            ue, ve = eager.read()
        u0, v0 = O.init_cube(shape=shape, side=12)
        uo, vo = O.run(u0, v0, 32, **p)
        assert np.array_equal(ue, uo) and np.array_equal(ve, vo)


def test_tune_leaves_state_and_picks_valid_config(torch):
    shape = (64, 64, 128)
    p = dict(P0, noise=1e-3, seed=21)
    with _sim(shape, cube_side=20, **p) as s:
        s.step(3)
        before = s.read()
        cfg, rows = s.tune(reps=1)
        after = s.read()
        assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
        assert s.current()[2] == 3
        assert len(rows) > 10 and all(r["ms_per_step"] > 0 for r in rows)
        best = min(rows, key=lambda r: r["ms_per_step"])
        assert (cfg["tile"], cfg["tblock"], cfg["zchunk"]) == (best["tile"], best["tblock"], best["zchunk"])
        s.step(5)
        u, v = s.read()
    u0, v0 = O.init_cube(shape=shape, side=20)
    ue, ve = O.run(u0, v0, 8, **p)
    assert np.array_equal(u, ue) and np.array_equal(v, ve)


def test_tune_cache_roundtrip(torch, tmp_path, monkeypatch):
    """With GS_TUNE_CACHE set, gs_tune records its choice and a new handle for
    the same grid class starts with it; gs_batch_tune does the same per grid
    class of a batch. The recorded configurations give the oracle's result."""
    import json
    from paper_2309_10292_amd import gs
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("GS_TUNE_CACHE", str(cache))
    shape = (32, 40, 64)
    p = dict(P0, noise=1e-3, seed=8)
    with _sim(shape, cube_side=10, **p) as s:
        cfg, _ = s.tune(reps=1)
    entries = [json.loads(l) for l in cache.read_text().splitlines()]
    assert len(entries) == 1
    e = entries[0]
    assert (e["kind"], e["storage"], e["nx"], e["ny"], e["nz"], e["noise"]) == ("single", 0, 64, 40, 32, 1)
    assert (e["tile"], e["tblock"], e["zchunk"]) == (cfg["tile"], cfg["tblock"], cfg["zchunk"])
    with _sim(shape, cube_side=10, **p) as s:
        assert s.config() == cfg
        s.step(7)
        u, v = s.read()
    u0, v0 = O.init_cube(shape=shape, side=10)
    ue, ve = O.run(u0, v0, 7, **p)
    assert np.array_equal(u, ue) and np.array_equal(v, ve)
    # batched: one entry per grid class, used by a new batch
    sims = [dict(L=32, F=0.02, k=0.048), dict(L=48, F=0.03, k=0.055), dict(L=32, F=0.045, k=0.06)]
    with gs.Batch(sims, cube_side=8, Du=0.2, Dv=0.1, dt=1.0) as b:
        table = b.tune(reps=1)
        chosen = {e["nx"]: (e["tile"], e["tblock"], e["zchunk"]) for e in table}
    entries = [json.loads(l) for l in cache.read_text().splitlines()]
    batch = {e["nx"]: (e["tile"], e["tblock"], e["zchunk"]) for e in entries if e["kind"] == "batch"}
    assert batch == chosen and len(entries) == 3
    with gs.Batch(sims, cube_side=8, Du=0.2, Dv=0.1, dt=1.0) as b:
        for i, sm in enumerate(sims):
            c = b.config(i)
            assert (c["tile"], c["tblock"], c["zchunk"]) == chosen[sm["L"]]
