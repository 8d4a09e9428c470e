"""Batched persistent sweeps against the FP64 oracle run per simulation."""
import numpy as np
import pytest

from oracle import oracle as O
from synth import batch_sweep
from tests.gpu_util import max_abs, require_gpu

pytestmark = pytest.mark.gpu

SHARED = dict(Du=0.2, Dv=0.1, dt=1.0)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _oracle(sim, i, n, noise=0.0, seed=0, side=12):
    shape = (sim.get("nz", sim.get("L")), sim.get("ny", sim.get("L")), sim.get("nx", sim.get("L")))
    u0, v0 = O.init_cube(shape=shape, side=side)
    return O.run(u0, v0, n, F=sim["F"], k=sim["k"], noise=noise, seed=seed + i, **SHARED)


def test_batch_mixed_sizes_bitwise(torch):
    """Uneven grids, own F and k each, noise keyed per simulation (seed + i);
    step counts that are not multiples of the fused depth."""
    from paper_2309_10292_amd import gs
    sims = [dict(nx=32, ny=32, nz=32, F=0.02, k=0.048), dict(nx=48, ny=40, nz=36, F=0.035, k=0.06),
            dict(nx=16, ny=20, nz=24, F=0.05, k=0.065), dict(nx=64, ny=24, nz=70, F=0.012, k=0.045)]
    for T in (1, 2, 3):
        for tile in gs.tblock_tiles():
            if T > gs.max_tblock(tile, "f64", batch=True):
                continue
            with gs.Batch(sims, noise=1e-3, seed=100, cube_side=8, tile=tile, tblock=T, zchunk=16, **SHARED) as b:
                b.step(7)
                for i, sm in enumerate(sims):
                    u, v = b.read(i)
                    ue, ve = _oracle(sm, i, 7, noise=1e-3, seed=100, side=8)
                    assert np.array_equal(u, ue) and np.array_equal(v, ve), (T, tile, i, max_abs(u, ue))


def test_batch_graph_and_tune(torch):
    """The autotuner picks a configuration per grid size without changing any
    state; graph replays (with eager steps between them) then match the oracle."""
    from paper_2309_10292_amd import gs
    sims = [dict(L=32, F=0.02, k=0.048), dict(L=48, F=0.03, k=0.055), dict(L=32, F=0.045, k=0.06),
            dict(L=64, F=0.025, k=0.05)]
    with gs.Batch(sims, cube_side=10, noise=1e-4, seed=5, **SHARED) as b:
        b.step(3)
        before = [b.read(i) for i in range(len(sims))]
        table = b.tune(reps=1)
        assert {(e["nx"], e["n_sims"]) for e in table} == {(32, 2), (48, 1), (64, 1)}
        for i in range(len(sims)):
            u, v = b.read(i)
            assert np.array_equal(u, before[i][0]) and np.array_equal(v, before[i][1])
        for rep in range(3):
            b.step_graph(5)
            b.step(1)
            torch.cuda.synchronize()
        for i, sm in enumerate(sims):
            u, v = b.read(i)
            ue, ve = _oracle(sm, i, 3 + 3 * 6, noise=1e-4, seed=5, side=10)
            assert np.array_equal(u, ue) and np.array_equal(v, ve), i


def test_batch_sweep_sample_bitwise(torch):
    """A sample of the (F, k) sweep's simulations (sizes 32..192) for 10
    steps, with the library's default configuration."""
    from paper_2309_10292_amd import gs
    sims = batch_sweep(12, seed=3)
    with gs.Batch(sims, **SHARED) as b:
        b.step(10)
        for i in (0, 5, 11):
            u, v = b.read(i)
            ue, ve = _oracle(sims[i], i, 10)
            assert np.array_equal(u, ue) and np.array_equal(v, ve), i
        d = b.diagnostics(3)
        e = O.diagnostics(*_oracle(sims[3], 3, 10))
        assert abs(d["sum_u"] - e["sum_u"]) <= 1e-13 * abs(e["sum_u"])
