"""The FP64 oracle against closed forms, invariants, a dense brute force and an
independent Philox (see tests/pins.py for what each check rests on)."""
import math

import numpy as np
import pytest

from tests import pins


@pytest.mark.parametrize("check", pins.ALL, ids=[f.__name__ for f in pins.ALL])
def test_pin(check):
    check()


def test_noise_statistics(oracle):
    """r is uniform on (-1, 1): mean 0, variance 1/3, KS test, open endpoints."""
    from scipy import stats
    r = oracle.noise_field(230910292, 7, (1 << 18,)).ravel()
    assert np.all(r > -1.0) and np.all(r < 1.0)
    assert abs(r.mean()) < 5e-3
    assert abs(r.var() - 1.0 / 3.0) < 5e-3
    assert stats.kstest(r, "uniform", args=(-1.0, 2.0)).pvalue > 1e-3
    # consecutive steps and seeds give uncorrelated fields
    r2 = oracle.noise_field(230910292, 8, (1 << 18,)).ravel()
    assert abs(np.corrcoef(r, r2)[0, 1]) < 0.01


def test_run_composition_with_noise(oracle):
    """n steps == a steps then n-a steps resumed at step index a (noise keyed by
    the global step), bit for bit."""
    u0, v0 = oracle.init_cube(L=16, side=6)
    p = dict(Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1.0, noise=0.05, seed=42)
    u, v = oracle.run(u0, v0, 12, **p)
    ua, va = oracle.run(u0, v0, 5, **p)
    ub, vb = oracle.run(ua, va, 7, step0=5, **p)
    assert np.array_equal(u, ub) and np.array_equal(v, vb)


def test_laplacian_matches_roll_sum(oracle):
    """Single-field Laplacian against the same stencil built from np.roll."""
    f = np.random.default_rng(1).uniform(-1, 1, size=(6, 7, 9))
    s = sum(np.roll(f, d, axis=a) for a in range(3) for d in (1, -1))
    err = np.max(np.abs(oracle.laplacian(f) - (s - 6 * f) / 6))
    assert err <= 2e-15


def test_threads_do_not_change_result(oracle):
    u0, v0 = oracle.init_cube(L=24, side=8)
    p = dict(Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1.0, noise=1e-3, seed=5)
    n0 = oracle.max_threads()
    oracle.set_threads(1)
    a = oracle.run(u0, v0, 10, **p)
    oracle.set_threads(max(2, n0))
    b = oracle.run(u0, v0, 10, **p)
    oracle.set_threads(n0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_window_matches_periodic_run(oracle):
    """Cells evaluated one window at a time (noise keyed by global index) equal
    the same cells of the whole periodic run, including windows that wrap."""
    shape = (20, 18, 24)
    u0, v0 = np.random.default_rng(9).uniform(0.1, 0.9, size=(2,) + shape)
    p = dict(Du=0.2, Dv=0.1, F=0.03, k=0.05, dt=0.9, noise=0.02, seed=77, step0=11)
    n = 4
    u, v = oracle.run(u0, v0, n, **p)
    for corner in [(0, 0, 0), (20, 15, 17), (5, 7, 3)]:
        w = 14
        uw, vw = oracle.run_window(oracle.extract_window(u0, *corner, w), oracle.extract_window(v0, *corner, w),
                                   shape, corner, n, **p)
        inner = slice(n, w - n)
        ue = oracle.extract_window(u, *corner, w)[inner, inner, inner]
        ve = oracle.extract_window(v, *corner, w)[inner, inner, inner]
        assert np.array_equal(uw[inner, inner, inner], ue) and np.array_equal(vw[inner, inner, inner], ve)
