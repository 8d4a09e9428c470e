"""Pins of the FP64 oracle: checks against facts fixed by the paper's
equations and by mathematics, not against the oracle itself.

Each check takes an optional oracle build `impl` (default: the real one) and
raises AssertionError on failure. tests/test_oracle_pins.py runs them on the
real oracle; tests/test_oracle_mutations.py runs them on deliberately broken
copies of the oracle source and requires every copy to be caught.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O
from tests import pyphilox


def _coords(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x, y, z


def _eig(shape, m):
    """Eigenvalue of the 7-point periodic Laplacian (sum - 6c)/6 for the Fourier
    mode with integer wave numbers m = (mx, my, mz): the discrete second
    difference of cos(theta j) is 2(cos theta - 1) cos(theta j)."""
    nz, ny, nx = shape
    th = (2 * math.pi * m[0] / nx, 2 * math.pi * m[1] / ny, 2 * math.pi * m[2] / nz)
    return (2 * math.cos(th[0]) + 2 * math.cos(th[1]) + 2 * math.cos(th[2]) - 6.0) / 6.0, th


def _mode(shape, th, phase=0.3):
    x, y, z = _coords(shape)
    return np.cos(th[0] * x + th[1] * y + th[2] * z + phase)


def fourier_u(impl=None, shape=(8, 10, 12), m=(1, 2, 3), Du=0.2, F=0.015, dt=0.8, n=30, eps=0.5):
    """Pure diffusion + feed on a u-mode: v = 0, u = 1 + eps*mode. The reaction
    vanishes, so (Eq. 2a) u - 1 is multiplied each step by 1 + dt (Du lam - F)."""
    lam, th = _eig(shape, m)
    g = 1.0 + dt * (Du * lam - F)
    mode = _mode(shape, th)
    u0 = 1.0 + eps * mode
    v0 = np.zeros(shape)
    u, v = O.run(u0, v0, n, Du=Du, Dv=0.1, F=F, k=0.05, dt=dt, impl=impl)
    exact = g ** n * eps * mode
    err = np.max(np.abs((u - 1.0) - exact))
    assert np.all(v == 0.0), "v must stay exactly zero"
    assert err <= 1e-13, f"u-mode decay off closed form by {err}"


def fourier_v(impl=None, shape=(10, 12, 8), m=(2, 1, 1), Dv=0.1, k=0.03, dt=0.7, n=30, eps=0.5):
    """Diffusion + kill on a v-mode: u = 0, F = 0, so u stays 0 and each step
    multiplies v by 1 + dt (Dv lam - k) (Eq. 2b)."""
    lam, th = _eig(shape, m)
    g = 1.0 + dt * (Dv * lam - k)
    mode = _mode(shape, th)
    u0 = np.zeros(shape)
    v0 = eps * mode
    u, v = O.run(u0, v0, n, Du=0.2, Dv=Dv, F=0.0, k=k, dt=dt, impl=impl)
    err = np.max(np.abs(v - g ** n * v0))
    assert np.all(u == 0.0), "u must stay exactly zero"
    assert err <= 1e-13, f"v-mode decay off closed form by {err}"


def laplacian_modes(impl=None, shape=(6, 8, 10)):
    """The single-field Laplacian of a Fourier mode is its eigenvalue times the
    mode, for several modes (pins each axis' neighbour pairs and the 1/6)."""
    for m in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 3, 1), (5, 4, 3)]:
        lam, th = _eig(shape, m)
        f = _mode(shape, th)
        err = np.max(np.abs(O.laplacian(f, impl=impl) - lam * f))
        assert err <= 1e-14, f"laplacian of mode {m} off by {err}"
    c = np.full(shape, 0.7)
    assert np.all(O.laplacian(c, impl=impl) == 0.0), "laplacian of a constant must be exactly 0"


def _fixed_point_nontrivial(F, k):
    """Uniform steady states of the reaction terms of Eq. 1a/1b (noise 0):
    u v^2 = (F + k) v and u v^2 = F (1 - u). With v != 0 this gives
    (F + k) v^2 - F v + F (F + k) = 0 and u = (F + k) / v."""
    a, b, c = F + k, -F, F * (F + k)
    disc = b * b - 4 * a * c
    assert disc > 0
    vs = [(-b + s * math.sqrt(disc)) / (2 * a) for s in (1, -1)]
    return [((F + k) / v, v) for v in vs]


def reaction_fixed_points(impl=None, shape=(4, 4, 8), F=0.05, k=0.04, dt=0.6, n=5):
    """A uniform state at a steady state of the reaction ODE stays there (the
    Laplacian of a constant is 0): pins -uv^2, +uv^2, F(1-u) and -(F+k)v."""
    for us, vs in _fixed_point_nontrivial(F, k) + [(1.0, 0.0)]:
        u0 = np.full(shape, us)
        v0 = np.full(shape, vs)
        u, v = O.run(u0, v0, n, Du=0.2, Dv=0.1, F=F, k=k, dt=dt, impl=impl)
        err = max(np.max(np.abs(u - us)), np.max(np.abs(v - vs)))
        assert err <= 1e-13, f"steady state ({us}, {vs}) drifted by {err}"


def trivial_fixed_point_bitwise(impl=None, shape=(8, 8, 8)):
    """u=1, v=0 is stationary bit for bit: neighbour sum 6 exactly, lap 0, F(1-u) 0."""
    u0, v0 = np.ones(shape), np.zeros(shape)
    u, v = O.run(u0, v0, 20, Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1.0, impl=impl)
    assert np.array_equal(u, u0) and np.array_equal(v, v0)


def mass_conservation(impl=None, shape=(10, 12, 14), n=40):
    """With F = k = 0 and no noise the reaction moves u v^2 from u to v and the
    periodic Laplacian sums to zero, so sum(u + v) is invariant (Eq. 1a + 1b),
    and sum(v) cannot decrease while u >= 0."""
    rng = np.random.default_rng(7)
    u0 = rng.uniform(0.0, 1.0, size=shape)
    v0 = rng.uniform(0.0, 0.3, size=shape)
    m0 = math.fsum(u0.ravel()) + math.fsum(v0.ravel())
    u, v = u0, v0
    sv_prev = math.fsum(v0.ravel())
    for s in range(n):
        u, v = O.run(u, v, 1, Du=0.2, Dv=0.1, F=0.0, k=0.0, dt=0.9, step0=s, impl=impl)
        sv = math.fsum(v.ravel())
        assert sv >= sv_prev - 1e-12 * abs(sv_prev), "sum(v) decreased with F=k=0"
        sv_prev = sv
    m1 = math.fsum(u.ravel()) + math.fsum(v.ravel())
    assert abs(m1 - m0) <= 1e-12 * abs(m0), f"mass drift {abs(m1 - m0) / abs(m0)}"


def dense_brute_force(impl=None, shape=(6, 8, 10), n=4, noise=0.01, dt=0.9, seed=99, step0=3):
    """Independent construction of the whole scheme: the periodic Laplacian as a
    dense matrix (Kronecker sum of three 1-D cycle matrices), the source terms
    of Eq. 1a/1b vectorised, forward Euler (Eq. 2a/2b) and the noise from the
    pure-Python Philox."""
    nz, ny, nx = shape

    def cyc(m):
        C = np.zeros((m, m))
        for i in range(m):
            C[i, (i + 1) % m] += 1.0
            C[i, (i - 1) % m] += 1.0
        return C

    A = (np.kron(np.eye(nz), np.kron(np.eye(ny), cyc(nx)))
         + np.kron(np.eye(nz), np.kron(cyc(ny), np.eye(nx)))
         + np.kron(cyc(nz), np.kron(np.eye(ny), np.eye(nx))))
    Lap = (A - 6.0 * np.eye(nx * ny * nz)) / 6.0
    p = dict(Du=0.17, Dv=0.09, F=0.031, k=0.052)
    rng = np.random.default_rng(11)
    u0 = rng.uniform(0.2, 1.0, size=shape)
    v0 = rng.uniform(0.0, 0.5, size=shape)
    u, v = u0.ravel().copy(), v0.ravel().copy()
    N = u.size
    for s in range(n):
        t = step0 + s
        r = np.array([pyphilox.uniform_pm1(seed, t, i) for i in range(N)])
        uvv = u * v * v
        du = p["Du"] * (Lap @ u) - uvv + p["F"] * (1 - u) + noise * r
        dv = p["Dv"] * (Lap @ v) + uvv - (p["F"] + p["k"]) * v
        u, v = u + dt * du, v + dt * dv
    uo, vo = O.run(u0, v0, n, dt=dt, noise=noise, seed=seed, step0=step0, impl=impl, **p)
    err = max(np.max(np.abs(uo.ravel() - u)), np.max(np.abs(vo.ravel() - v)))
    assert err <= 1e-14, f"dense brute force differs by {err}"


def translation_equivariance(impl=None, shape=(8, 8, 8), n=10):
    """A periodic shift of the initial state shifts the result, bit for bit
    (noise 0, so nothing depends on absolute position)."""
    u0, v0 = np.random.default_rng(3).uniform(0, 1, size=(2,) + shape)
    p = dict(Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1.0, impl=impl)
    u, v = O.run(u0, v0, n, **p)
    sh = (1, 2, 3)
    us, vs = O.run(np.roll(u0, sh, axis=(0, 1, 2)), np.roll(v0, sh, axis=(0, 1, 2)), n, **p)
    assert np.array_equal(us, np.roll(u, sh, axis=(0, 1, 2)))
    assert np.array_equal(vs, np.roll(v, sh, axis=(0, 1, 2)))


def reflection_symmetry(impl=None, shape=(8, 8, 8), n=10):
    """Mirroring any axis of the state mirrors the result bit for bit (each
    neighbour pair is summed symmetrically); swapping x and y transposes it."""
    u0, v0 = np.random.default_rng(4).uniform(0, 1, size=(2,) + shape)
    p = dict(Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1.0, impl=impl)
    u, v = O.run(u0, v0, n, **p)
    for ax in range(3):
        um, vm = O.run(np.flip(u0, ax).copy(), np.flip(v0, ax).copy(), n, **p)
        assert np.array_equal(um, np.flip(u, ax)) and np.array_equal(vm, np.flip(v, ax)), ax
    ut, vt = O.run(u0.transpose(0, 2, 1).copy(), v0.transpose(0, 2, 1).copy(), n, **p)
    assert np.array_equal(ut, u.transpose(0, 2, 1)) and np.array_equal(vt, v.transpose(0, 2, 1))


def noise_placement(impl=None, shape=(4, 6, 8), noise=0.1, dt=0.5, seed=12345, t=17):
    """One step from the fixed point (1, 0): only u moves, by exactly dt * n * r
    with r the (seed, step, cell)-keyed value of the independent Philox."""
    u0, v0 = np.ones(shape), np.zeros(shape)
    u, v = O.run(u0, v0, 1, Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=dt, noise=noise,
                 seed=seed, step0=t, impl=impl)
    N = u.size
    r = np.array([pyphilox.uniform_pm1(seed, t, i) for i in range(N)])
    exp = 1.0 + (noise * r) * dt
    assert np.array_equal(u.ravel(), exp), "u after one noisy step from (1,0)"
    assert np.all(v == 0.0)


def philox_vs_python(impl=None, n=300):
    rng = np.random.default_rng(5)
    for _ in range(n):
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)]
        assert O.philox4x32_10(ctr, key, impl=impl) == pyphilox.block(ctr, key), (ctr, key)
    for seed, t, idx in [(0, 0, 0), (230910292, 999, 134217727), (2 ** 64 - 1, 2 ** 33 + 5, 2 ** 40 + 3)]:
        for j in range(4):
            assert O.noise_r(seed, t, idx + j, impl=impl) == pyphilox.uniform_pm1(seed, t, idx + j)


def init_cube_slices(impl=None):
    for shape, side in [((64, 64, 64), 12), ((20, 16, 24), 5)]:
        u, v = O.init_cube(shape=shape, side=side, cu=0.25, cv=0.33, impl=impl)
        ue, ve = np.ones(shape), np.zeros(shape)
        lo = [(n - side) // 2 for n in shape]
        sl = tuple(slice(a, a + side) for a in lo)
        ue[sl], ve[sl] = 0.25, 0.33
        assert np.array_equal(u, ue) and np.array_equal(v, ve)


ALL = [fourier_u, fourier_v, laplacian_modes, reaction_fixed_points, trivial_fixed_point_bitwise,
       mass_conservation, dense_brute_force, translation_equivariance, reflection_symmetry,
       noise_placement, philox_vs_python, init_cube_slices]
