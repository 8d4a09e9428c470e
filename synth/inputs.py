"""Workload definitions and seeded random draws.

Parameter values follow the paper's problem statement (Section 3.1, Eq. 1a/1b)
and its provenance record (Listing 1: Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1).
The initial condition (a centred cube of side 12 holding u=0.25, v=0.33 in a
u=1, v=0 background) is not in the paper; it is the workload definition this
project measures on. Nothing here evaluates the Gray-Scott update.
"""
from __future__ import annotations

import numpy as np

# Default Philox seed for noisy runs (the paper names no seed).
DEFAULT_SEED = 230910292

BASE = dict(Du=0.2, Dv=0.1, F=0.02, k=0.048, dt=1.0, noise=0.0,
            seed=DEFAULT_SEED, step0=0, cube_side=12, cube_u=0.25, cube_v=0.33)


def workload(name: str) -> dict:
    """Return the parameter dict of a named workload.

    small_l64      : L=64 cube, FP64, noise 0, 100 steps (whole-field parity case)
    weak_share_l512: L=512 cube, 1000 steps, noise 1e-7 (one GPU's share of a
                     weak-scaling run at half the paper's 1024^3 per GPU)
    precision_l1024: L=1024 cube, F=0.03, k=0.06, 200 steps, noise 0
    """
    p = dict(BASE)
    if name == "small_l64":
        p.update(L=64, steps=100)
    elif name == "weak_share_l512":
        p.update(L=512, steps=1000, noise=1e-7)
    elif name == "precision_l1024":
        p.update(L=1024, steps=200, F=0.03, k=0.06)
    else:
        raise KeyError(name)
    return p


def random_state(shape, seed: int, lo_u=0.0, hi_u=1.0, lo_v=0.0, hi_v=1.0):
    """Uniform random (u, v) float64 arrays of `shape` (z, y, x)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(lo_u, hi_u, size=shape)
    v = rng.uniform(lo_v, hi_v, size=shape)
    return u, v


def subnormal_field(shape, seed: int, m_max: int = 1 << 20):
    """A float64 array of `shape` holding m 2^-1074 with m uniform in
    [0, m_max): subnormal values (and zeros), as in the decayed tails of a
    field."""
    rng = np.random.default_rng(seed)
    m = rng.integers(0, m_max, size=shape, dtype=np.uint64)
    return m.view(np.float64)


def batch_sweep(n_sims: int = 256, seed: int = DEFAULT_SEED,
                sides=tuple(range(32, 193, 16)), f_range=(0.01, 0.06),
                k_range=(0.04, 0.07)):
    """Independent simulations for a batched (F, k) sweep.

    Returns a list of dicts {L, F, k}; L is drawn uniformly from `sides`
    (32, 48, ..., 192 by default), F and k uniformly from their ranges.
    """
    rng = np.random.default_rng(seed)
    Ls = rng.choice(np.asarray(sides), size=n_sims)
    Fs = rng.uniform(*f_range, size=n_sims)
    ks = rng.uniform(*k_range, size=n_sims)
    return [dict(L=int(L), F=float(F), k=float(k)) for L, F, k in zip(Ls, Fs, ks)]


def random_blobs(n: int, L: int, seed: int, side_range=(6, 24)):
    """Random blob placements for surrogate training trajectories.

    Each blob is a cube with side drawn uniformly from side_range (inclusive)
    at a uniformly random corner (periodic, so any corner is valid), plus
    (F, k) drawn as in `batch_sweep`. Returns a list of dicts
    {x0, y0, z0, side, F, k}.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        x0, y0, z0 = (int(c) for c in rng.integers(0, L, size=3))
        F = float(rng.uniform(0.01, 0.06))
        k = float(rng.uniform(0.04, 0.07))
        out.append(dict(x0=x0, y0=y0, z0=z0, side=side, F=F, k=k))
    return out


def conv_weights(c_in: int, c_out: int, seed: int, scale: float | None = None):
    """He-style random 3x3x3 conv weights (c_out, c_in, 3, 3, 3) and biases, float64."""
    rng = np.random.default_rng(seed)
    if scale is None:
        scale = np.sqrt(2.0 / (c_in * 27))
    w = rng.normal(0.0, scale, size=(c_out, c_in, 3, 3, 3))
    b = rng.normal(0.0, 0.01, size=(c_out,))
    return w, b


SURROGATE_CHANNELS = (4, 32, 32, 32, 2)


def surrogate_init(seed: int):
    """Initial parameters of the 16-step surrogate network as one flat float32
    vector (per layer W[c_out][c_in][3][3][3] then b[c_out]): He-normal
    weights, last layer scaled by 0.1 (the network starts near the identity
    map through its residual output), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    ch = SURROGATE_CHANNELS
    for l in range(4):
        ci, co = ch[l], ch[l + 1]
        scale = np.sqrt(2.0 / (ci * 27)) * (0.1 if l == 3 else 1.0)
        parts.append(rng.normal(0.0, scale, size=co * ci * 27))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
