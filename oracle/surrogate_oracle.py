"""FP64 CPU oracle of the learned 16-step surrogate's network.

TEST INFRASTRUCTURE ONLY: imported by tests (and the smoke/benchmark legs),
never by the HIP library or its binding. Plain numpy in float64.

Network (the surrogate workload's statement, not the paper's; the readings
are listed with the workload's definition):
  input  x0: 4 channels per cell: u, v, (F - 0.035) / 0.025, (k - 0.055) / 0.015
  layer l = 1..4: z_l = conv3x3x3_circular(a_{l-1}; W_l) + b_l
                  a_l = GELU(z_l) for l = 1, 2, 3 (exact, erf form)
  channels 4 -> 32 -> 32 -> 32 -> 2
  output (u, v) 16 steps ahead = (u, v) + z_4            (residual)
  loss   mean over samples, both fields and all cells of (pred - target)^2

Arrays are (C, nz, ny, nx) per sample; W_l has shape (C_out, C_in, 3, 3, 3)
with W[co, ci, dz, dy, dx] multiplying the input at (z + dz - 1, y + dy - 1,
x + dx - 1), periodic.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

CHANNELS = (4, 32, 32, 32, 2)
F_CENTER, F_SCALE = 0.035, 0.025
K_CENTER, K_SCALE = 0.055, 0.015


def offsets():
    """The 27 (dz, dy, dx) offsets in the order d = 9 dz + 3 dy + dx."""
    return [(dz, dy, dx) for dz in range(3) for dy in range(3) for dx in range(3)]


def shifted(a: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """b[..., z, y, x] = a[..., z + dz - 1, y + dy - 1, x + dx - 1] (periodic)."""
    return np.roll(a, shift=(1 - dz, 1 - dy, 1 - dx), axis=(-3, -2, -1))


def conv3d(a: np.ndarray, W: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """Circular 3x3x3 convolution (cross-correlation) of a (C_in, Z, Y, X)."""
    out = np.zeros((W.shape[0],) + a.shape[1:], dtype=np.float64)
    for dz, dy, dx in offsets():
        s = shifted(a, dz, dy, dx)
        out += np.einsum("oi,izyx->ozyx", W[:, :, dz, dy, dx], s)
    if b is not None:
        out += b[:, None, None, None]
    return out


def conv3d_input_grad(g: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Gradient of sum(g * conv3d(a, W)) with respect to a, for g of shape
    (C_out, Z, Y, X): the transposed convolution. Output position p receives
    W[o, i, d] g[o] from every output q whose offset-d neighbour is p, i.e.
    q = p - (d - 1)."""
    out = np.zeros((W.shape[1],) + g.shape[1:], dtype=np.float64)
    for dz, dy, dx in offsets():
        out += shifted(np.einsum("oi,ozyx->izyx", W[:, :, dz, dy, dx], g), 2 - dz, 2 - dy, 2 - dx)
    return out


def conv3d_weight_grad(g: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Gradient of sum(g * conv3d(a, W)) with respect to W: for every offset
    d, the correlation of the output gradient with the shifted input."""
    gW = np.zeros((g.shape[0], a.shape[0], 3, 3, 3), dtype=np.float64)
    for dz, dy, dx in offsets():
        gW[:, :, dz, dy, dx] = np.einsum("ozyx,izyx->oi", g, shifted(a, dz, dy, dx))
    return gW


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def make_input(u: np.ndarray, v: np.ndarray, F: float, k: float) -> np.ndarray:
    x = np.empty((4,) + u.shape, dtype=np.float64)
    x[0], x[1] = u, v
    x[2] = (F - F_CENTER) / F_SCALE
    x[3] = (k - K_CENTER) / K_SCALE
    return x


def forward(params, u, v, F, k, keep=False):
    """params: list of (W, b) per layer. Returns (pred_u, pred_v) and, with
    keep, the per-layer inputs and pre-activations."""
    a = make_input(u, v, F, k)
    acts, pre = [a], []
    for l, (W, b) in enumerate(params):
        z = conv3d(a, W, b)
        pre.append(z)
        a = gelu(z) if l < len(params) - 1 else z
        acts.append(a)
    pu = u + a[0]
    pv = v + a[1]
    return ((pu, pv), (acts, pre)) if keep else (pu, pv)


def loss_and_grads(params, samples):
    """Mean squared error over samples [(u, v, F, k, u_target, v_target)] and
    its gradients with respect to every W and b (backpropagation written out:
    the transposed convolution for inputs, the correlation of inputs with
    output gradients for weights)."""
    n_terms = sum(2 * s[0].size for s in samples)
    loss = 0.0
    grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    for (u, v, F, k, ut, vt) in samples:
        (pu, pv), (acts, pre) = forward(params, u, v, F, k, keep=True)
        ru, rv = pu - ut, pv - vt
        loss += float(np.sum(ru * ru) + np.sum(rv * rv))
        g = np.zeros_like(pre[-1])
        g[0] = 2.0 * ru / n_terms
        g[1] = 2.0 * rv / n_terms
        for l in range(len(params) - 1, -1, -1):
            W, b = params[l]
            a_in = acts[l]
            gW, gb = grads[l]
            gb += g.sum(axis=(1, 2, 3))
            for dz, dy, dx in offsets():
                gW[:, :, dz, dy, dx] += np.einsum("ozyx,izyx->oi", g, shifted(a_in, dz, dy, dx))
            if l == 0:
                break
            # gradient with respect to a_{l-1}: transposed convolution
            ga = np.zeros_like(a_in)
            for dz, dy, dx in offsets():
                ga += shifted(np.einsum("oi,ozyx->izyx", W[:, :, dz, dy, dx], g), 2 - dz, 2 - dy, 2 - dx)
            g = ga * gelu_grad(pre[l - 1])
    return loss / n_terms, grads


def init_params(seed: int):
    """He-style normal initialisation, small last layer (near-identity map)."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(4):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        scale = math.sqrt(2.0 / (ci * 27)) * (0.1 if l == 3 else 1.0)
        params.append((rng.normal(0.0, scale, size=(co, ci, 3, 3, 3)), np.zeros(co)))
    return params


def flatten(params) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(vec: np.ndarray):
    params, o = [], 0
    for l in range(4):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        nW = co * ci * 27
        W = vec[o:o + nW].reshape(co, ci, 3, 3, 3)
        o += nW
        b = vec[o:o + co]
        o += co
        params.append((W.copy(), b.copy()))
    return params


N_PARAMS = sum(CHANNELS[l + 1] * CHANNELS[l] * 27 + CHANNELS[l + 1] for l in range(4))
