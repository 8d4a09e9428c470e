"""Pins of the surrogate's FP64 network oracle: closed forms (identity and
shift kernels), torch's CPU convolution with circular padding (an independent
library routine), the erf form of GELU, and finite differences of the loss."""
import math

import numpy as np
import pytest

from oracle import surrogate_oracle as S


def test_param_count():
    assert S.N_PARAMS == 60480 + 98


def test_identity_and_shift_kernels():
    a = np.random.default_rng(0).normal(size=(3, 5, 6, 7))
    W = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        W[c, c, 1, 1, 1] = 1.0
    assert np.array_equal(S.conv3d(a, W), a)
    W2 = np.zeros((1, 1, 3, 3, 3))
    W2[0, 0, 2, 1, 0] = 1.0  # reads (z + 1, y, x - 1)
    out = S.conv3d(a[:1], W2)
    assert np.array_equal(out[0], np.roll(a[0], shift=(-1, 0, 1), axis=(0, 1, 2)))


def test_conv_matches_torch_circular():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    a = rng.normal(size=(4, 6, 5, 8))
    W = rng.normal(size=(7, 4, 3, 3, 3))
    b = rng.normal(size=(7,))
    t = torch.from_numpy(a)[None]
    tp = torch.nn.functional.pad(t, (1, 1, 1, 1, 1, 1), mode="circular")
    ref = torch.nn.functional.conv3d(tp, torch.from_numpy(W), torch.from_numpy(b))[0].numpy()
    assert np.max(np.abs(S.conv3d(a, W, b) - ref)) < 1e-12


def test_conv_gradients_match_torch_autograd():
    """The data-gradient (transposed) convolution and the weight gradient of
    one circular convolution against torch's autograd in FP64."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    a = rng.normal(size=(5, 4, 6, 7))
    W = rng.normal(size=(3, 5, 3, 3, 3))
    g = rng.normal(size=(3, 4, 6, 7))
    at = torch.from_numpy(a)[None].requires_grad_(True)
    Wt = torch.from_numpy(W).requires_grad_(True)
    out = torch.nn.functional.conv3d(torch.nn.functional.pad(at, (1, 1, 1, 1, 1, 1), mode="circular"), Wt)
    (out * torch.from_numpy(g)[None]).sum().backward()
    assert np.max(np.abs(S.conv3d_input_grad(g, W) - at.grad[0].numpy())) < 1e-11
    assert np.max(np.abs(S.conv3d_weight_grad(g, a) - Wt.grad.numpy())) < 1e-11


def test_gelu_closed_form():
    z = np.linspace(-6, 6, 101)
    exp = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in z])
    assert np.max(np.abs(S.gelu(z) - exp)) < 1e-15
    h = 1e-6
    fd = (S.gelu(z + h) - S.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(S.gelu_grad(z) - fd)) < 1e-8


def _small_params(seed=2):
    rng = np.random.default_rng(seed)
    params = []
    for l in range(4):
        ci, co = S.CHANNELS[l], S.CHANNELS[l + 1]
        params.append((rng.normal(0, 0.3 / math.sqrt(ci * 27) * 3, size=(co, ci, 3, 3, 3)),
                       rng.normal(0, 0.05, size=co)))
    return params


def _samples(shape=(4, 4, 5), n=2, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        u, v = rng.uniform(0.2, 1.0, size=shape), rng.uniform(0.0, 0.4, size=shape)
        out.append((u, v, float(rng.uniform(0.01, 0.06)), float(rng.uniform(0.04, 0.07)),
                    u + 0.01 * rng.normal(size=shape), v + 0.01 * rng.normal(size=shape)))
    return out


def test_gradients_match_finite_differences():
    params = _small_params()
    samples = _samples()
    loss, grads = S.loss_and_grads(params, samples)
    vec = S.flatten(params)
    g = S.flatten(grads)
    rng = np.random.default_rng(4)
    idx = rng.choice(vec.size, size=40, replace=False)
    # include biases and every layer
    offs = np.cumsum([0] + [W.size + b.size for W, b in params])
    idx = np.concatenate([idx, offs[1:] - 1, offs[:-1] + 5])
    h = 1e-5
    for i in idx:
        vp, vm = vec.copy(), vec.copy()
        vp[i] += h
        vm[i] -= h
        lp, _ = S.loss_and_grads(S.unflatten(vp), samples)
        lm, _ = S.loss_and_grads(S.unflatten(vm), samples)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, g[i])


def test_gradients_match_torch_autograd():
    torch = pytest.importorskip("torch")
    params = _small_params(seed=5)
    samples = _samples(seed=6)
    loss, grads = S.loss_and_grads(params, samples)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    n_terms = sum(2 * s[0].size for s in samples)
    tl = 0
    for (u, v, F, k, ut, vt) in samples:
        x = torch.from_numpy(S.make_input(u, v, F, k))[None]
        a = x
        for l, (W, b) in enumerate(tp):
            z = torch.nn.functional.conv3d(torch.nn.functional.pad(a, (1,) * 6, mode="circular"), W, b)
            a = torch.nn.functional.gelu(z) if l < 3 else z
        pu = torch.from_numpy(u) + a[0, 0]
        pv = torch.from_numpy(v) + a[0, 1]
        tl = tl + ((pu - torch.from_numpy(ut)) ** 2).sum() + ((pv - torch.from_numpy(vt)) ** 2).sum()
    tl = tl / n_terms
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-12 * abs(loss)
    for (W, b), (gW, gb) in zip(tp, grads):
        assert np.max(np.abs(W.grad.numpy() - gW)) <= 1e-10 * (1 + np.max(np.abs(gW)))
        assert np.max(np.abs(b.grad.numpy() - gb)) <= 1e-10 * (1 + np.max(np.abs(gb)))
