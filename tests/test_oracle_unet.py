"""Pins of the denoiser oracle against things other than its own code: scipy's 2-D
correlation, adjoint (dot-product) identities, central finite differences of the loss,
weight settings whose output has a closed form (the skip path, the path through every
pooling level, the input-channel order, the head bias), and Adam's closed-form steps."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet_oracle as U
from paper_2510_24154_amd import synth

RNG = np.random.default_rng(1234)


@pytest.mark.parametrize("k", [1, 3])
def test_conv_is_scipy_same_correlation(k):
    x = RNG.standard_normal((2, 7, 9, 3))
    W = RNG.standard_normal((4, k, k, 3))
    b = RNG.standard_normal(4)
    out = U.conv(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[n, :, :, c], W[o, :, :, c], mode="same") for c in range(3)) + b[o]
            np.testing.assert_allclose(out[n, :, :, o], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("k", [1, 3])
def test_conv_backward_is_the_adjoint(k):
    x = RNG.standard_normal((2, 6, 8, 5))
    W = RNG.standard_normal((3, k, k, 5))
    g = RNG.standard_normal((2, 6, 8, 3))
    V = RNG.standard_normal(W.shape)
    dx, dW, db = U.conv_backward(x, W, g)
    zero = np.zeros(3)
    lhs = np.sum(U.conv(x, W, zero) * g)
    assert abs(lhs - np.sum(x * dx)) < 1e-10 * abs(lhs) + 1e-10          # <Ax, g> = <x, A^T g>
    lhs = np.sum(U.conv(x, V, zero) * g)
    assert abs(lhs - np.sum(V * dW)) < 1e-10 * abs(lhs) + 1e-10          # linear in W
    np.testing.assert_allclose(db, g.sum(axis=(0, 1, 2)), rtol=1e-13)


def test_pool_and_upsample_adjoints():
    x = RNG.standard_normal((2, 6, 10, 3))
    y = RNG.standard_normal((2, 3, 5, 3))
    assert abs(np.sum(U.pool(x) * y) - np.sum(x * U.pool_backward(y))) < 1e-12
    assert abs(np.sum(U.upsample(y) * x) - np.sum(y * U.upsample_backward(x))) < 1e-12
    np.testing.assert_array_equal(U.pool(U.upsample(y)), y)
    assert np.all(U.pool(np.full((1, 4, 4, 1), 2.5)) == 2.5)
    assert U.pool(np.arange(16.0).reshape(1, 4, 4, 1))[0, 0, 0, 0] == (0 + 1 + 4 + 5) / 4


def _zero_params(levels, base, cin=2):
    return {n: (np.zeros((co, k, k, ci)), np.zeros(co)) for n, k, ci, co in U.layer_shapes(levels, base, cin)}


def _centre(P, name, o, c, v=1.0):
    W, b = P[name]
    W[o, W.shape[1] // 2, W.shape[2] // 2, c] = v


def test_forward_skip_path_closed_form():
    """Identity on channel 0 through e0a, e0b, the skip half of cat0, d0a, d0b and the head:
    out = x0 + relu(x0) = 2 x0 for x0 >= 0 (nothing else reaches the output)."""
    L, B = 4, 4
    P = _zero_params(L, B)
    for n in ("e0a", "e0b", "d0a", "d0b", "head"):
        _centre(P, n, 0, 0)
    x = RNG.uniform(0, 3, (2, 16, 24, 2))
    out, _ = U.forward(P, x, L)
    np.testing.assert_allclose(out, 2 * x[..., 0], rtol=0, atol=1e-14)


def test_forward_bottleneck_path_closed_form():
    """Identity on channel 0 down every level and back up every 1x1 up-convolution, with
    each decoder level reading the upsampled half of its concatenation: the output is
    x0 plus the 8x8 block mean of x0 repeated over its block."""
    L, B = 4, 4
    P = _zero_params(L, B)
    for l in range(L):
        _centre(P, f"e{l}a", 0, 0)
        _centre(P, f"e{l}b", 0, 0)
    for l in range(L - 1):
        _centre(P, f"u{l}", 0, 0)
        _centre(P, f"d{l}a", 0, B << l)       # first channel of the upsampled half
        _centre(P, f"d{l}b", 0, 0)
    _centre(P, "head", 0, 0)
    x = RNG.uniform(0, 3, (1, 16, 32, 2))
    out, _ = U.forward(P, x, L)
    x0 = x[0, :, :, 0]
    m = x0.reshape(2, 8, 4, 8).mean(axis=(1, 3))
    expect = x0 + np.repeat(np.repeat(m, 8, axis=0), 8, axis=1)
    np.testing.assert_allclose(out[0], expect, rtol=0, atol=1e-13)


def test_forward_reads_the_thickness_channel_second_and_head_bias():
    L, B = 4, 4
    P = _zero_params(L, B)
    for n in ("e0b", "d0a", "d0b", "head"):
        _centre(P, n, 0, 0)
    _centre(P, "e0a", 0, 1)                    # channel 1 = thickness
    P["head"][1][0] = 0.25
    x = RNG.uniform(0, 3, (1, 8, 16, 2))
    out, _ = U.forward(P, x, L)
    np.testing.assert_allclose(out[0], x[0, :, :, 0] + x[0, :, :, 1] + 0.25, rtol=0, atol=1e-14)


def test_normalise():
    noisy = RNG.uniform(0, 1e-4, (2, 8, 8))
    th = RNG.uniform(0, 30, (2, 8, 8))
    x, s = U.normalise(noisy, th)
    np.testing.assert_allclose(x[..., 0].mean(axis=(1, 2)), 1.0, rtol=1e-14)
    np.testing.assert_allclose(x[..., 1] * 20.0, th, rtol=1e-15)
    np.testing.assert_allclose(s, noisy.mean(axis=(1, 2)), rtol=1e-15)


@pytest.mark.parametrize("levels,base", [(3, 4), (4, 2)])
def test_network_gradients_match_finite_differences(levels, base):
    """Every layer's weight and bias gradient against central differences of the loss."""
    sh = U.layer_shapes(levels, base)
    P = {k: (W.astype(np.float64), b.astype(np.float64) + 0.05)
         for k, (W, b) in synth.unet_params([s for s in sh], seed=3, head_scale=0.3).items()}
    f = 1 << (levels - 1)
    x = RNG.uniform(0, 2, (2, 2 * f, 3 * f, 2))
    y = RNG.uniform(0, 2, (2, 2 * f, 3 * f))
    out, act = U.forward(P, x, levels)
    g = U.backward(P, act, out, y, levels)
    assert set(g) == {s[0] for s in sh}
    h = 1e-6
    for name, k, ci, co in sh:
        W, b = P[name]
        for which, arr in ((0, W), (1, b)):
            for _ in range(3):
                idx = tuple(int(RNG.integers(0, s)) for s in arr.shape)
                keep = arr[idx]
                arr[idx] = keep + h
                lp = U.loss(U.forward(P, x, levels)[0], y)
                arr[idx] = keep - h
                lm = U.loss(U.forward(P, x, levels)[0], y)
                arr[idx] = keep
                fd = (lp - lm) / (2 * h)
                an = g[name][which][idx]
                assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-4), (name, which, idx, fd, an)


def test_adam_closed_form_steps():
    """From zero moments the bias-corrected ratio is g/|g|: every step of a constant
    gradient moves theta by lr g / (|g| + eps), whatever t."""
    g = np.array([3.0, -0.5, 1e-3])
    th = np.array([1.0, 2.0, 3.0])
    m = v = np.zeros(3)
    for t in range(1, 6):
        new, m, v = U.adam(th, g, m, v, t, lr=0.01)
        np.testing.assert_allclose(th - new, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)
        th = new
    # the moments themselves: m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2
    np.testing.assert_allclose(m, (1 - 0.9 ** 5) * g, rtol=1e-12)
    np.testing.assert_allclose(v, (1 - 0.999 ** 5) * g * g, rtol=1e-12)


def test_bf16_rounding_model_sits_inside_the_gpu_gradient_tolerance():
    """The rounding model (BF16 storage of activations and activation gradients, FP32
    weight gradients) on the GPU gradient test's case: its distance from the FP64 oracle is
    what the GPU kernels are expected to show, and it stays below the GPU test's bound
    with a margin of 1.5."""
    from tests import _bf16_model as M
    from tests.test_gpu_denoise import GRAD_CASE, GRAD_TOL, net_case
    P, noisy, th, target = net_case(**GRAD_CASE)
    x, s = U.normalise(noisy, th)
    y = target / s[:, None, None]
    out, act = U.forward(P, x)
    ref = U.backward(P, act, out, y)
    G = M.gradients(P, x, y)
    worst = max(np.linalg.norm(G[k] - ref[k][0]) / np.linalg.norm(ref[k][0]) for k in ref)
    assert 0.001 < worst < GRAD_TOL / 1.5, worst
