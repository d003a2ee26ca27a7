"""CPU oracle of the learned EPID-image denoiser -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU baseline may
import this module; the engine never imports or calls it.

The paper proposes removing the statistical noise of a low-count Monte Carlo image with a
trained network, so that a quick simulation plus one network pass replaces a long
simulation (Sec. 4.1).  It gives no architecture.  The network written out here is the
reading used throughout: a 4-level U-Net with 32 base channels and 3x3 convolutions.

* Input: two channels per pixel:
  - the low-count image divided by its mean over the frame, s;
  - the radiological thickness (Sec. 2.2) divided by 20 cm.
* Output: the noisy image channel plus a learned correction, in units of s.
* Encoder: level l (l = 0..3, c_l = 32 * 2^l channels) applies conv3x3 + ReLU twice.
  Levels are joined by 2x2 average pooling.
* Decoder: level l (l = 2, 1, 0):
  - a 1x1 convolution of the level below (c_{l+1} -> c_l, no ReLU);
  - a nearest-neighbour 2x upsampling;
  - concatenation after the encoder's level-l output (skip first);
  - two conv3x3 + ReLU.
* Head: a 1x1 convolution to one channel, added to the noisy image channel.
* Loss: mean squared error against the high-count image over pixels and images.
* Optimiser: Adam (Kingma and Ba, 2015) with bias-corrected moments.

Everything is FP64 numpy.  Tensors are NHWC: (images, rows, columns, channels); weights
are (c_out, k, k, c_in).  A convolution is the sum over its k*k taps of a tensordot of the
shifted, zero-padded input with that tap's weights.  Backward passes are the adjoints
written out layer by layer.
"""
from __future__ import annotations

import numpy as np

LEVELS, BASE, IN_CH = 4, 32, 2
THICK_SCALE = 20.0   # cm; the thickness channel is t / 20 cm


def layer_shapes(levels=LEVELS, base=BASE, cin=IN_CH):
    """(name, k, c_in, c_out) of every convolution, in forward order."""
    c = [base << l for l in range(levels)]
    out, prev = [], cin
    for l in range(levels):
        out += [(f"e{l}a", 3, prev, c[l]), (f"e{l}b", 3, c[l], c[l])]
        prev = c[l]
    for l in range(levels - 2, -1, -1):
        out += [(f"u{l}", 1, c[l + 1], c[l]), (f"d{l}a", 3, 2 * c[l], c[l]), (f"d{l}b", 3, c[l], c[l])]
    out.append(("head", 1, c[0], 1))
    return out


# ---------------------------------------------------------------------------------------
# layers
# ---------------------------------------------------------------------------------------
def conv(x, W, b):
    """out[n,y,x,o] = b[o] + sum over taps (i,j) and channels c of
    xpad[n, y+i, x+j, c] * W[o,i,j,c], with zero padding (k-1)/2 (a 'same' correlation)."""
    k = W.shape[1]
    p = (k - 1) // 2
    N, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    out = np.zeros((N, H, Wd, W.shape[0])) + b
    for i in range(k):
        for j in range(k):
            out += np.tensordot(xp[:, i:i + H, j:j + Wd, :], W[:, i, j, :], axes=([3], [1]))
    return out


def conv_backward(x, W, g):
    """Adjoint of conv for an upstream gradient g = dL/dout: returns (dL/dx, dL/dW, dL/db)."""
    k = W.shape[1]
    p = (k - 1) // 2
    N, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (p, p), (p, p), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for i in range(k):
        for j in range(k):
            dW[:, i, j, :] = np.tensordot(g, xp[:, i:i + H, j:j + Wd, :], axes=([0, 1, 2], [0, 1, 2]))
            dxp[:, i:i + H, j:j + Wd, :] += np.tensordot(g, W[:, i, j, :], axes=([3], [0]))
    return dxp[:, p:p + H, p:p + Wd, :], dW, g.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


def pool(x):
    """2x2 average pooling (rows and columns even)."""
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_backward(g):
    """Adjoint of pool: each input pixel receives a quarter of its block's gradient."""
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def upsample(x):
    """Nearest-neighbour 2x upsampling."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample_backward(g):
    """Adjoint of upsample: the sum of each 2x2 block."""
    N, H, W, C = g.shape
    return g.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# ---------------------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------------------
def normalise(noisy, thickness):
    """Network input and scale from a batch of images (N, H, W) and thickness maps:
    s = mean of each noisy image over its frame (1 when that mean is not positive, e.g. an
    empty image); x = [noisy / s, thickness / 20 cm]."""
    noisy = np.asarray(noisy, np.float64)
    s = noisy.reshape(noisy.shape[0], -1).mean(axis=1)
    s = np.where(s > 0, s, 1.0)
    x = np.stack([noisy / s[:, None, None], np.asarray(thickness, np.float64) / THICK_SCALE], axis=-1)
    return x, s


def _p64(params):
    return {k: (np.asarray(W, np.float64), np.asarray(b, np.float64)) for k, (W, b) in params.items()}


def forward(params, x, levels=LEVELS):
    """Network output (N, H, W) for input x (N, H, W, 2), and the activations the backward
    pass needs.  params: {name: (W, b)}."""
    P = _p64(params)
    act = {"x": x}
    h = x
    for l in range(levels):                       # encoder
        act[f"in_e{l}"] = h
        act[f"e{l}a"] = relu(conv(h, *P[f"e{l}a"]))
        act[f"e{l}b"] = relu(conv(act[f"e{l}a"], *P[f"e{l}b"]))
        h = act[f"e{l}b"]
        if l < levels - 1:
            h = pool(h)
    for l in range(levels - 2, -1, -1):           # decoder
        act[f"in_u{l}"] = h
        up = upsample(conv(h, *P[f"u{l}"]))
        act[f"cat{l}"] = np.concatenate([act[f"e{l}b"], up], axis=-1)
        act[f"d{l}a"] = relu(conv(act[f"cat{l}"], *P[f"d{l}a"]))
        act[f"d{l}b"] = relu(conv(act[f"d{l}a"], *P[f"d{l}b"]))
        h = act[f"d{l}b"]
    return x[..., 0] + conv(h, *P["head"])[..., 0], act


def loss(out, target):
    """Mean squared error over every pixel of every image."""
    return float(np.mean((np.asarray(out) - np.asarray(target)) ** 2))


def backward(params, act, out, target, levels=LEVELS):
    """Gradients {name: (dW, db)} of loss(out, target), walking forward's layers in reverse."""
    P = _p64(params)
    grads = {}
    g = 2.0 * (out - target)[..., None] / out.size          # dL/d(head output)
    g, *grads["head"] = conv_backward(act["d0b"], P["head"][0], g)
    skip = {}
    for l in range(0, levels - 1):                            # decoder, top level first
        g = g * (act[f"d{l}b"] > 0)
        g, *grads[f"d{l}b"] = conv_backward(act[f"d{l}a"], P[f"d{l}b"][0], g)
        g = g * (act[f"d{l}a"] > 0)
        gcat, *grads[f"d{l}a"] = conv_backward(act[f"cat{l}"], P[f"d{l}a"][0], g)
        c = act[f"e{l}b"].shape[-1]
        skip[l] = gcat[..., :c]
        g, *grads[f"u{l}"] = conv_backward(act[f"in_u{l}"], P[f"u{l}"][0], upsample_backward(gcat[..., c:]))
    for l in range(levels - 1, -1, -1):                       # encoder, bottom level first
        if l < levels - 1:
            g = skip[l] + pool_backward(g)
        g = g * (act[f"e{l}b"] > 0)
        g, *grads[f"e{l}b"] = conv_backward(act[f"e{l}a"], P[f"e{l}b"][0], g)
        g = g * (act[f"e{l}a"] > 0)
        g, *grads[f"e{l}a"] = conv_backward(act[f"in_e{l}"], P[f"e{l}a"][0], g)
    return {k: tuple(v) for k, v in grads.items()}


def denoise(params, noisy, thickness, levels=LEVELS):
    """Denoised images (N, H, W) in the units of the noisy images."""
    x, s = normalise(noisy, thickness)
    out, _ = forward(params, x, levels)
    return out * s[:, None, None]


# ---------------------------------------------------------------------------------------
# optimiser
# ---------------------------------------------------------------------------------------
def adam(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1): moments m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    bias-corrected m^ = m / (1 - b1^t), v^ = v / (1 - b2^t), theta <- theta - lr m^ / (sqrt(v^) + eps).
    Returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
