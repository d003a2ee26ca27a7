"""Rounding model behind the denoiser's whole-network GPU tolerances (test helper).

It repeats the oracle's network with every activation and every activation gradient
rounded to BF16 (round to nearest even) at the points where the kernels store them, and
the weights rounded as the kernels use them.  The head weights and the weight gradients
stay unrounded, as in the kernels (the head runs in FP32; weight gradients are FP32).
Comparing this model with the FP64 oracle measures how far BF16 storage alone moves the
output and the gradients; the GPU tolerances are set above that.  Built from the oracle's
layer functions; the engine never imports it."""
import numpy as np

from oracle import unet_oracle as U


def rb(a):
    """Round to BF16 (nearest even) and return the value as float64."""
    f = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    f = (f + 0x7FFF + ((f >> 16) & 1)) >> 16
    return (f.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def gradients(P, x, y, L=U.LEVELS):
    """Weight gradients {name: dW} of the MSE loss with BF16 storage of activations and
    activation gradients."""
    Pr = {k: (rb(W), np.asarray(b, np.float64)) for k, (W, b) in P.items()}
    Pr["head"] = tuple(np.asarray(a, np.float64) for a in P["head"])
    A = {}
    h = rb(x)
    A["in_e0"] = h
    for l in range(L):
        A[f"ea{l}"] = rb(U.relu(U.conv(h, *Pr[f"e{l}a"])))
        A[f"eb{l}"] = h = rb(U.relu(U.conv(A[f"ea{l}"], *Pr[f"e{l}b"])))
        if l < L - 1:
            A[f"in_e{l + 1}"] = h = rb(U.pool(h))
    for l in range(L - 2, -1, -1):
        A[f"in_u{l}"] = h
        u = rb(U.conv(h, *Pr[f"u{l}"]))
        A[f"cat{l}"] = np.concatenate([A[f"eb{l}"], U.upsample(u)], -1)
        A[f"da{l}"] = rb(U.relu(U.conv(A[f"cat{l}"], *Pr[f"d{l}a"])))
        A[f"db{l}"] = h = rb(U.relu(U.conv(A[f"da{l}"], *Pr[f"d{l}b"])))
    out = x[..., 0] + U.conv(h, *Pr["head"])[..., 0]
    G = {}
    gr = 2 * (out - y)[..., None] / out.size
    dx, G["head"], _ = U.conv_backward(A["db0"], Pr["head"][0], gr)
    g = rb(dx * (A["db0"] > 0))
    gcat = {}
    for l in range(L - 1):
        dx, G[f"d{l}b"], _ = U.conv_backward(A[f"da{l}"], Pr[f"d{l}b"][0], g)
        g = rb(dx * (A[f"da{l}"] > 0))
        dx, G[f"d{l}a"], _ = U.conv_backward(A[f"cat{l}"], Pr[f"d{l}a"][0], g)
        gcat[l] = rb(dx)
        c = A[f"eb{l}"].shape[-1]
        gu = rb(U.upsample_backward(gcat[l][..., c:]))
        dx, G[f"u{l}"], _ = U.conv_backward(A[f"in_u{l}"], Pr[f"u{l}"][0], gu)
        g = rb(dx * (A[f"in_u{l}"] > 0))
    gp = None
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            c = A[f"eb{l}"].shape[-1]
            g = rb((gcat[l][..., :c] + U.pool_backward(gp)) * (A[f"eb{l}"] > 0))
        dx, G[f"e{l}b"], _ = U.conv_backward(A[f"ea{l}"], Pr[f"e{l}b"][0], g)
        g = rb(dx * (A[f"ea{l}"] > 0))
        dx, G[f"e{l}a"], _ = U.conv_backward(A[f"in_e{l}"], Pr[f"e{l}a"][0], g)
        gp = rb(dx)
    return G
