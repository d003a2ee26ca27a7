"""GPU parity of the denoiser (BF16 MFMA kernels through the C ABI) against the FP64 oracle.

Per layer, the oracle gets the same BF16-rounded operands, so the differences are FP32
accumulation and the final rounding of BF16 outputs (half an ulp, 2^-9 relative; the test
allows 2^-8).  The accumulation bound is one FP32 rounding (2^-24) of the running sum of
|terms| per sequential addition -- one per MFMA step of 32 products, per pixel chunk of a
weight gradient -- doubled for margin.  A whole network rounds every activation and activation gradient to
BF16 on the way (about 14 roundings on a path, each up to 2^-9 relative), so its outputs
and gradients are compared by relative L2 error with a bound of a few percent and by the
cosine of the angle between gradient vectors."""
import numpy as np
import pytest

from oracle import unet_oracle as U
from paper_2510_24154_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_24154_amd import denoise
    return denoise


def bf(a):
    """numpy float64 -> torch bfloat16 on the GPU (round to nearest even) and the exact
    float64 value of the rounded numbers."""
    import torch
    t = torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16)
    return t.cuda(), t.to(torch.float64).numpy()


def host(t):
    import torch
    return t.to(torch.float64).cpu().numpy()


def acc_bound(k, c_in):
    """FP32 accumulation bound per unit of sum |terms|: one rounding per MFMA step of 32
    products (k*k*c_in/32 steps), two for the bias and the final add, at 2^-24 each, doubled."""
    return (-(-k * k * c_in // 32) + 2) * 2.0 ** -23


def within(dev, ref, absum, rel_out=2.0 ** -8, rel_acc=2.0 ** -20):
    err = np.abs(dev - ref) - (rel_out * np.abs(ref) + rel_acc * absum + 1e-30)
    return float(err.max()), np.unravel_index(int(np.argmax(err)), err.shape)


CONV_CASES = [  # (n, h, w, c_in, ld_in, c_out, ld_out, k)
    (2, 7, 13, 8, 8, 32, 32, 3),        # the input layer's 8 channels; 182 pixels (ragged tiles)
    (1, 16, 24, 32, 64, 64, 64, 3),     # channel slice of a wider tensor as input
    (3, 9, 10, 64, 64, 32, 96, 3),      # output into a slice (concatenation buffer)
    (2, 8, 8, 128, 128, 64, 64, 1),     # 1x1
    (1, 5, 40, 256, 256, 128, 128, 3),
]


@pytest.mark.parametrize("case", CONV_CASES)
@pytest.mark.parametrize("mode", ["relu_bias", "gated", "plain"])
def test_conv_forward_matches_oracle(D, case, mode):
    import torch
    n, h, w, ci, ldi, co, ldo, k = case
    rng = np.random.default_rng([*case, ["relu_bias", "gated", "plain"].index(mode)])
    xs = rng.standard_normal((n, h, w, ldi))
    ws = rng.standard_normal((co, k, k, ci)) / np.sqrt(k * k * ci)
    b = rng.standard_normal(co).astype(np.float32) * 0.1
    x_t, x64 = bf(xs)
    w_t, w64 = bf(ws)
    y = torch.zeros((n, h, w, ldo), dtype=torch.bfloat16, device="cuda")
    gate_t = g64 = None
    if mode == "gated":
        gate_t, g64 = bf(rng.standard_normal((n, h, w, co)))
    D.conv(x_t[..., :ci], w_t, torch.as_tensor(b).cuda() if mode != "plain" else None, y[..., :co], k,
           relu=mode == "relu_bias", gate=gate_t)
    torch.cuda.synchronize()
    ref = U.conv(x64[..., :ci], w64, b.astype(np.float64) if mode != "plain" else np.zeros(co))
    absum = U.conv(np.abs(x64[..., :ci]), np.abs(w64), np.abs(b.astype(np.float64)))
    if mode == "relu_bias":
        ref = np.maximum(ref, 0)
    if mode == "gated":
        ref = np.where(g64 > 0, ref, 0.0)
    dev = host(y)
    e, at = within(dev[..., :co], ref, absum, rel_acc=acc_bound(k, ci))
    assert e <= 0, (e, at, dev[..., :co][at], ref[at])
    assert np.all(dev[..., co:] == 0)   # nothing written outside the slice


@pytest.mark.parametrize("case", CONV_CASES)
def test_backward_data_matches_oracle(D, case):
    """The forward kernel on the gradient with flipped, transposed weights is the adjoint."""
    import torch
    n, h, w, ci, _, co, _, k = case
    rng = np.random.default_rng(7)
    x = rng.standard_normal((n, h, w, ci))
    w32 = torch.as_tensor((rng.standard_normal((co, k, k, ci)) / np.sqrt(k * k * ci)).astype(np.float32)).cuda()
    wf, wb = D.weights(w32)
    w64 = host(wf)
    assert np.array_equal(host(wb), np.flip(w64, axis=(1, 2)).transpose(3, 1, 2, 0))
    g_t, g64 = bf(rng.standard_normal((n, h, w, co)))
    dx = torch.zeros((n, h, w, ci), dtype=torch.bfloat16, device="cuda")
    if ci % 32:   # the input layer's data gradient is never needed, and not supported
        from paper_2510_24154_amd import EpidmcError
        with pytest.raises(EpidmcError, match="E_SHAPE"):
            D.conv(g_t, wb, None, dx, k, relu=False)
        return
    D.conv(g_t, wb, None, dx, k, relu=False)
    torch.cuda.synchronize()
    ref, _, _ = U.conv_backward(x, w64, g64)
    absum, _, _ = U.conv_backward(np.abs(x), np.abs(w64), np.abs(g64))
    e, at = within(host(dx), ref, absum, rel_acc=acc_bound(k, co))
    assert e <= 0, (e, at)


WG_CASES = [  # (n, h, w, c_in, ld_in, c_out, k)
    (2, 7, 13, 8, 8, 32, 3),
    (1, 16, 24, 64, 128, 64, 3),
    (3, 9, 10, 32, 32, 32, 1),
    (1, 33, 40, 128, 128, 128, 3),      # several pixel chunks
    (2, 8, 8, 256, 256, 128, 1),
]


@pytest.mark.parametrize("case", WG_CASES)
def test_backward_weights_matches_oracle(D, case):
    import torch
    n, h, w, ci, ldi, co, k = case
    rng = np.random.default_rng(11)
    x_t, x64 = bf(rng.standard_normal((n, h, w, ldi)))
    g_t, g64 = bf(rng.standard_normal((n, h, w, co)))
    dw, db = D.wgrad(x_t[..., :ci], g_t, k)
    torch.cuda.synchronize()
    W0 = np.zeros((co, k, k, ci))
    _, ref_w, ref_b = U.conv_backward(x64[..., :ci], W0, g64)
    _, abs_w, abs_b = U.conv_backward(np.abs(x64[..., :ci]), W0, np.abs(g64))
    e, at = within(dw.cpu().numpy().astype(np.float64), ref_w, abs_w, rel_out=0.0, rel_acc=2.0 ** -18)
    assert e <= 0, (e, at)
    e, at = within(db.cpu().numpy().astype(np.float64), ref_b, abs_b, rel_out=0.0, rel_acc=2.0 ** -18)
    assert e <= 0, (e, at)
    # deterministic: the same call again gives the same bits
    dw2, db2 = D.wgrad(x_t[..., :ci], g_t, k)
    assert torch.equal(dw, dw2) and torch.equal(db, db2)


def test_pool_upsample_skip_match_oracle(D):
    import torch
    rng = np.random.default_rng(5)
    n, h, w, c = 2, 10, 14, 32
    x_t, x64 = bf(rng.standard_normal((n, h, w, 2 * c)))
    y = torch.empty((n, h // 2, w // 2, c), dtype=torch.bfloat16, device="cuda")
    D.pool(x_t[..., :c], y)
    ref = U.pool(x64[..., :c])
    e, at = within(host(y), ref, U.pool(np.abs(x64[..., :c])))
    assert e <= 0
    up = torch.zeros((n, h, w, 2 * c), dtype=torch.bfloat16, device="cuda")
    D.upsample(y, up[..., c:])
    assert np.array_equal(host(up)[..., c:], U.upsample(host(y)))
    assert np.all(host(up)[..., :c] == 0)
    gb = torch.empty((n, h // 2, w // 2, c), dtype=torch.bfloat16, device="cuda")
    D.upsample_backward(x_t[..., c:], gb)
    e, _ = within(host(gb), U.upsample_backward(x64[..., c:]), U.upsample_backward(np.abs(x64[..., c:])))
    assert e <= 0
    gp_t, gp64 = bf(rng.standard_normal((n, h // 2, w // 2, c)))
    act_t, act64 = bf(rng.standard_normal((n, h, w, c)))
    out = torch.empty((n, h, w, c), dtype=torch.bfloat16, device="cuda")
    D.skip_backward(x_t[..., :c], gp_t, act_t, out)
    torch.cuda.synchronize()
    ref = np.where(act64 > 0, x64[..., :c] + U.pool_backward(gp64), 0.0)
    e, _ = within(host(out), ref, np.abs(x64[..., :c]) + U.pool_backward(np.abs(gp64)))
    assert e <= 0


# ---- the whole network -------------------------------------------------------------------
def net_case(n=2, h=16, w=24, seed=3, bias=0.02):
    shapes = [s for s in U.layer_shapes()]
    P = synth.unet_params(shapes, seed=seed, head_scale=0.05)
    rng = np.random.default_rng(seed)
    P = {k: (W, (b + bias * rng.standard_normal(b.shape)).astype(np.float32)) for k, (W, b) in P.items()}
    noisy = rng.gamma(2.0, 1e-5, (n, h, w))
    th = rng.uniform(5, 30, (n, h, w))
    target = noisy * rng.uniform(0.8, 1.2, (n, h, w))
    return P, noisy, th, target


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_network_forward_matches_oracle(D):
    import torch
    P, noisy, th, _ = net_case()
    net = D.Unet(0).bind(2, 16, 24)
    net.set_params(P)
    back = net.get_params()
    for k, (W, b) in P.items():
        assert np.array_equal(back[k][0], W) and np.array_equal(back[k][1], b)
    dev = net.forward(torch.as_tensor(noisy).cuda(), torch.as_tensor(th).cuda()).cpu().numpy()
    ref = U.denoise(P, noisy, th)
    x, s = U.normalise(noisy, th)
    r_dev, r_ref = dev / s[:, None, None] - x[..., 0], ref / s[:, None, None] - x[..., 0]
    print("forward: rel L2 of the learned correction", rel_l2(r_dev, r_ref))
    assert rel_l2(r_dev, r_ref) < 0.03
    # a batch of one gives the first image's result (no cross-image leakage)
    one = net.forward(torch.as_tensor(noisy[:1]).cuda(), torch.as_tensor(th[:1]).cuda()).cpu().numpy()
    np.testing.assert_array_equal(one[0], dev[0])


GRAD_CASE = dict(n=2, h=32, w=48, seed=4)
GRAD_TOL = 0.06   # relative L2 per layer; the BF16 rounding model alone reaches 3.5% here


def test_network_gradients_match_oracle(D):
    import torch
    P, noisy, th, target = net_case(**GRAD_CASE)
    net = D.Unet(0).bind(2, 32, 48)
    net.set_params(P)
    loss, g = net.gradient(*(torch.as_tensor(a).cuda() for a in (noisy, th, target)))
    x, s = U.normalise(noisy, th)
    out, act = U.forward(P, x)
    y = target / s[:, None, None]
    ref_loss = U.loss(out, y)
    gr = U.backward(P, act, out, y)
    assert loss == pytest.approx(ref_loss, rel=0.02)
    for name, (dW, db) in gr.items():
        gd, gbias = g[name]
        a, b = gd.reshape(-1).astype(np.float64), dW.reshape(-1)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300))
        print(f"{name}: rel L2 {rel_l2(a, b):.4f} cos {cos:.6f} bias rel {rel_l2(gbias.astype(np.float64), db):.4f}")
        assert rel_l2(a, b) < GRAD_TOL and cos > 0.998, name
        assert rel_l2(gbias.astype(np.float64), db) < GRAD_TOL, name


def test_adam_step_matches_oracle(D):
    import torch
    P, noisy, th, target = net_case(seed=6)
    net = D.Unet(0).bind(2, 16, 24)
    net.set_params(P)
    args = [torch.as_tensor(a).cuda() for a in (noisy, th, target)]
    _, g = net.gradient(*args)             # the gradient the step will use
    net.train_step(*args, lr=1e-3)
    new = net.get_params()
    for name, (W, b) in P.items():
        for which, th0 in ((0, W), (1, b)):
            gg = g[name][which].astype(np.float64)
            ref, _, _ = U.adam(th0.astype(np.float64), gg, 0.0, 0.0, 1, lr=1e-3)
            np.testing.assert_allclose(new[name][which], ref, rtol=0, atol=2e-6, err_msg=name)


def test_full_size_interior_matches_oracle_on_a_crop(D):
    """The benchmark's image size (1024 x 768, one image): the network's interior output
    equals the oracle's on a 256 x 256 crop of the same normalised input, 64 pixels away
    from the crop's edges (beyond the receptive field's reach of the zero padding)."""
    import torch
    rng = np.random.default_rng(9)
    P = synth.unet_params(U.layer_shapes(), seed=9, head_scale=0.05)
    noisy = rng.gamma(2.0, 1e-5, (1, 1024, 768))
    th = rng.uniform(5, 30, (1, 1024, 768))
    net = D.Unet(0).bind(1, 1024, 768)
    net.set_params(P)
    dev = net.forward(torch.as_tensor(noisy).cuda(), torch.as_tensor(th).cuda()).cpu().numpy()[0]
    x, s = U.normalise(noisy, th)
    for (r0, c0) in ((384, 256), (0, 0), (768, 512)):
        crop = x[:, r0:r0 + 256, c0:c0 + 256]
        out, _ = U.forward(P, crop)
        ref = out[0] * s[0]
        m = 64
        rr = slice(m if r0 > 0 else 0, 256 - m if r0 + 256 < 1024 else 256)
        cc = slice(m if c0 > 0 else 0, 256 - m if c0 + 256 < 768 else 256)
        d = dev[r0:r0 + 256, c0:c0 + 256][rr, cc] / s[0] - crop[0][rr, cc, 0]
        e = ref[rr, cc] / s[0] - crop[0][rr, cc, 0]
        print("crop", r0, c0, "rel L2", rel_l2(d, e))
        assert rel_l2(d, e) < 0.03


# ---- what the trained network gains -------------------------------------------------------
def small_field(seed):
    """A training or evaluation field on a 128 x 96 image of 3.12 mm pixels (64 times the
    area of the full image's pixels) and a 64 x 64 x 32 phantom of 8 mm voxels."""
    return synth.denoise_field(seed, shape=(64, 64, 32), spacing=0.8, npx=(96, 128), pitch=0.312)


def in_field_rmse(est, ref):
    """RMS difference over the pixels at >= 10% of the reference's maximum, relative to the
    reference's mean there (per image, then averaged)."""
    out = []
    for e, r in zip(est, ref):
        sel = r >= 0.1 * r.max()
        out.append(np.sqrt(np.mean((e[sel] - r[sel]) ** 2)) / r[sel].mean())
    return float(np.mean(out))


def test_trained_denoiser_beats_plain_monte_carlo(D):
    """Train on 48 engine-generated fields (3e4 histories in, 3e6 as target, about the
    full image's deposits per pixel at 2e6 and 2e8 histories), then on 6 held-out fields
    compare with an independent 3e7-history reference: the denoised 3e4-history image is
    closer to it than the plain 3e4-history image, and closer than a plain image of 4x the
    histories (1.2e5)."""
    import torch
    n_low, n_high = 30_000, 3_000_000
    low, high, th = D.make_pairs([small_field(s) for s in range(48)], n_low, n_high, seed=5)
    net = D.Unet(0).bind(8, 128, 96)
    net.set_params(synth.unet_params(U.layer_shapes(), seed=1, head_scale=0.01))
    losses = D.train(net, low, high, th, steps=400, batch=8, lr=2e-3, lr_end=1e-4, seed=1)
    print("training loss: first 20 steps", losses[:20].mean(), "last 20", losses[-20:].mean())
    assert losses[-20:].mean() < 0.7 * losses[:20].mean()
    tests = [small_field(1000 + s) for s in range(6)]
    t_low, t_ref, t_th = D.make_pairs(tests, n_low, 30_000_000, seed=6)
    t_4x, _, _ = D.make_pairs(tests, 4 * n_low, 64, seed=7)
    den = torch.cat([net.forward(t_low[i:i + 6], t_th[i:i + 6]) for i in range(0, 6, 6)])
    ref = t_ref.cpu().numpy()
    e_plain = in_field_rmse(t_low.cpu().numpy(), ref)
    e_4x = in_field_rmse(t_4x.cpu().numpy(), ref)
    e_den = in_field_rmse(den.cpu().numpy(), ref)
    print(f"in-field relative RMSE: plain {e_plain:.4f}, plain x4 {e_4x:.4f}, denoised {e_den:.4f}")
    assert e_den < 0.5 * e_plain
    assert e_den < e_4x


# ---- edge cases and error behaviour ------------------------------------------------------------
def test_boundary_rejects_bad_shapes_and_states(D):
    import torch
    from paper_2510_24154_amd import EpidmcError
    net = D.Unet(0)
    with pytest.raises(EpidmcError, match="E_SHAPE"):
        net.bind(1, 20, 24)                    # rows not a multiple of 8
    net.bind(2, 16, 24)
    z = torch.zeros((2, 16, 24), dtype=torch.float64, device="cuda")
    with pytest.raises(EpidmcError, match="E_NOT_READY"):
        net.forward(z, z)                      # parameters not set
    net.set_params(synth.unet_params(U.layer_shapes(), seed=2))
    z3 = torch.zeros((3, 16, 24), dtype=torch.float64, device="cuda")
    with pytest.raises(EpidmcError, match="E_SHAPE"):
        net.forward(z3, z3)                    # batch larger than the bound one
    x = torch.zeros((1, 8, 8, 32), dtype=torch.bfloat16, device="cuda")
    w = torch.zeros((16, 3, 3, 32), dtype=torch.bfloat16, device="cuda")
    y = torch.zeros((1, 8, 8, 16), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(EpidmcError, match="E_SHAPE"):
        D.conv(x, w, None, y, 3)               # 16 output channels: not a multiple of 32
    import ctypes as ct
    lib = D._lib()
    g = torch.zeros((1, 8, 8, 32), dtype=torch.bfloat16, device="cuda")
    dw = torch.zeros((32, 3, 3, 32), dtype=torch.float32, device="cuda")
    scratch = torch.zeros(16, dtype=torch.float32, device="cuda")
    rc = lib.epidmc_dn_wgrad(D._p(x), 32, 32, D._p(g), 32, 32, 1, 8, 8, 3, D._p(dw), None, D._p(scratch), 16,
                             ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -5                            # EPIDMC_E_WORKSPACE: scratch too small


def test_empty_image_uses_unit_scale(D):
    """An all-zero low-count image has no mean to divide by: both sides take s = 1, and the
    output is the learned correction alone."""
    import torch
    P, _, th, _ = net_case(n=1, seed=8)
    noisy = np.zeros((1, 16, 24))
    net = D.Unet(0).bind(1, 16, 24)
    net.set_params(P)
    dev = net.forward(torch.as_tensor(noisy).cuda(), torch.as_tensor(th).cuda()).cpu().numpy()
    ref = U.denoise(P, noisy, th)
    assert np.all(np.isfinite(dev))
    assert rel_l2(dev, ref) < 0.03


def test_forward_replays_from_a_hip_graph(D):
    """The forward pass captured once and replayed: every replay, with new inputs written in
    place and eager work between replays, gives the eager result bit for bit."""
    import torch
    P, noisy, th, _ = net_case(n=2, h=32, w=48, seed=12)
    net = D.Unet(0).bind(2, 32, 48)
    net.set_params(P)
    x = torch.as_tensor(noisy).cuda()
    t = torch.as_tensor(th).cuda()
    out = torch.empty_like(x)
    g = net.capture_forward(x, t, out)
    rng = np.random.default_rng(12)
    for rep in range(4):
        x.copy_(torch.as_tensor(rng.gamma(2.0, 1e-5, noisy.shape)))
        t.copy_(torch.as_tensor(rng.uniform(5, 30, th.shape)))
        g.replay()
        torch.cuda.synchronize()
        replayed = out.clone()
        eager = net.forward(x, t)          # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(replayed, eager), rep
        assert float(replayed.abs().sum()) > 0


def test_weight_moving_average_follows_the_steps(D):
    """With decay d each Adam step sets ema <- d ema + (1 - d) theta; set_params resets it."""
    import torch
    P, noisy, th, target = net_case(seed=14)
    net = D.Unet(0).bind(2, 16, 24)
    net.set_params(P)
    net.set_ema(0.9)
    args = [torch.as_tensor(a).cuda() for a in (noisy, th, target)]
    ema = {k: (W.astype(np.float64), b.astype(np.float64)) for k, (W, b) in P.items()}
    for _ in range(3):
        net.train_step(*args, lr=1e-3)
        cur = net.get_params()
        ema = {k: (0.9 * ema[k][0] + 0.1 * cur[k][0], 0.9 * ema[k][1] + 0.1 * cur[k][1]) for k in ema}
    got = net.get_ema_params()
    for k in ema:
        np.testing.assert_allclose(got[k][0], ema[k][0], rtol=0, atol=1e-6, err_msg=k)
        np.testing.assert_allclose(got[k][1], ema[k][1], rtol=0, atol=1e-6, err_msg=k)
    assert not np.array_equal(got["e1b"][0], net.get_params()["e1b"][0])
    net.set_params(P)                          # resets the average
    np.testing.assert_array_equal(net.get_ema_params()["d0a"][0], P["d0a"][0])
    from paper_2510_24154_amd import EpidmcError
    with pytest.raises(EpidmcError, match="E_ARG"):
        net.set_ema(1.0)


def test_gradient_at_the_training_shape_matches_a_directional_difference(D):
    """At the benchmark's training shape (8 crops of 256 x 256), the loss change along the
    normalised gradient, by a central difference of two GPU forward passes, matches the
    gradient's norm.  The step moves the loss by about 1%, far above the BF16 rounding of
    the loss, so 10% agreement checks the backward pass at full size."""
    import torch
    rng = np.random.default_rng(21)
    n, h, w = 8, 256, 256
    P = synth.unet_params(U.layer_shapes(), seed=21, head_scale=0.05)
    noisy = rng.gamma(2.0, 1e-5, (n, h, w))
    th = rng.uniform(5, 30, (n, h, w))
    target = noisy * rng.uniform(0.8, 1.2, (n, h, w))
    net = D.Unet(0).bind(n, h, w)
    net.set_params(P)
    args = [torch.as_tensor(a).cuda() for a in (noisy, th, target)]
    loss0, g = net.gradient(*args)
    gn = np.sqrt(sum(float(np.sum(gw.astype(np.float64) ** 2) + np.sum(gb.astype(np.float64) ** 2))
                     for gw, gb in g.values()))
    eps = 0.01 * loss0 / gn                    # a step that changes the loss by about 1%
    def moved(sign):
        Q = {k: (W + sign * eps * g[k][0] / gn, b + sign * eps * g[k][1] / gn) for k, (W, b) in P.items()}
        net.set_params(Q)
        return net.gradient(*args)[0]
    d = (moved(+1) - moved(-1)) / (2 * eps)
    print("directional derivative", d, "gradient norm", gn, "loss", loss0)
    assert d == pytest.approx(gn, rel=0.1)
