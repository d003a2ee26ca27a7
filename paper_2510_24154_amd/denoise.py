"""Python binding of the learned denoiser (include/epidmc_denoise.h): argument marshalling
only.  Every layer runs in the HIP kernels of libepidmc.so; torch supplies device memory
and the stream.  A noisy low-count image and its radiological-thickness map go in; the
denoised image comes out (Sec. 4.1 proposes replacing a long simulation by a short one
plus a trained network)."""
from __future__ import annotations

import ctypes as ct

import numpy as np

DN_EXPORTS = [
    "epidmc_dn_conv", "epidmc_dn_wgrad_scratch", "epidmc_dn_wgrad", "epidmc_dn_wgrad_noalloc",
    "epidmc_dn_weights", "epidmc_dn_pool",
    "epidmc_dn_upsample", "epidmc_dn_upsample_backward", "epidmc_dn_skip_backward",
    "epidmc_unet_create", "epidmc_unet_destroy", "epidmc_unet_last_error", "epidmc_unet_param_count",
    "epidmc_unet_layer", "epidmc_unet_layers", "epidmc_unet_workspace_size", "epidmc_unet_bind",
    "epidmc_unet_set_params", "epidmc_unet_get_params", "epidmc_unet_forward", "epidmc_unet_gradient",
    "epidmc_unet_train_step", "epidmc_unet_set_ema", "epidmc_unet_get_ema_params",
]


def declare(L):
    """Argument types of the denoiser entry points on the loaded library."""
    vp, i32, f32, sz = ct.c_void_p, ct.c_int, ct.c_float, ct.c_size_t
    sig = {
        "epidmc_dn_conv": [vp, i32, i32, vp, vp, vp, i32, i32, vp, i32, i32, i32, i32, i32, i32, vp],
        "epidmc_dn_wgrad_scratch": [i32, i32, i32, i32, i32, i32, ct.POINTER(sz)],
        "epidmc_dn_wgrad": [vp, i32, i32, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp, sz, vp],
        "epidmc_dn_wgrad_noalloc": [vp, i32, i32, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp],
        "epidmc_dn_weights": [vp, i32, i32, i32, vp, vp, vp],
        "epidmc_dn_pool": [vp, i32, vp, i32, i32, i32, i32, i32, vp],
        "epidmc_dn_upsample": [vp, i32, vp, i32, i32, i32, i32, i32, vp],
        "epidmc_dn_upsample_backward": [vp, i32, vp, i32, i32, i32, i32, i32, vp],
        "epidmc_dn_skip_backward": [vp, i32, vp, i32, vp, i32, vp, i32, i32, i32, i32, i32, vp],
        "epidmc_unet_create": [ct.POINTER(vp), i32],
        "epidmc_unet_destroy": [vp],
        "epidmc_unet_param_count": [vp, ct.POINTER(sz)],
        "epidmc_unet_layer": [vp, i32, ct.c_char_p, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32),
                              ct.POINTER(sz), ct.POINTER(sz)],
        "epidmc_unet_workspace_size": [vp, i32, i32, i32, ct.POINTER(sz)],
        "epidmc_unet_bind": [vp, vp, sz, i32, i32, i32, vp],
        "epidmc_unet_set_params": [vp, vp, vp],
        "epidmc_unet_get_params": [vp, vp, vp],
        "epidmc_unet_forward": [vp, vp, vp, vp, i32, vp],
        "epidmc_unet_gradient": [vp, vp, vp, vp, i32, vp, vp, vp],
        "epidmc_unet_train_step": [vp, vp, vp, vp, i32, f32, vp, vp],
        "epidmc_unet_set_ema": [vp, f32],
        "epidmc_unet_get_ema_params": [vp, vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ct.c_int
    L.epidmc_unet_layers.argtypes = [vp]
    L.epidmc_unet_layers.restype = ct.c_int
    L.epidmc_unet_last_error.argtypes = [vp]
    L.epidmc_unet_last_error.restype = ct.c_char_p


def _lib():
    from . import load_library
    return load_library()


def _p(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _stream(torch):
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(code, what):
    if code != 0:
        from . import EpidmcError
        raise EpidmcError(code, what)


# ---- layer operations (BF16 tensors of shape (n, h, w, channels) or channel slices) ----
def _ld(t):
    return t.stride(2)


def conv(x, w_bf16, bias, y, k, relu=True, gate=None):
    """y = act(conv_k(x, w) + bias) on the device; x, y, gate torch.bfloat16 NHWC (channel
    slices allowed), w_bf16 (c_out, k, k, c_in) bfloat16, bias float32 or None."""
    import torch
    n, h, wd, ci = x.shape
    co = y.shape[3]
    _check(_lib().epidmc_dn_conv(_p(x), _ld(x), ci, _p(w_bf16), _p(bias), _p(y), _ld(y), co, _p(gate),
                                 _ld(gate) if gate is not None else 0, n, h, wd, k, int(relu), _stream(torch)),
           "epidmc_dn_conv")
    return y


def wgrad(x, g, k, with_bias=True):
    """(dW float32 (c_out, k, k, c_in), db float32 (c_out,) or None) on the device."""
    import torch
    n, h, wd, ci = x.shape
    co = g.shape[3]
    fl = ct.c_size_t()
    _check(_lib().epidmc_dn_wgrad_scratch(n, h, wd, k, ci, co, ct.byref(fl)), "epidmc_dn_wgrad_scratch")
    scratch = torch.empty(max(1, fl.value), dtype=torch.float32, device=x.device)
    dw = torch.empty((co, k, k, ci), dtype=torch.float32, device=x.device)
    db = torch.empty(co, dtype=torch.float32, device=x.device) if with_bias else None
    _check(_lib().epidmc_dn_wgrad(_p(x), _ld(x), ci, _p(g), _ld(g), co, n, h, wd, k, _p(dw), _p(db), _p(scratch),
                                  fl.value, _stream(torch)), "epidmc_dn_wgrad")
    return dw, db


# floats of the library-held scratch of epidmc_dn_wgrad_noalloc (EPIDMC_DN_WGRAD_NOALLOC_FLOATS)
WGRAD_NOALLOC_FLOATS = 10 << 20


def wgrad_noalloc(x, g, k, with_bias=True, dw=None, db=None):
    """epidmc_dn_wgrad with the library's own scratch (the call allocates nothing; dw and db
    are allocated here unless given)."""
    import torch
    n, h, wd, ci = x.shape
    co = g.shape[3]
    if dw is None:
        dw = torch.empty((co, k, k, ci), dtype=torch.float32, device=x.device)
    if db is None and with_bias:
        db = torch.empty(co, dtype=torch.float32, device=x.device)
    _check(_lib().epidmc_dn_wgrad_noalloc(_p(x), _ld(x), ci, _p(g), _ld(g), co, n, h, wd, k, _p(dw),
                                          _p(db) if with_bias else None, _stream(torch)),
           "epidmc_dn_wgrad_noalloc")
    return dw, (db if with_bias else None)


def weights(w_f32, backward=True):
    """(w_fwd, w_bwd) bfloat16 copies of float32 weights (c_out, k, k, c_in)."""
    import torch
    co, k, _, ci = w_f32.shape
    wf = torch.empty_like(w_f32, dtype=torch.bfloat16)
    wb = torch.empty((ci, k, k, co), dtype=torch.bfloat16, device=w_f32.device) if backward else None
    _check(_lib().epidmc_dn_weights(_p(w_f32.contiguous()), co, k, ci, _p(wf), _p(wb), _stream(torch)),
           "epidmc_dn_weights")
    return wf, wb


def pool(x, y):
    import torch
    n, h, wd, c = x.shape
    _check(_lib().epidmc_dn_pool(_p(x), _ld(x), _p(y), _ld(y), c, n, h, wd, _stream(torch)), "epidmc_dn_pool")
    return y


def upsample(x, y):
    import torch
    n, h, wd, c = x.shape
    _check(_lib().epidmc_dn_upsample(_p(x), _ld(x), _p(y), _ld(y), c, n, h, wd, _stream(torch)),
           "epidmc_dn_upsample")
    return y


def upsample_backward(g, y):
    import torch
    n, h, wd, c = g.shape
    _check(_lib().epidmc_dn_upsample_backward(_p(g), _ld(g), _p(y), _ld(y), c, n, h, wd, _stream(torch)),
           "epidmc_dn_upsample_backward")
    return y


def skip_backward(g_skip, g_pool, act, out):
    import torch
    n, h, wd, c = g_skip.shape
    _check(_lib().epidmc_dn_skip_backward(_p(g_skip), _ld(g_skip), _p(g_pool), _ld(g_pool), _p(act), _ld(act),
                                          _p(out), _ld(out), c, n, h, wd, _stream(torch)), "epidmc_dn_skip_backward")
    return out


# ---- the network ----------------------------------------------------------------------
class Unet:
    """The 4-level U-Net on one GPU.  Parameters travel as {name: (W (c_out, k, k, c_in),
    b (c_out,))} with the first layer's c_in = 2 (the library pads it to 8 with zeros)."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.L = _lib()
        self.dev = torch.device("cuda", device)
        h = ct.c_void_p()
        _check(self.L.epidmc_unet_create(ct.byref(h), device), "epidmc_unet_create")
        self.h = h
        n = ct.c_size_t()
        self._c(self.L.epidmc_unet_param_count(self.h, ct.byref(n)), "param_count")
        self.nparam = n.value
        self.layers = []
        for i in range(self.L.epidmc_unet_layers(self.h)):
            nm = ct.create_string_buffer(8)
            k, ci, co = ct.c_int(), ct.c_int(), ct.c_int()
            ow, ob = ct.c_size_t(), ct.c_size_t()
            self._c(self.L.epidmc_unet_layer(self.h, i, nm, ct.byref(k), ct.byref(ci), ct.byref(co), ct.byref(ow),
                                             ct.byref(ob)), "layer")
            self.layers.append((nm.value.decode(), k.value, ci.value, co.value, ow.value, ob.value))
        self.ws = None

    def _c(self, code, what):
        if code != 0:
            from . import EpidmcError
            msg = self.L.epidmc_unet_last_error(self.h).decode(errors="replace")
            raise EpidmcError(code, f"{what}: {msg}")

    def __del__(self):
        try:
            self.L.epidmc_unet_destroy(self.h)
        except Exception:
            pass

    def bind(self, n, h, w):
        t = self.torch
        b = ct.c_size_t()
        self._c(self.L.epidmc_unet_workspace_size(self.h, n, h, w, ct.byref(b)), "workspace_size")
        self.ws = t.empty(b.value + 256, dtype=t.uint8, device=self.dev)
        base = (self.ws.data_ptr() + 255) // 256 * 256
        self._c(self.L.epidmc_unet_bind(self.h, ct.c_void_p(base), b.value, n, h, w, _stream(t)), "bind")
        self.shape = (n, h, w)
        return self

    def shapes(self):
        """(name, k, c_in, c_out) of every layer as the parameters travel (c_in = 2 first)."""
        return [(nm, k, 2 if nm == "e0a" else ci, co) for nm, k, ci, co, _, _ in self.layers]

    def flat(self, params):
        """Flat FP32 parameter vector (host numpy) from {name: (W, b)}."""
        v = np.zeros(self.nparam, np.float32)
        for name, k, ci, co, ow, ob in self.layers:
            W, b = params[name]
            W = np.asarray(W, np.float32)
            if W.shape[3] < ci:
                W = np.concatenate([W, np.zeros(W.shape[:3] + (ci - W.shape[3],), np.float32)], axis=3)
            assert W.shape == (co, k, k, ci), (name, W.shape)
            v[ow:ow + W.size] = W.reshape(-1)
            v[ob:ob + co] = np.asarray(b, np.float32)
        return v

    def unflat(self, v, cin0=2):
        out = {}
        for name, k, ci, co, ow, ob in self.layers:
            W = np.asarray(v[ow:ow + co * k * k * ci]).reshape(co, k, k, ci)
            if name == "e0a":
                W = W[..., :cin0]
            out[name] = (W.copy(), np.asarray(v[ob:ob + co]).copy())
        return out

    def set_params(self, params):
        t = self.torch
        d = t.as_tensor(self.flat(params), device=self.dev)
        self._c(self.L.epidmc_unet_set_params(self.h, _p(d), _stream(t)), "set_params")
        t.cuda.current_stream().synchronize()

    def get_params(self):
        t = self.torch
        d = t.empty(self.nparam, dtype=t.float32, device=self.dev)
        self._c(self.L.epidmc_unet_get_params(self.h, _p(d), _stream(t)), "get_params")
        return self.unflat(d.cpu().numpy())

    def set_ema(self, decay):
        """Keep an exponential moving average of the weights with this decay (0: off)."""
        self._c(self.L.epidmc_unet_set_ema(self.h, float(decay)), "set_ema")

    def get_ema_params(self):
        t = self.torch
        d = t.empty(self.nparam, dtype=t.float32, device=self.dev)
        self._c(self.L.epidmc_unet_get_ema_params(self.h, _p(d), _stream(t)), "get_ema_params")
        return self.unflat(d.cpu().numpy())

    def forward(self, noisy, thickness, out=None):
        """Denoised images from FP64 device tensors (n, h, w)."""
        t = self.torch
        n = noisy.shape[0]
        out = t.empty_like(noisy) if out is None else out
        self._c(self.L.epidmc_unet_forward(self.h, _p(noisy), _p(thickness), _p(out), n, _stream(t)), "forward")
        return out

    def capture_forward(self, noisy, thickness, out):
        """Record one forward pass over these (fixed) FP64 device tensors into a HIP graph and
        return it; graph.replay() then re-runs the whole pass (about 30 kernels) with one
        launch.  The pass issues kernels only (no memory set, copy or synchronisation), so
        it can be captured; refresh the tensors' contents in place between replays."""
        t = self.torch
        n = noisy.shape[0]
        t.cuda.synchronize()
        g = t.cuda.CUDAGraph()
        with t.cuda.graph(g):
            self._c(self.L.epidmc_unet_forward(self.h, _p(noisy), _p(thickness), _p(out), n, _stream(t)),
                    "forward")
        return g

    def gradient(self, noisy, thickness, target):
        """(loss, {name: (dW, db)}) for a batch (FP64 device tensors (n, h, w))."""
        t = self.torch
        g = t.empty(self.nparam, dtype=t.float32, device=self.dev)
        loss = t.empty(1, dtype=t.float64, device=self.dev)
        self._c(self.L.epidmc_unet_gradient(self.h, _p(noisy), _p(thickness), _p(target), noisy.shape[0], _p(g),
                                            _p(loss), _stream(t)), "gradient")
        return float(loss.item()), self.unflat(g.cpu().numpy())

    def train_step(self, noisy, thickness, target, lr, loss=None):
        """One Adam step; the loss goes to the FP64 device scalar `loss` when given."""
        t = self.torch
        self._c(self.L.epidmc_unet_train_step(self.h, _p(noisy), _p(thickness), _p(target), noisy.shape[0],
                                              float(lr), _p(loss), _stream(t)), "train_step")


# ---- training data and training --------------------------------------------------------
def make_pairs(fields, n_low, n_high, seed=1, max_chunk=1 << 24, device=0, engine=None, report=None):
    """Low- and high-count images and radiological-thickness maps of a list of field
    configurations, each transported by the engine on the GPU.  Returns (low, high,
    thickness), FP64 device tensors of shape (fields, npx_v, npx_u).  For a one-segment
    field the low image takes history ids [0, n_low) and the high one [n_low, n_low +
    n_high); a field of several segments is delivered whole at each count, by two engines
    of different seeds.  Either way the two are independent estimates of the same expected
    image."""
    import torch
    from . import Engine, synth
    eng = engine or Engine(device, seed)
    eng_hi = None
    low = high = th = None
    chunk = int(min(max_chunk, max(n_low, n_high)))
    for i, cfg in enumerate(fields):
        segmented = np.asarray(cfg["source"]["aperture"]["a"]).shape[0] > 1
        if segmented:
            # a field of several segments is delivered whole at each count: the low image
            # by one engine, the high one by a second engine with another seed
            eng.configure(synth.with_histories_scaled(cfg, int(n_low)), batches=64, max_chunk=chunk)
        else:
            eng.configure(cfg, batches=64, max_chunk=chunk)
        eng.bind()
        eng.run(int(n_low))
        a = eng.image()[0]
        if low is None:
            shape = (len(fields),) + tuple(a.shape)
            low, high, th = (torch.empty(shape, dtype=torch.float64, device=a.device) for _ in range(3))
        low[i] = a
        th[i] = eng.radiological_thickness()
        if segmented:
            if eng_hi is None:
                eng_hi = Engine(device, seed + 7919)
            eng_hi.configure(synth.with_histories_scaled(cfg, int(n_high)), batches=64, max_chunk=chunk)
            eng_hi.bind()
            eng_hi.run(int(n_high))
            high[i] = eng_hi.image()[0]
        else:
            eng.reset()
            eng.run(int(n_high), first=int(n_low))
            high[i] = eng.image()[0]
        if report and (i + 1) % report == 0:
            print(f"[denoiser] {i + 1}/{len(fields)} fields transported", flush=True)
    torch.cuda.synchronize()
    return low, high, th


def train(net, low, high, th, steps, batch=8, crop=None, lr=1e-3, lr_end=1e-4, seed=0, report=None):
    """Adam on random crops (crop x crop, aligned to 8 pixels) of random training images
    with random horizontal and vertical flips; the learning rate falls from lr to lr_end on
    a cosine.  Returns the per-step losses (host numpy)."""
    import math
    import torch
    rng = np.random.default_rng(seed)
    N, H, W = low.shape
    ch, cw = (H, W) if crop is None else (min(crop, H), min(crop, W))
    loss = torch.zeros(steps, dtype=torch.float64, device=low.device)
    for it in range(steps):
        idx = torch.as_tensor(rng.integers(0, N, batch), device=low.device)
        r0 = 8 * int(rng.integers(0, (H - ch) // 8 + 1))
        c0 = 8 * int(rng.integers(0, (W - cw) // 8 + 1))
        parts = []
        for t in (low, th, high):
            x = t[idx, r0:r0 + ch, c0:c0 + cw]
            parts.append(x)
        if rng.random() < 0.5:
            parts = [x.flip(1) for x in parts]
        if rng.random() < 0.5:
            parts = [x.flip(2) for x in parts]
        parts = [x.contiguous() for x in parts]
        a = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * it / max(1, steps - 1)))
        net.train_step(parts[0], parts[1], parts[2], a, loss=loss[it:it + 1])
        if report and (it + 1) % report == 0:
            print(f"[denoiser] step {it + 1}/{steps} loss {float(loss[it]):.5g}", flush=True)
    return loss.cpu().numpy()
