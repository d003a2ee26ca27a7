"""MI355X (gfx950) EPID transit Monte Carlo engine -- Python binding.

A thin ctypes layer over ``libepidmc.so`` (declared in ``include/epidmc.h``):
argument marshalling only.  Every step of the transport runs in the library's
HIP kernels; PyTorch provides the device memory (the workspace and the output
images) and the stream.  There is no CPU fallback: constructing an Engine
without the built library raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libepidmc.so")

MAX_ELEM = 8
TALLY_FP64, TALLY_FIXED64, TALLY_KAHAN32 = 0, 1, 2
PHYS_KERMA, PHYS_COUPLED = 0, 1
PROC_COMPTON, PROC_PHOTO, PROC_PAIR, DIAG_NO_HARD, DIAG_NO_MSC = 1, 2, 4, 8, 16

STATUS = {0: "OK", -1: "E_ARG", -2: "E_SHAPE", -3: "E_RANGE", -4: "E_NOT_READY", -5: "E_WORKSPACE",
          -6: "E_DEVICE", -7: "E_OVERFLOW", -8: "E_NAN"}


class EpidmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Material(ct.Structure):
    _fields_ = [("n_elem", ct.c_int), ("Z", ct.c_int * MAX_ELEM), ("A", ct.c_double * MAX_ELEM),
                ("w", ct.c_double * MAX_ELEM), ("I_eV", ct.c_double)]


class HUCurve(ct.Structure):
    _fields_ = [("n_points", ct.c_int), ("hu", ct.c_void_p), ("rho", ct.c_void_p),
                ("n_ranges", ct.c_int), ("hu_upper", ct.c_void_p), ("material", ct.c_void_p)]


class Layer(ct.Structure):
    _fields_ = [("material", ct.c_int), ("thickness", ct.c_float), ("density", ct.c_float)]


class Beam(ct.Structure):
    _fields_ = [("kind", ct.c_int), ("src", ct.c_float * 3), ("iso_z", ct.c_float)]


class Particle(ct.Structure):
    _fields_ = [(n, ct.c_float) for n in ("x", "y", "z", "u", "v", "w", "E")] + [("type", ct.c_int)]


class Counters(ct.Structure):
    _fields_ = [(n, ct.c_uint64) for n in (
        "histories", "n_compton", "n_photo", "n_pair", "n_annih", "n_brems", "n_moller",
        "woodcock_steps", "epid_photon_steps", "e_steps_phantom", "e_steps_epid",
        "photon_epid_entries", "unscattered_at_epid", "tally_deposits")] + [
        ("queue_items", ct.c_uint64 * 4), ("lane_iters", ct.c_uint64 * 4), ("wave_iters", ct.c_uint64 * 4),
        ("launches", ct.c_uint64), ("queue_peak", ct.c_uint64), ("error_word", ct.c_uint32),
        ("max_ledger_resid", ct.c_double), ("e_in", ct.c_double), ("e_deposited", ct.c_double),
        ("e_escaped", ct.c_double), ("kernel_ms", ct.c_double * 4), ("kernel_launches", ct.c_uint64 * 4)]

    def as_dict(self):
        d = {}
        for n, _ in self._fields_:
            v = getattr(self, n)
            d[n] = list(v) if isinstance(v, ct.Array) else v
        return d


from .denoise import DN_EXPORTS, declare as declare_denoiser  # noqa: E402

EXPORTS = [
    "epidmc_create", "epidmc_destroy", "epidmc_last_error", "epidmc_set_materials", "epidmc_set_physics",
    "epidmc_set_phantom_hu", "epidmc_set_phantom_direct", "epidmc_set_epid", "epidmc_set_source_spectrum",
    "epidmc_set_source_phsp", "epidmc_set_segments", "epidmc_set_tally", "epidmc_set_diagnostics",
    "epidmc_set_profiling", "epidmc_set_passes", "epidmc_set_graph",
    "epidmc_workspace_size", "epidmc_bind_workspace", "epidmc_run", "epidmc_run_until", "epidmc_read_image",
    "epidmc_sigma_bar", "epidmc_reset_tally", "epidmc_get_counters",
    "epidmc_radiological_thickness", "epidmc_field_size", "epidmc_dose_response",
    "epidmc_resample_response_table",
    "epidmc_debug_philox", "epidmc_debug_sample", "epidmc_debug_table", "epidmc_debug_records",
    "epidmc_debug_queue_capacity",
    "epidmc_microbench",
] + DN_EXPORTS

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libepidmc.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = ct.CDLL(path)
    vp, i32, u32, u64, f32, f64 = ct.c_void_p, ct.c_int, ct.c_uint32, ct.c_uint64, ct.c_float, ct.c_double
    sig = {
        "epidmc_create": [ct.POINTER(vp), i32, u64],
        "epidmc_destroy": [vp],
        "epidmc_set_materials": [vp, ct.POINTER(Material), i32],
        "epidmc_set_physics": [vp, i32, u32, f32, f32],
        "epidmc_set_phantom_hu": [vp, vp, i32, i32, i32, vp, vp, ct.POINTER(HUCurve)],
        "epidmc_set_phantom_direct": [vp, vp, vp, i32, i32, i32, vp, vp],
        "epidmc_set_epid": [vp, ct.POINTER(Layer), i32, i32, f32, i32, i32, f32, f32],
        "epidmc_set_source_spectrum": [vp, vp, vp, i32, ct.POINTER(Beam)],
        "epidmc_set_source_phsp": [vp, ct.POINTER(Particle), u64],
        "epidmc_set_segments": [vp, i32, i32, f32, f32, vp, vp, vp],
        "epidmc_set_tally": [vp, i32, i32, u64],
        "epidmc_set_diagnostics": [vp, i32],
        "epidmc_set_profiling": [vp, i32],
        "epidmc_set_passes": [vp, i32, i32],
        "epidmc_set_graph": [vp, i32, i32],
        "epidmc_workspace_size": [vp, ct.POINTER(ct.c_size_t)],
        "epidmc_bind_workspace": [vp, vp, ct.c_size_t, vp],
        "epidmc_run": [vp, u64, u64, vp],
        "epidmc_run_until": [vp, f64, f64, u64, u64, u64, vp, ct.POINTER(u64), ct.POINTER(f64)],
        "epidmc_read_image": [vp, vp, vp, vp],
        "epidmc_sigma_bar": [vp, f64, vp, ct.POINTER(f64)],
        "epidmc_reset_tally": [vp, vp],
        "epidmc_get_counters": [vp, ct.POINTER(Counters)],
        "epidmc_radiological_thickness": [vp, vp, vp],
        "epidmc_field_size": [vp, ct.POINTER(f64)],
        "epidmc_dose_response": [vp, vp, vp, f64, vp, i32, vp, i32, vp, vp, vp],
        "epidmc_resample_response_table": [vp, i32, vp, i32, vp, vp, i32, vp, i32, vp],
        "epidmc_debug_philox": [vp, vp, vp, u64, vp],
        "epidmc_debug_sample": [vp, i32, f64, f64, f64, vp, u64, vp],
        "epidmc_debug_table": [vp, i32, i32, vp, vp, u64, vp],
        "epidmc_debug_records": [vp, vp, vp, u64, ct.POINTER(u64), vp],
        "epidmc_debug_queue_capacity": [vp, i32, u32],
        "epidmc_microbench": [i32, vp, ct.c_size_t, i32, u32, u32, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ct.c_int
    L.epidmc_last_error.argtypes = [vp]
    L.epidmc_last_error.restype = ct.c_char_p
    declare_denoiser(L)
    _lib = L
    return L


def _f3(v):
    return (ct.c_float * 3)(*[float(x) for x in v])


def _np(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


class Engine:
    """One engine context on one GPU.  Configure with the set_* methods (or from a
    workload description), bind() the workspace, then run()."""

    def __init__(self, device: int = 0, seed: int = 1):
        import torch
        self.torch = torch
        self.L = load_library()
        self.device = torch.device("cuda", device)
        h = ct.c_void_p()
        self._check(self.L.epidmc_create(ct.byref(h), device, int(seed)), ctx=None)
        self.h = h
        self.ws = None
        self._keep = []

    # -- plumbing -------------------------------------------------------------
    def _check(self, rc, ctx="self"):
        if rc != 0:
            msg = self.L.epidmc_last_error(self.h).decode() if ctx is not None else "create failed"
            raise EpidmcError(rc, msg)

    def _stream(self):
        return ct.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            self.L.epidmc_destroy(self.h)
            self.h = None
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- model ------------------------------------------------------------------
    def set_materials(self, mats):
        arr = (Material * len(mats))()
        for i, m in enumerate(mats):
            arr[i].n_elem = len(m["Z"])
            for k, (z, a, w) in enumerate(zip(m["Z"], m["A"], m["w"])):
                arr[i].Z[k], arr[i].A[k], arr[i].w[k] = int(z), float(a), float(w)
            arr[i].I_eV = float(m["I_eV"])
        self._check(self.L.epidmc_set_materials(self.h, arr, len(mats)))

    def set_physics(self, coupled, mask, pcut, ecut):
        self._check(self.L.epidmc_set_physics(self.h, int(coupled), int(mask), float(pcut), float(ecut)))

    def set_phantom_hu(self, hu, shape, spacing, origin, curve, ranges):
        hu = _np(hu, np.int16)
        ch, cr = _np(curve["hu"], np.float64), _np(curve["rho"], np.float64)
        up, mo = _np(ranges["hu_upper"], np.float64), _np(ranges["mat"], np.int32)
        c = HUCurve(ch.size, ch.ctypes.data, cr.ctypes.data, mo.size, up.ctypes.data, mo.ctypes.data)
        nx, ny, nz = shape
        self._check(self.L.epidmc_set_phantom_hu(self.h, hu.ctypes.data, nx, ny, nz, _f3(spacing), _f3(origin),
                                                 ct.byref(c)))

    def set_phantom_direct(self, mat, rho, shape, spacing, origin):
        mat, rho = _np(mat, np.uint8), _np(rho, np.float32)
        nx, ny, nz = shape
        self._check(self.L.epidmc_set_phantom_direct(self.h, mat.ctypes.data, rho.ctypes.data, nx, ny, nz,
                                                     _f3(spacing), _f3(origin)))

    def set_epid(self, layers, scoring, front_z, npx_u, npx_v, pitch_u, pitch_v):
        arr = (Layer * len(layers))(*[Layer(int(l["mat"]), float(l["t"]), float(l["rho"])) for l in layers])
        self._check(self.L.epidmc_set_epid(self.h, arr, len(layers), int(scoring), float(front_z), int(npx_u),
                                           int(npx_v), float(pitch_u), float(pitch_v)))
        self.shape = (int(npx_v), int(npx_u))

    def set_source_spectrum(self, edges, weights, beam):
        e, w = _np(edges, np.float32), _np(weights, np.float32)
        b = Beam(int(beam["kind"]), _f3(beam["src"]), float(beam["iso_z"]))
        self._check(self.L.epidmc_set_source_spectrum(self.h, e.ctypes.data, w.ctypes.data, w.size, ct.byref(b)))

    def set_source_phsp(self, particles):
        p = _np(particles, np.float64).reshape(-1, 8)
        arr = (Particle * len(p))()
        for i, q in enumerate(p):
            arr[i] = Particle(*[float(x) for x in q[:7]], int(q[7]))
        self._check(self.L.epidmc_set_source_phsp(self.h, arr, len(p)))

    def set_segments(self, a, b, leaf_w, y0, counts=None):
        a, b = _np(a, np.float32), _np(b, np.float32)
        n_seg, n_pairs = a.shape
        cnt = _np(counts if counts is not None else np.zeros(n_seg), np.uint64)
        self._check(self.L.epidmc_set_segments(self.h, n_seg, n_pairs, float(leaf_w), float(y0), a.ctypes.data,
                                               b.ctypes.data, cnt.ctypes.data))

    def set_tally(self, mode=TALLY_FP64, batches=64, max_chunk=1 << 21):
        self._check(self.L.epidmc_set_tally(self.h, int(mode), int(batches), int(max_chunk)))

    def set_diagnostics(self, on=True):
        self._check(self.L.epidmc_set_diagnostics(self.h, 1 if on else 0))

    def set_profiling(self, on=True):
        self._check(self.L.epidmc_set_profiling(self.h, 1 if on else 0))

    def set_passes(self, device_passes=-1, items_per_lane=2):
        self._check(self.L.epidmc_set_passes(self.h, int(device_passes), int(items_per_lane)))

    def set_graph(self, on=True, passes=0):
        self._check(self.L.epidmc_set_graph(self.h, 1 if on else 0, int(passes)))

    def configure(self, cfg, tally=TALLY_FP64, batches=64, max_chunk=1 << 21, diag=False, phsp=None):
        """Apply a workload description (see paper_2510_24154_amd.synth)."""
        self.set_materials(cfg["materials"])
        ph = cfg["physics"]
        self.set_physics(ph["coupled"], ph["proc_mask"], ph["pcut"], ph["ecut"])
        P = cfg["phantom"]
        if P["kind"] == "hu":
            self.set_phantom_hu(P["hu"], P["shape"], P["spacing"], P["origin"], P["curve"], P["ranges"])
        else:
            self.set_phantom_direct(P["mat"], P["rho"], P["shape"], P["spacing"], P["origin"])
        E = cfg["epid"]
        self.set_epid(E["layers"], E["scoring"], E["front_z"], E["npx_u"], E["npx_v"], E["pitch_u"], E["pitch_v"])
        S = cfg["source"]
        self.set_source_spectrum(S["edges"], S["weights"], S["beam"])
        ap = S["aperture"]
        self.set_segments(ap["a"], ap["b"], ap["leaf_w"], ap["y0"], ap["counts"])
        if phsp is not None:
            self.set_source_phsp(phsp)
        self.set_tally(tally, batches, max_chunk)
        self.set_diagnostics(diag)
        return self

    # -- memory and runs ----------------------------------------------------------
    def workspace_size(self):
        n = ct.c_size_t()
        self._check(self.L.epidmc_workspace_size(self.h, ct.byref(n)))
        return n.value

    def bind(self):
        n = self.workspace_size()
        self.ws = self.torch.empty(n + 256, dtype=self.torch.uint8, device=self.device)
        ptr = self.ws.data_ptr()
        off = (-ptr) % 256
        self._check(self.L.epidmc_bind_workspace(self.h, ct.c_void_p(ptr + off), n, self._stream()))
        return n

    def run(self, n, first=0):
        self._check(self.L.epidmc_run(self.h, int(first), int(n), self._stream()))

    def run_until(self, target, thr=0.5, first=0, step=1_000_000, max_hist=1 << 31):
        done, sb = ct.c_uint64(), ct.c_double()
        self._check(self.L.epidmc_run_until(self.h, float(target), float(thr), int(first), int(step), int(max_hist),
                                            self._stream(), ct.byref(done), ct.byref(sb)))
        return done.value, sb.value

    def image(self):
        t = self.torch
        mean = t.empty(self.shape, dtype=t.float64, device=self.device)
        var = t.empty(self.shape, dtype=t.float64, device=self.device)
        self._check(self.L.epidmc_read_image(self.h, ct.c_void_p(mean.data_ptr()), ct.c_void_p(var.data_ptr()),
                                             self._stream()))
        return mean, var

    def radiological_thickness(self):
        """Per-pixel radiological thickness (cm), a float64 device tensor of the image shape."""
        out = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        self._check(self.L.epidmc_radiological_thickness(self.h, ct.c_void_p(out.data_ptr()), self._stream()))
        return out

    def field_size(self):
        out = ct.c_double()
        self._check(self.L.epidmc_field_size(self.h, ct.byref(out)))
        return out.value

    def dose_response(self, image, thickness, s, t_nodes, s_nodes, k):
        """k(thickness, s) * image on the device, k bilinear on the table k[s_j][t_i]."""
        t = self.torch
        img = image.to(device=self.device, dtype=t.float64).contiguous()
        th = thickness.to(device=self.device, dtype=t.float64).contiguous()
        npix = self.shape[0] * self.shape[1]
        if img.numel() != npix or th.numel() != npix:
            raise ValueError(f"image and thickness need {npix} pixels, got {img.numel()} and {th.numel()}")
        out = t.empty_like(img)
        tn = np.ascontiguousarray(t_nodes, dtype=np.float64)
        sn = np.ascontiguousarray(s_nodes, dtype=np.float64)
        kk = np.ascontiguousarray(k, dtype=np.float64)
        self._check(self.L.epidmc_dose_response(self.h, ct.c_void_p(img.data_ptr()), ct.c_void_p(th.data_ptr()),
                                                float(s), tn.ctypes.data, tn.size, sn.ctypes.data, sn.size,
                                                kk.ctypes.data, ct.c_void_p(out.data_ptr()), self._stream()))
        return out

    def sigma_bar(self, thr=0.5):
        out = ct.c_double()
        self._check(self.L.epidmc_sigma_bar(self.h, float(thr), self._stream(), ct.byref(out)))
        return out.value

    def reset(self):
        self._check(self.L.epidmc_reset_tally(self.h, self._stream()))

    def counters(self):
        c = Counters()
        self._check(self.L.epidmc_get_counters(self.h, ct.byref(c)))
        return c.as_dict()

    # -- probes of the device building blocks ------------------------------------------
    def debug_philox(self, ctr):
        t = self.torch
        ctr = t.as_tensor(np.asarray(ctr, dtype=np.uint32).view(np.int32), device=self.device).contiguous()
        out = t.empty_like(ctr)
        n = ctr.numel() // 4
        self._check(self.L.epidmc_debug_philox(self.h, ct.c_void_p(ctr.data_ptr()), ct.c_void_p(out.data_ptr()), n,
                                               self._stream()))
        return out.cpu().numpy().view(np.uint32).reshape(-1, 4)

    def debug_sample(self, kind, n, p0=0.0, p1=0.0, p2=0.0):
        t = self.torch
        width = 8 if kind == 4 else 1
        out = t.empty(n * width, dtype=t.float32, device=self.device)
        self._check(self.L.epidmc_debug_sample(self.h, int(kind), float(p0), float(p1), float(p2),
                                               ct.c_void_p(out.data_ptr()), int(n), self._stream()))
        return out.cpu().numpy().reshape(n, width) if width > 1 else out.cpu().numpy()

    def debug_queue_capacity(self, kind, per_segment):
        """Test hook: particles per segment of queue `kind` (1-3) from the next bind on (0: the
        size derived from the chunk).  Unbinds."""
        self._check(self.L.epidmc_debug_queue_capacity(self.h, int(kind), int(per_segment)))

    def debug_records(self, cap):
        """Kahan-mode deposit records of the last chunk: (image element, MeV) as numpy arrays
        and the chunk's record count."""
        t = self.torch
        pix = t.empty(max(1, cap), dtype=t.int32, device=self.device)
        e = t.empty(max(1, cap), dtype=t.float32, device=self.device)
        n = ct.c_uint64()
        self._check(self.L.epidmc_debug_records(self.h, ct.c_void_p(pix.data_ptr()), ct.c_void_p(e.data_ptr()), int(cap),
                                                ct.byref(n), self._stream()))
        k = min(cap, n.value)
        return pix[:k].cpu().numpy().view(np.uint32), e[:k].cpu().numpy(), n.value

    def debug_table(self, kind, index, energies):
        t = self.torch
        E = t.as_tensor(np.asarray(energies, dtype=np.float32), device=self.device).contiguous()
        out = t.empty_like(E)
        self._check(self.L.epidmc_debug_table(self.h, int(kind), int(index), ct.c_void_p(E.data_ptr()),
                                              ct.c_void_p(out.data_ptr()), E.numel(), self._stream()))
        return out.cpu().numpy()


def resample_response_table(t_nodes, s_nodes, k, t_out, s_out):
    """k(t, s) resampled onto the nodes t_out x s_out (epidmc_resample_response_table, host
    code of the engine): returns k_out[j][i] at (t_out[i], s_out[j])."""
    L = load_library()
    tn = np.ascontiguousarray(t_nodes, dtype=np.float64)
    sn = np.ascontiguousarray(s_nodes, dtype=np.float64)
    kk = np.ascontiguousarray(k, dtype=np.float64).reshape(sn.size, tn.size)
    to = np.ascontiguousarray(t_out, dtype=np.float64)
    so = np.ascontiguousarray(s_out, dtype=np.float64)
    out = np.empty((so.size, to.size), dtype=np.float64)
    st = L.epidmc_resample_response_table(tn.ctypes.data, tn.size, sn.ctypes.data, sn.size, kk.ctypes.data,
                                          to.ctypes.data, to.size, so.ctypes.data, so.size, out.ctypes.data)
    if st != 0:
        raise ValueError(f"epidmc_resample_response_table failed: status {st}")
    return out


MB_COPY, MB_GATHER, MB_ATOMIC_F64, MB_ATOMIC_I64 = 0, 1, 2, 3


def microbench(kind, buf, log2_elems=0, ops_per_thread=0, threads=0):
    """Launch one measurement probe (epidmc_microbench) on torch's current stream over the
    device tensor `buf` (its bytes are overwritten); the caller times it."""
    import torch
    L = load_library()
    rc = L.epidmc_microbench(int(kind), ct.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                             int(log2_elems), int(ops_per_thread), int(threads),
                             ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise EpidmcError(rc, "epidmc_microbench")
