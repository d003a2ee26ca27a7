"""CPU oracle of the EPID transit Monte Carlo hot path -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The engine (``paper_2510_24154_amd``)
never imports, links or calls it.

This module only marshals a workload description (see
``paper_2510_24154_amd.synth``) into the C structures of ``epid_oracle.h``; all
arithmetic is in ``epid_oracle.c``.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libepid_oracle.so")
MAX_ELEM, MAX_MAT, MAX_LAYERS = 8, 16, 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-Wall", "-fPIC", "-shared", "-o", tmp,
                               os.path.join(_HERE, "epid_oracle.c"), "-lm", "-lpthread"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Material(ct.Structure):
    _fields_ = [("n_elem", ct.c_int), ("Z", ct.c_int * MAX_ELEM), ("A", ct.c_double * MAX_ELEM),
                ("w", ct.c_double * MAX_ELEM), ("I_eV", ct.c_double)]


class Config(ct.Structure):
    _fields_ = [
        ("coupled", ct.c_int), ("proc_mask", ct.c_uint32), ("pcut", ct.c_double), ("ecut", ct.c_double),
        ("n_mat", ct.c_int), ("mat", Material * MAX_MAT),
        ("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
        ("spacing", ct.c_double * 3), ("origin", ct.c_double * 3),
        ("vox_mat", ct.POINTER(ct.c_uint8)), ("vox_rho", ct.POINTER(ct.c_double)),
        ("n_layers", ct.c_int), ("layer_mat", ct.c_int * MAX_LAYERS),
        ("layer_rho", ct.c_double * MAX_LAYERS), ("layer_t", ct.c_double * MAX_LAYERS),
        ("scoring_layer", ct.c_int), ("front_z", ct.c_double),
        ("npx_u", ct.c_int), ("npx_v", ct.c_int), ("pitch_u", ct.c_double), ("pitch_v", ct.c_double),
        ("beam_kind", ct.c_int), ("src", ct.c_double * 3), ("iso_z", ct.c_double),
        ("nbins", ct.c_int), ("edges", ct.POINTER(ct.c_double)), ("weights", ct.POINTER(ct.c_double)),
        ("n_seg", ct.c_int), ("n_pairs", ct.c_int), ("leaf_w", ct.c_double), ("y0", ct.c_double),
        ("a", ct.POINTER(ct.c_double)), ("b", ct.POINTER(ct.c_double)),
        ("seg_hist", ct.POINTER(ct.c_uint64)),
        ("n_phsp", ct.c_uint64), ("phsp", ct.POINTER(ct.c_double)),
        ("seed", ct.c_uint64),
        ("step_floor", ct.c_double),
    ]


# event kinds of the trace (epid_oracle.h, orc_event)
EV_DEPOSIT, EV_ESTEP, EV_COMPTON, EV_PHOTO, EV_PAIR, EV_ANNIH, EV_MOLLER, EV_BREMS, EV_NULL = range(9)


class Event(ct.Structure):
    _fields_ = [("hist", ct.c_uint64), ("kind", ct.c_int32), ("region", ct.c_int32), ("layer", ct.c_int32),
                ("pixel", ct.c_int32), ("pos", ct.c_double * 3), ("E0", ct.c_double), ("E1", ct.c_double),
                ("d0", ct.c_double * 3), ("d1", ct.c_double * 3), ("Ec", ct.c_double * 2),
                ("dc", (ct.c_double * 3) * 2), ("aux", ct.c_double * 2)]


EVENT_DTYPE = np.dtype([("hist", np.uint64), ("kind", np.int32), ("region", np.int32), ("layer", np.int32),
                        ("pixel", np.int32), ("pos", np.float64, 3), ("E0", np.float64), ("E1", np.float64),
                        ("d0", np.float64, 3), ("d1", np.float64, 3), ("Ec", np.float64, 2),
                        ("dc", np.float64, (2, 3)), ("aux", np.float64, 2)])
assert EVENT_DTYPE.itemsize == ct.sizeof(Event)
# floor on boundary-limited electron steps, as a fraction of the cell's smallest side: 0 in the
# reading (a step never crosses a face); a test sets another value to measure what a floor does
STEP_FLOOR = 0.0


class Counters(ct.Structure):
    _fields_ = [(n, ct.c_uint64) for n in (
        "n_hist", "n_compton", "n_photo", "n_pair", "n_annih", "n_brems", "n_moller",
        "e_steps", "voxel_visits", "photon_epid_entries", "unscattered_at_epid", "n_tally_deposits",
        "n_first_collision")] + \
        [(n, ct.c_double) for n in (
            "e_first_collision", "e_track", "e_in", "e_dep_phantom", "e_dep_epid", "e_dep_other", "e_escaped", "e_rest_balance",
            "max_ledger_resid")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None
_override = None
_lock = threading.Lock()


class using:
    """Context manager: route every call of this module through the oracle library at
    `path` (a test build of the oracle's source) instead of the default one."""

    def __init__(self, path: str):
        self.L = _declare(ct.CDLL(path))

    def __enter__(self):
        global _override
        self.prev, _override = _override, self.L
        return self.L

    def __exit__(self, *exc):
        global _override
        _override = self.prev
        return False


def lib():
    global _lib
    if _override is not None:
        return _override
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                build()
            _lib = _declare(ct.CDLL(LIB_PATH))
    return _lib


def _declare(L):
    d, p = ct.c_double, ct.c_void_p
    L.orc_run.argtypes = [ct.POINTER(Config), ct.c_uint64, ct.c_uint64, p, p, ct.POINTER(Counters)]
    L.orc_run.restype = ct.c_int
    L.orc_run_traced.argtypes = [ct.POINTER(Config), ct.c_uint64, ct.c_uint64, p, p, ct.POINTER(Counters),
                                 p, ct.c_uint64, ct.POINTER(ct.c_uint64)]
    L.orc_run_traced.restype = ct.c_int
    L.orc_map_hu.argtypes = [p, ct.c_uint64, ct.c_int, p, p, ct.c_int, p, p, p, p]
    L.orc_map_hu.restype = ct.c_int
    for name, args in {
        "orc_sigma_kn": [d], "orc_kn_sample": [d, d], "orc_kn_cdf": [d, d],
        "orc_x0": [ct.POINTER(Material)], "orc_highland": [d, d, d],
        "orc_lcol": [ct.POINTER(Material), d, ct.c_int, d],
        "orc_lres": [ct.POINTER(Material), d, d, d],
        "orc_sigma_moller": [ct.POINTER(Material), d, d],
        "orc_sigma_brems": [ct.POINTER(Material), d, d],
        "orc_moller_sample": [d, d, d],
        "orc_brems_sample": [d, d, d],
        "orc_srad": [ct.POINTER(Material), d],
        "orc_sigma_hard_max": [ct.POINTER(Material), d, d, d],
        "orc_range_diff": [ct.POINTER(Material), d, d, d, d],
        "orc_range_inverse": [ct.POINTER(Material), d, d, d, d],
    }.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = d
    L.orc_source.argtypes = [ct.POINTER(Config), ct.c_uint64, p]
    L.orc_source.restype = ct.c_int
    L.orc_photon_mu.argtypes = [ct.POINTER(Material), d, p]
    L.orc_photon_mu.restype = None
    L.orc_philox4x32_10.argtypes = [p, p, p]
    L.orc_philox4x32_10.restype = None
    L.orc_radiological_thickness.argtypes = [ct.POINTER(Config), p]
    L.orc_radiological_thickness.restype = ct.c_int
    L.orc_equivalent_square.argtypes = [ct.POINTER(Config)]
    L.orc_equivalent_square.restype = d
    L.orc_response_factor.argtypes = [p, ct.c_int, p, ct.c_int, p, d, d]
    L.orc_response_factor.restype = d
    return L


def material(m: dict) -> Material:
    s = Material()
    s.n_elem = len(m["Z"])
    for i, (z, a, w) in enumerate(zip(m["Z"], m["A"], m["w"])):
        s.Z[i], s.A[i], s.w[i] = int(z), float(a), float(w)
    s.I_eV = float(m["I_eV"])
    return s


def _dptr(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def map_hu(hu, curve, ranges):
    hu = np.ascontiguousarray(hu, dtype=np.int16)
    ch = np.ascontiguousarray(curve["hu"], dtype=np.float64)
    cr = np.ascontiguousarray(curve["rho"], dtype=np.float64)
    up = np.ascontiguousarray(ranges["hu_upper"], dtype=np.float64)
    mo = np.ascontiguousarray(ranges["mat"], dtype=np.int32)
    om = np.empty(hu.size, dtype=np.uint8)
    orho = np.empty(hu.size, dtype=np.float64)
    rc = lib().orc_map_hu(hu.ctypes.data, hu.size, ch.size, ch.ctypes.data, cr.ctypes.data,
                          mo.size, up.ctypes.data, mo.ctypes.data, om.ctypes.data, orho.ctypes.data)
    if rc != 0:
        raise ValueError("orc_map_hu failed")
    return om, orho


class Prepared:
    """A workload marshalled into an oracle Config (keeps the arrays alive)."""

    def __init__(self, cfg: dict, seed: int, phsp=None):
        c = Config()
        ph = cfg["physics"]
        c.coupled, c.proc_mask, c.pcut, c.ecut = ph["coupled"], ph["proc_mask"], ph["pcut"], ph["ecut"]
        mats = cfg["materials"]
        c.n_mat = len(mats)
        for i, m in enumerate(mats):
            c.mat[i] = material(m)
        P = cfg["phantom"]
        c.nx, c.ny, c.nz = P["shape"]
        for a in range(3):
            c.spacing[a], c.origin[a] = P["spacing"][a], P["origin"][a]
        if P["kind"] == "hu":
            self.vm, self.vr = map_hu(P["hu"], P["curve"], P["ranges"])
        else:
            self.vm = np.ascontiguousarray(P["mat"], dtype=np.uint8)
            self.vr = np.ascontiguousarray(P["rho"], dtype=np.float64)
        c.vox_mat = self.vm.ctypes.data_as(ct.POINTER(ct.c_uint8))
        c.vox_rho = _dptr(self.vr)
        E = cfg["epid"]
        c.n_layers = len(E["layers"])
        for i, L in enumerate(E["layers"]):
            c.layer_mat[i], c.layer_t[i], c.layer_rho[i] = L["mat"], L["t"], L["rho"]
        c.scoring_layer, c.front_z = E["scoring"], E["front_z"]
        c.npx_u, c.npx_v, c.pitch_u, c.pitch_v = E["npx_u"], E["npx_v"], E["pitch_u"], E["pitch_v"]
        S = cfg["source"]
        c.beam_kind = S["beam"]["kind"]
        for a in range(3):
            c.src[a] = S["beam"]["src"][a]
        c.iso_z = S["beam"]["iso_z"]
        self.edges = np.ascontiguousarray(S["edges"], dtype=np.float64)
        self.weights = np.ascontiguousarray(S["weights"], dtype=np.float64)
        c.nbins = self.weights.size
        c.edges, c.weights = _dptr(self.edges), _dptr(self.weights)
        ap = S["aperture"]
        self.a = np.ascontiguousarray(ap["a"], dtype=np.float64)
        self.b = np.ascontiguousarray(ap["b"], dtype=np.float64)
        self.cnt = np.ascontiguousarray(ap["counts"], dtype=np.uint64)
        c.n_seg, c.n_pairs = self.a.shape
        c.leaf_w, c.y0 = ap["leaf_w"], ap["y0"]
        c.a, c.b = _dptr(self.a), _dptr(self.b)
        c.seg_hist = self.cnt.ctypes.data_as(ct.POINTER(ct.c_uint64))
        if phsp is not None:
            self.phsp = np.ascontiguousarray(phsp, dtype=np.float64).reshape(-1, 8)
            c.n_phsp, c.phsp = self.phsp.shape[0], _dptr(self.phsp)
        c.seed = int(seed)
        c.step_floor = float(ph.get("step_floor", STEP_FLOOR))
        self.c = c
        self.npix = E["npx_u"] * E["npx_v"]
        self.shape = (E["npx_v"], E["npx_u"])


def source(cfg: dict, hs, seed: int = 1001, phsp=None):
    """Source particles (x y z u v w E type) of the given history ids."""
    P = Prepared(cfg, seed, phsp)
    out = np.zeros((len(hs), 8))
    for i, h in enumerate(hs):
        lib().orc_source(ct.byref(P.c), int(h), out[i].ctypes.data)
    return out


def run(cfg: dict, n: int, seed: int = 1001, first: int = 0, threads: int = 1, phsp=None,
        prepared: Prepared | None = None):
    """Run histories [first, first+n) on `threads` threads over disjoint ranges.

    Returns (mean, var_of_mean, sum, sum2, counters-dict); mean is MeV per history
    per pixel, shape (npx_v, npx_u)."""
    P = prepared or Prepared(cfg, seed, phsp)
    L = lib()
    threads = max(1, min(threads, n))
    bounds = [first + (n * i) // threads for i in range(threads + 1)]
    outs = [(np.zeros(P.npix), np.zeros(P.npix), Counters()) for _ in range(threads)]
    errs = [0] * threads

    def work(i):
        s, s2, c = outs[i]
        errs[i] = L.orc_run(ct.byref(P.c), bounds[i], bounds[i + 1] - bounds[i],
                            s.ctypes.data, s2.ctypes.data, ct.byref(c))

    ts = [threading.Thread(target=work, args=(i,)) for i in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    if any(errs):
        raise RuntimeError(f"orc_run failed: {errs}")
    s = sum(o[0] for o in outs)
    s2 = sum(o[1] for o in outs)
    cnt = {}
    for o in outs:
        for k, v in o[2].as_dict().items():
            cnt[k] = max(cnt.get(k, 0.0), v) if k == "max_ledger_resid" else cnt.get(k, 0) + v
    mean = s / n
    var = (s2 / n - mean * mean) / max(1, n - 1)
    return mean.reshape(P.shape), np.maximum(var, 0).reshape(P.shape), s, s2, cnt


def run_traced(cfg: dict, n: int, seed: int = 1001, first: int = 0, cap: int = 1 << 20, phsp=None):
    """Single-threaded run of histories [first, first+n) that also returns every event in
    order as a structured array (EVENT_DTYPE); raises if more than `cap` events happen.

    Returns (mean, var_of_mean, sum, sum2, counters-dict, events)."""
    P = Prepared(cfg, seed, phsp)
    ev = np.zeros(cap, dtype=EVENT_DTYPE)
    s, s2, c = np.zeros(P.npix), np.zeros(P.npix), Counters()
    nev = ct.c_uint64(0)
    rc = lib().orc_run_traced(ct.byref(P.c), first, n, s.ctypes.data, s2.ctypes.data, ct.byref(c),
                              ev.ctypes.data, cap, ct.byref(nev))
    if rc != 0:
        raise RuntimeError(f"orc_run_traced failed: {rc}")
    if nev.value > cap:
        raise RuntimeError(f"{nev.value} events exceed the trace capacity {cap}")
    mean = s / n
    var = (s2 / n - mean * mean) / max(1, n - 1)
    return mean.reshape(P.shape), np.maximum(var, 0).reshape(P.shape), s, s2, c.as_dict(), ev[:nev.value]


def radiological_thickness(cfg: dict) -> np.ndarray:
    """Radiological thickness (cm of unit density) of the phantom along each pixel's ray,
    shape (npx_v, npx_u) (Sec. 2.2, item 1)."""
    P = Prepared(cfg, 0)
    out = np.zeros(P.npix)
    if lib().orc_radiological_thickness(ct.byref(P.c), out.ctypes.data) != 0:
        raise ValueError("orc_radiological_thickness failed")
    return out.reshape(P.shape)


def equivalent_square(cfg: dict) -> float:
    """Equivalent square (cm) of the open aperture's bounding rectangle (Sec. 2.2, Eq. 1)."""
    P = Prepared(cfg, 0)
    return float(lib().orc_equivalent_square(ct.byref(P.c)))


def response_factor(t_nodes, s_nodes, k, t, s) -> np.ndarray:
    """k(t, s) by clamped bilinear interpolation on the table k[s_j][t_i] (Eq. 2, Table 1);
    t and s may be arrays of the same shape."""
    tn = np.ascontiguousarray(t_nodes, dtype=np.float64)
    sn = np.ascontiguousarray(s_nodes, dtype=np.float64)
    kk = np.ascontiguousarray(k, dtype=np.float64).reshape(sn.size, tn.size)
    t = np.asarray(t, dtype=np.float64)
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), t.shape)
    f = lib().orc_response_factor
    out = np.array([f(tn.ctypes.data, tn.size, sn.ctypes.data, sn.size, kk.ctypes.data, float(a), float(b))
                    for a, b in zip(t.ravel(), s.ravel())])
    return out.reshape(t.shape)

