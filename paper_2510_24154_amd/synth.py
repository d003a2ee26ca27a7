"""Seeded synthetic inputs for the EPID transit Monte Carlo workloads.

This module only *describes* workloads: material compositions, geometry,
HU phantoms, source spectra, MLC apertures and history counts.  It contains
none of the transport arithmetic, so both the HIP engine and the CPU oracle
can be fed from it without sharing any of the method's code.

The paper's clinical inputs (VitalBeam phase space, patient CT, RTPLAN, the
AS1200 layer specification, measured images; Sec. 2.1.1-2.1.3, 2.3) are not
public.  Every workload here is a seeded synthetic stand-in with the shapes
of the paper's setting: a point source 100 cm above the isocentre, the EPID
scoring plane at 150 cm (Sec. 2.3.1-2.3.2), a copper build-up plate, a
reflector, a Gd2O2S phosphor and a protective glass layer (Sec. 2.1.3).
"""
from __future__ import annotations

import copy
import numpy as np

# --------------------------------------------------------------------------
# materials: elemental mass fractions from the chemical formulas (or a fixed
# soft-bone recipe), mean excitation energies as model inputs
# --------------------------------------------------------------------------
_H, _C, _N, _O = (1, 1.008), (6, 12.011), (7, 14.007), (8, 15.999)
_MG, _SI, _P, _S = (12, 24.305), (14, 28.085), (15, 30.974), (16, 32.06)
_AR, _CA, _CU, _GD = (18, 39.948), (20, 40.078), (29, 63.546), (64, 157.25)


def _formula(parts):
    """parts: list of ((Z, A), count) -> (Z list, A list, mass fractions)."""
    mass = sum(el[1] * n for el, n in parts)
    return ([el[0] for el, _ in parts], [el[1] for el, _ in parts],
            [el[1] * n / mass for el, n in parts])


def _mat(name, Z, A, w, I_eV, rho):
    w = np.asarray(w, dtype=np.float64)
    return {"name": name, "Z": list(Z), "A": list(A), "w": list(w / w.sum()),
            "I_eV": float(I_eV), "rho": float(rho)}


WATER = _mat("water", *_formula([(_H, 2), (_O, 1)]), 75.0, 1.0)
LUNG = _mat("lung", *_formula([(_H, 2), (_O, 1)]), 75.0, 0.30)
AIR = _mat("air", [7, 8, 18], [_N[1], _O[1], _AR[1]], [0.7553, 0.2318, 0.0129], 85.7, 0.0012)
BONE = _mat("bone", [1, 6, 7, 8, 12, 15, 16, 20],
            [_H[1], _C[1], _N[1], _O[1], _MG[1], _P[1], _S[1], _CA[1]],
            [0.064, 0.278, 0.027, 0.410, 0.002, 0.070, 0.002, 0.147], 106.4, 1.60)
COPPER = _mat("copper", [29], [_CU[1]], [1.0], 322.0, 8.96)
PET = _mat("pet", *_formula([(_C, 10), (_H, 8), (_O, 4)]), 78.7, 1.38)
GOS = _mat("gd2o2s", *_formula([(_GD, 2), (_O, 2), (_S, 1)]), 400.0, 7.44)
GLASS = _mat("glass", *_formula([(_SI, 1), (_O, 2)]), 139.2, 2.50)

# default HU -> density curve (piecewise linear) and HU -> material ranges
HU_CURVE = {"hu": [-1000.0, 0.0, 3000.0], "rho": [0.0, 1.0, 2.8]}
HU_RANGES = {"hu_upper": [-950.0, -200.0, 300.0], "mat": [0, 1, 2, 3]}  # air, lung, water, bone

PHOTON_CUT = 0.010   # MeV (Sec. 2.1.2)
ELECTRON_CUT = 0.200  # MeV (Sec. 2.1.2)


def _epid(layers, scoring, front_z, npx_u, npx_v, pitch):
    return {"layers": layers, "scoring": scoring, "front_z": float(front_z),
            "npx_u": int(npx_u), "npx_v": int(npx_v), "pitch_u": float(pitch), "pitch_v": float(pitch)}


def _open_field(half_x, half_y, leaf_w=0.5):
    n = int(round(2 * half_y / leaf_w))
    return {"n_pairs": n, "leaf_w": leaf_w, "y0": -half_y,
            "a": np.full((1, n), -half_x), "b": np.full((1, n), half_x),
            "counts": np.array([0], dtype=np.uint64)}


# --------------------------------------------------------------------------
# workload 1: photon-only KERMA, 2 MeV parallel beam, 20 cm water box
# --------------------------------------------------------------------------
def kerma_water(nvox=100, npx=128, spacing=None, pitch=None):
    """2 MeV mono-energetic 10x10 cm parallel beam onto a 20 cm water cube of
    2 mm voxels; a 2 mm Cu + 0.3 mm Gd2O2S + 1 mm glass stack 50 cm behind the
    exit face; 128x128 image of 2 mm pixels in the phosphor; Compton and
    photoelectric only, electrons deposited where they are set in motion."""
    spacing = 20.0 / nvox if spacing is None else spacing
    pitch = 25.6 / npx if pitch is None else pitch
    n = nvox
    return {
        "name": "kerma_water",
        "materials": [copy.deepcopy(m) for m in (WATER, COPPER, GOS, GLASS)],
        "physics": {"coupled": 0, "proc_mask": 0b011, "pcut": PHOTON_CUT, "ecut": ELECTRON_CUT},
        "phantom": {"kind": "direct", "shape": (n, n, n), "spacing": (spacing,) * 3,
                    "origin": (-10.0, -10.0, 0.0),
                    "mat": np.zeros(n * n * n, dtype=np.uint8),
                    "rho": np.ones(n * n * n, dtype=np.float32)},
        "epid": _epid([{"mat": 1, "t": 0.2, "rho": 8.96},
                       {"mat": 2, "t": 0.03, "rho": 7.44},
                       {"mat": 3, "t": 0.1, "rho": 2.5}], 1, 70.0, npx, npx, pitch),
        "source": {"beam": {"kind": 0, "src": (0.0, 0.0, 0.0), "iso_z": 0.0},
                   "edges": np.array([2.0, 2.0]), "weights": np.array([1.0]),
                   "aperture": _open_field(5.0, 5.0)},
    }


# --------------------------------------------------------------------------
# workload 2: coupled transport, 6 MV-like spectrum, heterogeneous phantom
# --------------------------------------------------------------------------
def ellipsoid_list(seed=2):
    """Seeded lung (HU -700) and bone (HU +1000) ellipsoids in a 51.2 x 51.2 x
    25.6 cm phantom centred on the isocentre (z = 100 cm)."""
    rng = np.random.default_rng(seed)
    ell = []
    for _ in range(2):
        ax = rng.uniform(3, 7, 2).tolist() + [rng.uniform(3, 8)]
        c = rng.uniform(-8, 8, 2).tolist() + [100.0 + rng.uniform(-6.4, 6.4)]
        ell.append({"hu": -700, "c": c, "ax": ax})
    for _ in range(4):
        ax = rng.uniform(0.5, 2.0, 3).tolist()
        c = rng.uniform(-8, 8, 2).tolist() + [100.0 + rng.uniform(-6.4, 6.4)]
        ell.append({"hu": 1000, "c": c, "ax": ax})
    return ell


def hu_grid(shape, spacing, origin, ellipsoids, background=0):
    """int16 HU grid, x fastest; a voxel takes the HU of the last ellipsoid containing its centre."""
    nx, ny, nz = shape
    xs = origin[0] + (np.arange(nx) + 0.5) * spacing[0]
    ys = origin[1] + (np.arange(ny) + 0.5) * spacing[1]
    zs = origin[2] + (np.arange(nz) + 0.5) * spacing[2]
    hu = np.full((nz, ny, nx), background, dtype=np.int16)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    for e in ellipsoids:
        (cx, cy, cz), (ax, ay, az) = e["c"], e["ax"]
        inside = ((X - cx) / ax) ** 2 + ((Y - cy) / ay) ** 2 + ((Z - cz) / az) ** 2 <= 1.0
        hu[inside] = e["hu"]
    return hu.reshape(-1)


def thin_target_spectrum(seed=3, e0=6.0, lo=0.1, hi=6.0, width=0.05):
    """Binned thin-target bremsstrahlung shape (1/k)(1 - k/E0) for E0 = 6 MeV
    electrons, integrated over 0.05 MeV bins from 0.1 to 6.0 MeV (118 bins),
    with a seeded per-bin jitter U(0.95, 1.05) and renormalisation."""
    nb = int(round((hi - lo) / width))
    edges = lo + width * np.arange(nb + 1)
    k1, k2 = edges[:-1], edges[1:]
    w = np.log(k2 / k1) - (k2 - k1) / e0
    w *= np.random.default_rng(seed).uniform(0.95, 1.05, nb)
    return edges, w / w.sum()


def coupled_hetero(shape=(256, 256, 128), spacing=0.2, npx=(768, 1024), pitch=0.039,
                   phantom_seed=2, spectrum_seed=3):
    """Coupled photon-electron transport: seeded 6 MV-like spectrum, 10x10 cm
    field at the isocentre from a point source 100 cm above it, heterogeneous
    phantom of 2 mm voxels (water, lung and bone ellipsoids), 4-layer EPID with
    its phosphor mid-plane at 150 cm, 1024x768 image of 0.39 mm pixels."""
    nx, ny, nz = shape
    sp = (float(spacing),) * 3 if np.isscalar(spacing) else tuple(float(s) for s in spacing)
    origin = (-0.5 * nx * sp[0], -0.5 * ny * sp[1], 100.0 - 0.5 * nz * sp[2])
    edges, w = thin_target_spectrum(spectrum_seed)
    layers = [{"mat": 4, "t": 0.2, "rho": 8.96}, {"mat": 5, "t": 0.02, "rho": 1.38},
              {"mat": 6, "t": 0.03, "rho": 7.44}, {"mat": 7, "t": 0.1, "rho": 2.5}]
    front = 150.0 - 0.015 - 0.02 - 0.2
    return {
        "name": "coupled_hetero",
        "materials": [copy.deepcopy(m) for m in (AIR, LUNG, WATER, BONE, COPPER, PET, GOS, GLASS)],
        "physics": {"coupled": 1, "proc_mask": 0b111, "pcut": PHOTON_CUT, "ecut": ELECTRON_CUT},
        "phantom": {"kind": "hu", "shape": (nx, ny, nz), "spacing": sp, "origin": origin,
                    "hu": hu_grid((nx, ny, nz), sp, origin, ellipsoid_list(phantom_seed)),
                    "curve": copy.deepcopy(HU_CURVE), "ranges": copy.deepcopy(HU_RANGES)},
        "epid": _epid(layers, 2, front, npx[0], npx[1], pitch),
        "source": {"beam": {"kind": 1, "src": (0.0, 0.0, 0.0), "iso_z": 100.0},
                   "edges": edges, "weights": w, "aperture": _open_field(5.0, 5.0)},
    }


def coupled_hetero_small():
    """The coupled workload on a coarse grid the oracle finishes quickly: same
    physical extents, 8 mm voxels, 96x128 image of 3.12 mm pixels."""
    return coupled_hetero(shape=(64, 64, 32), spacing=0.8, npx=(96, 128), pitch=0.312)


# --------------------------------------------------------------------------
# workload 3: IMRT-like field of 40 MLC segments with uneven history counts
# --------------------------------------------------------------------------
def mlc_segments(n_seg=40, n_pairs=60, leaf_w=0.5, total=300_000_000,
                 aperture_seed=4, count_seed=5, lo=1_000_000, hi=50_000_000):
    ra = np.random.default_rng(aperture_seed)
    g = ra.uniform(0, 10, (n_seg, n_pairs))
    c = ra.uniform(-5, 5, (n_seg, n_pairs))
    a, b = c - g / 2, c + g / 2
    rc = np.random.default_rng(count_seed)
    w = np.exp(rc.uniform(np.log(lo), np.log(hi), n_seg))
    n = np.clip(np.round(total * w / w.sum()), lo, hi).astype(np.int64)
    for _ in range(100):   # push the residual onto the unclamped segments
        r = total - int(n.sum())
        if r == 0:
            break
        free = np.where((n > lo) & (n < hi))[0] if r < 0 else np.where(n < hi)[0]
        step = np.sign(r) * np.maximum(1, np.abs(r) // max(1, len(free)))
        for i in free:
            if r == 0:
                break
            d = int(np.clip(n[i] + step, lo, hi) - n[i])
            d = d if abs(d) <= abs(r) else r
            n[i] += d
            r -= d
    return {"n_pairs": n_pairs, "leaf_w": leaf_w, "y0": -0.5 * n_pairs * leaf_w,
            "a": a, "b": b, "counts": n.astype(np.uint64)}


def imrt_field(total=300_000_000, **kw):
    cfg = coupled_hetero(**kw)
    cfg["name"] = "imrt40"
    cfg["source"]["aperture"] = mlc_segments(total=total)
    return cfg


def with_histories_scaled(cfg, total):
    """Copy of a multi-segment workload with every segment count scaled to sum to `total`."""
    cfg = copy.deepcopy(cfg)
    ap = cfg["source"]["aperture"]
    c = ap["counts"].astype(np.float64)
    n = np.maximum(1, np.floor(c * total / c.sum())).astype(np.int64)
    n[np.argmax(n)] += total - int(n.sum())
    ap["counts"] = n.astype(np.uint64)
    return cfg


# --------------------------------------------------------------------------
# workload 5: large anthropomorphic-like phantom under a 60-segment field
# --------------------------------------------------------------------------
def anthropomorphic_hu(shape=(512, 512, 200), spacing=0.1, iso_z=100.0):
    """int16 HU grid (x fastest) of a thorax-like phantom for a beam along +z (anterior to
    posterior): an elliptic cylinder of soft tissue (HU 40) along y, semi-axes 17 cm (x) and
    9.5 cm (z), with a 3 mm skin shell (HU 60), a pair of lungs (HU -750; ellipsoids at
    x = -/+8 cm, semi-axes 5.5 x 12 x 5.5 cm, 1 cm anterior of the centre) and a spine
    (HU 800; a cylinder along y of radius 1.8 cm, 6 cm posterior of the centre); air
    (HU -1000) outside."""
    nx, ny, nz = shape
    x = (np.arange(nx) + 0.5) * spacing - 0.5 * nx * spacing
    y = (np.arange(ny) + 0.5) * spacing - 0.5 * ny * spacing
    z = (np.arange(nz) + 0.5) * spacing - 0.5 * nz * spacing   # relative to the isocentre
    X, Y, Z = x[None, None, :], y[None, :, None], z[:, None, None]
    hu = np.full((nz, ny, nx), -1000, dtype=np.int16)
    r_body = (X / 17.0) ** 2 + (Z / 9.5) ** 2                  # constant along y
    body = np.broadcast_to(r_body <= 1.0, hu.shape)
    hu[body] = 60
    inner = np.broadcast_to((X / 16.7) ** 2 + (Z / 9.2) ** 2 <= 1.0, hu.shape)
    hu[inner] = 40
    for cx in (-8.0, 8.0):
        lung = ((X - cx) / 5.5) ** 2 + (Y / 12.0) ** 2 + ((Z + 1.0) / 5.5) ** 2 <= 1.0
        hu[lung] = -750
    spine = np.broadcast_to(X ** 2 + (Z - 6.0) ** 2 <= 1.8 ** 2, hu.shape)
    hu[spine] = 800
    return hu.reshape(-1)


def large_anthropomorphic(total=2_000_000_000, npx=(768, 1024), pitch=0.039):
    """The large heterogeneous case: the anthropomorphic-like phantom on 512x512x200 voxels
    of 1 mm (52 M voxels, 210 MB packed) centred on the isocentre, a 60-segment MLC field of
    uneven history counts summing to `total`, the 6 MV-like spectrum and the 4-layer EPID of
    the coupled workload."""
    shape, sp = (512, 512, 200), (0.1, 0.1, 0.1)
    cfg = coupled_hetero(shape=(8, 8, 8))   # everything but the phantom and the aperture
    origin = (-0.5 * shape[0] * sp[0], -0.5 * shape[1] * sp[1], 100.0 - 0.5 * shape[2] * sp[2])
    cfg["name"] = "large60"
    cfg["phantom"] = {"kind": "hu", "shape": shape, "spacing": sp, "origin": origin,
                      "hu": anthropomorphic_hu(shape, sp[0]),
                      "curve": copy.deepcopy(HU_CURVE), "ranges": copy.deepcopy(HU_RANGES)}
    cfg["epid"] = _epid(cfg["epid"]["layers"], 2, cfg["epid"]["front_z"], npx[0], npx[1], pitch)
    cfg["source"]["aperture"] = mlc_segments(n_seg=60, total=total, aperture_seed=6, count_seed=7,
                                             lo=total // 300, hi=total // 6)
    return cfg


def large_crop(npx=64, pitch=0.312, field=6.0):
    """A crop of the large case for transport parity with the oracle: the central 16 x 16 cm of
    the anthropomorphic-like phantom over its full 20 cm depth, 1 mm voxels (160 x 160 x 200:
    the spine, the inner lungs and the body wall), under an open field of `field` cm at the
    isocentre, with the 4-layer EPID and a coarse image (64 x 64 pixels of 3.12 mm)."""
    shape, sp = (160, 160, 200), (0.1, 0.1, 0.1)
    cfg = coupled_hetero(shape=(8, 8, 8), npx=(npx, npx), pitch=pitch)
    origin = (-0.5 * shape[0] * sp[0], -0.5 * shape[1] * sp[1], 100.0 - 0.5 * shape[2] * sp[2])
    cfg["name"] = "large_crop"
    cfg["phantom"] = {"kind": "hu", "shape": shape, "spacing": sp, "origin": origin,
                      "hu": anthropomorphic_hu(shape, sp[0]),
                      "curve": copy.deepcopy(HU_CURVE), "ranges": copy.deepcopy(HU_RANGES)}
    cfg["source"]["aperture"] = _open_field(0.5 * field, 0.5 * field)
    return cfg


def narrow_field(field=1.0, npx=64, pitch=0.039):
    """The coupled workload's phantom (256 x 256 x 128 voxels of 2 mm), spectrum and 4-layer
    EPID at its native 0.39 mm pixels, under a narrow open field of `field` cm at the
    isocentre onto an npx x npx image: an oracle run of a few million histories then gives
    hundreds of phosphor deposits per in-field pixel."""
    cfg = coupled_hetero(npx=(npx, npx), pitch=pitch)
    cfg["name"] = "narrow_field"
    cfg["source"]["aperture"] = _open_field(0.5 * field, 0.5 * field)
    return cfg


def phase_space_list(seed=8, n=8192, spectrum_seed=3):
    """A seeded stand-in for a list of particles leaving the collimators (rows x y z u v w E
    type; type 0 photon, 1 electron; cm, MeV) for the coupled workload's geometry: 75% photons
    with energies from the 6 MV-like spectrum on rays from the point source through a uniform
    point of the 10 x 10 cm field at the isocentre, starting on the plane z = 60 cm (above the
    phantom box); 10% electrons of 1-6 MeV on such rays; 10% electrons of 0.3-4 MeV that start
    inside the phantom (x, y within 5 cm of the axis, z 90-110 cm) in a forward direction; 5%
    photons starting at z = 60 cm on rays that miss the phantom box."""
    rng = np.random.default_rng(seed)
    edges, w = thin_target_spectrum(spectrum_seed)
    out = np.zeros((n, 8))
    kind = rng.choice(4, size=n, p=[0.75, 0.10, 0.10, 0.05])
    # rays from the source through the field: photons (0) and electrons (1)
    ray = kind <= 1
    px, py = rng.uniform(-5.0, 5.0, n), rng.uniform(-5.0, 5.0, n)
    d = np.stack([px, py, np.full(n, 100.0)], axis=1)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t = 60.0 / d[:, 2]
    out[ray, 0:3] = (d * t[:, None])[ray]
    out[ray, 3:6] = d[ray]
    # rays that miss the box: aimed outside |x| > 30 cm at z = 100
    miss = kind == 3
    mx = rng.choice([-1.0, 1.0], n) * rng.uniform(32.0, 40.0, n)
    dm = np.stack([mx, rng.uniform(-5.0, 5.0, n), np.full(n, 100.0)], axis=1)
    dm /= np.linalg.norm(dm, axis=1, keepdims=True)
    out[miss, 0:3] = (dm * (60.0 / dm[:, 2])[:, None])[miss]
    out[miss, 3:6] = dm[miss]
    # electrons inside the phantom, forward directions (w >= 0.3)
    ins = kind == 2
    out[ins, 0] = rng.uniform(-5.0, 5.0, n)[ins]
    out[ins, 1] = rng.uniform(-5.0, 5.0, n)[ins]
    out[ins, 2] = rng.uniform(90.0, 110.0, n)[ins]
    wz = rng.uniform(0.3, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    st = np.sqrt(1.0 - wz * wz)
    out[ins, 3], out[ins, 4], out[ins, 5] = (st * np.cos(ph))[ins], (st * np.sin(ph))[ins], wz[ins]
    # energies
    b = rng.choice(len(w), size=n, p=w)
    e_ph = edges[b] + rng.uniform(0.0, 1.0, n) * (edges[b + 1] - edges[b])
    out[:, 6] = np.where(kind == 1, rng.uniform(1.0, 6.0, n), np.where(kind == 2, rng.uniform(0.3, 4.0, n), e_ph))
    out[:, 7] = np.where((kind == 1) | (kind == 2), 1.0, 0.0)
    # single precision values, as the engine stores them, with unit directions
    out = out.astype(np.float32).astype(np.float64)
    out[:, 3:6] /= np.linalg.norm(out[:, 3:6], axis=1, keepdims=True)
    return out


def response_table_1():
    """The EPID dose-response correction factors k(t, s) the paper measured (Sec. 3.1, Eq. 2,
    Table 1): thickness nodes t (cm of solid water), field-side nodes s (cm), and k[j][i] at
    (t_i, s_j).  Input data for the correction; no arithmetic on it here."""
    t = np.array([0.0, 5.0, 10.0, 15.0, 20.0])
    s = np.array([5.0, 10.0, 15.0, 20.0])
    k = np.array([[0.999, 0.974, 0.960, 0.949, 0.949],
                  [1.001, 0.975, 0.967, 0.964, 0.953],
                  [0.995, 0.982, 0.983, 0.996, 0.986],
                  [0.991, 0.997, 1.015, 1.034, 1.043]])
    return t, s, k


def lut64_nodes():
    """Nodes of the large case's 64 x 64 correction table: thickness 0-40 cm and field side
    2-25 cm, each axis placed so that it contains Table 1's nodes (t = 0, 5, 10, 15, 20 cm;
    s = 5, 10, 15, 20 cm): t in steps of 0.625 cm up to 38.75 cm, then 40 cm; s in 11 equal
    steps from 2 to 5 cm and 13 equal steps in each 5 cm interval from 5 to 25 cm."""
    t = np.concatenate([np.arange(63) * 0.625, [40.0]])
    s = np.concatenate([2.0 + np.arange(11) * (3.0 / 11.0)] +
                       [lo + np.arange(13) * (5.0 / 13.0) for lo in (5.0, 10.0, 15.0, 20.0)] + [[25.0]])
    return t, s


# --------------------------------------------------------------------------
# learned denoiser: initial parameters and training fields
# --------------------------------------------------------------------------
def unet_params(shapes, seed=21, head_scale=0.01):
    """Seeded initial parameters for a list of convolution shapes [(name, k, c_in, c_out)]:
    W[name] of shape (c_out, k, k, c_in) ~ N(0, 2 / (k*k*c_in)) (He), b[name] = 0; the
    layer named "head" is drawn with standard deviation head_scale instead, so a residual
    network starts close to its input.  float32, returned as {name: (W, b)}."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, k, ci, co in shapes:
        sd = head_scale if name == "head" else np.sqrt(2.0 / (k * k * ci))
        W = (rng.standard_normal((co, k, k, ci)) * sd).astype(np.float32)
        out[name] = (W, np.zeros(co, np.float32))
    return out


def random_aperture(rng, n_pairs=60, leaf_w=0.5, max_gap=10.0, n_hist=1):
    """One seeded MLC segment: per leaf pair a gap U(0, max_gap) cm around a centre
    U(-5, 5) cm, pairs outside a random band of rows closed."""
    g = rng.uniform(0, max_gap, n_pairs)
    c = rng.uniform(-5, 5, n_pairs)
    lo, hi = sorted(rng.integers(0, n_pairs, 2))
    hi = max(hi, lo + 4)
    g[:lo] = 0.0
    g[hi:] = 0.0
    a, b = c - g / 2, c + g / 2
    return {"n_pairs": n_pairs, "leaf_w": leaf_w, "y0": -0.5 * n_pairs * leaf_w,
            "a": a[None, :], "b": b[None, :], "counts": np.array([n_hist], np.uint64)}


def thorax_hu(rng, shape=(128, 128, 50), spacing=0.4):
    """int16 HU grid (x fastest) of a seeded thorax-like phantom for a beam along +z: the
    large case's body (an elliptic cylinder of soft tissue with a skin shell, two lungs, a
    spine; air outside) with every size and position drawn around its values: body
    semi-axes 17 x 9.5 cm x U(0.8, 1.1), lungs at x = -/+8 cm + U(-2, 2), semi-axes
    (5.5, 12, 5.5) cm x U(0.7, 1.2), spine radius 1.8 cm x U(0.8, 1.2) at z offset
    6 cm + U(-1, 1)."""
    nx, ny, nz = shape
    x = (np.arange(nx) + 0.5) * spacing - 0.5 * nx * spacing
    y = (np.arange(ny) + 0.5) * spacing - 0.5 * ny * spacing
    z = (np.arange(nz) + 0.5) * spacing - 0.5 * nz * spacing
    X, Y, Z = x[None, None, :], y[None, :, None], z[:, None, None]
    bx, bz = 17.0 * rng.uniform(0.8, 1.1), 9.5 * rng.uniform(0.8, 1.1)
    hu = np.full((nz, ny, nx), -1000, dtype=np.int16)
    hu[np.broadcast_to((X / bx) ** 2 + (Z / bz) ** 2 <= 1.0, hu.shape)] = 60
    hu[np.broadcast_to((X / (bx - 0.3)) ** 2 + (Z / (bz - 0.3)) ** 2 <= 1.0, hu.shape)] = 40
    for side in (-1.0, 1.0):
        cx = side * 8.0 + rng.uniform(-2.0, 2.0)
        ax = np.array([5.5, 12.0, 5.5]) * rng.uniform(0.7, 1.2, 3)
        cz = -1.0 + rng.uniform(-1.0, 1.0)
        hu[((X - cx) / ax[0]) ** 2 + (Y / ax[1]) ** 2 + ((Z - cz) / ax[2]) ** 2 <= 1.0] = -750
    r = 1.8 * rng.uniform(0.8, 1.2)
    hu[np.broadcast_to(X ** 2 + (Z - 6.0 - rng.uniform(-1.0, 1.0)) ** 2 <= r * r, hu.shape)] = 800
    return hu.reshape(-1)


def denoise_field(seed, shape=(128, 128, 64), spacing=0.4, npx=(768, 1024), pitch=0.039, mixed=False):
    """A training or evaluation field for the denoiser: the coupled workload's source and
    EPID with a seeded ellipsoid phantom (4 mm voxels by default) and one seeded MLC
    segment.  With mixed=True every odd seed instead gives a seeded thorax-like phantom
    (128 x 128 x 50 voxels of 4 mm, the large case's extents) under a field of 5-20 seeded
    segments with uneven counts (relative counts; deliver it with with_histories_scaled).
    Returns a workload configuration."""
    rng = np.random.default_rng(10_000 + seed)
    if mixed and seed % 2 == 1:
        cfg = coupled_hetero(shape=(8, 8, 8), npx=npx, pitch=pitch)
        tshape, sp = (128, 128, 50), (0.4, 0.4, 0.4)
        origin = (-0.5 * tshape[0] * sp[0], -0.5 * tshape[1] * sp[1], 100.0 - 0.5 * tshape[2] * sp[2])
        cfg["phantom"] = {"kind": "hu", "shape": tshape, "spacing": sp, "origin": origin,
                          "hu": thorax_hu(rng, tshape, sp[0]),
                          "curve": copy.deepcopy(HU_CURVE), "ranges": copy.deepcopy(HU_RANGES)}
        n_seg = int(rng.integers(5, 21))
        cfg["source"]["aperture"] = mlc_segments(n_seg=n_seg, total=1_000_000 * n_seg, aperture_seed=30_000 + seed,
                                                 count_seed=40_000 + seed, lo=200_000, hi=5_000_000)
        cfg["name"] = f"denoise_field_{seed}_thorax"
        return cfg
    cfg = coupled_hetero(shape=shape, spacing=spacing, npx=npx, pitch=pitch, phantom_seed=20_000 + seed)
    cfg["name"] = f"denoise_field_{seed}"
    cfg["source"]["aperture"] = random_aperture(rng)
    return cfg
