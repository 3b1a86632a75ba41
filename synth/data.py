"""Seeded synthetic datasets shaped like the paper's simulations.

Recipe (every step is data generation, not reconstruction arithmetic):

* phantom: ellipsoids with additive increments (2D: a water disc with two hot
  ellipses and a cold disc; 3D: a head ellipsoid with a grey shell, white
  interior and five hot spheres);
* true projections: exact line integrals of the continuous phantom (TOF: exact
  integrals of the truncated, bin-integrated Gaussian TOF kernel);
* multiplicative factors a = exp(-mu L) from the chord L through the outer shape;
* activity scaled so that sum(a * p) equals the configured true counts (2D: so
  that total prompts equal the configured total, with r = 10% of mean(a p));
* background r: radially Gaussian-blurred (sigma 40 mm) copy of a * p plus a 1%
  floor, scaled so that sum(r) = 0.25 sum(a p) (r is 20% of prompts); in TOF
  it is spread uniformly over the TOF bins;
* counts y ~ Poisson(a p + r) per (TOF) bin, from a counter-based generator so a
  bin's value depends only on (seed, bin index).
"""

import ctypes
import math
import os
import subprocess

import numpy as np

from . import configs, scanner

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build(force=False):
    """Compile the generator helper with gcc (host code only)."""
    so = os.path.join(_HERE, "_gen.so")
    src = os.path.join(_HERE, "_gen.c")
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", so, src, "-lm"])
    return so


def _lib():
    global _LIB
    if _LIB is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.gen_project.argtypes = [ctypes.c_long, P, P, ctypes.c_long, P, P, ctypes.c_int, P,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        lib.gen_chord.argtypes = [ctypes.c_long, P, P, ctypes.c_long, P, P, P, P]
        lib.gen_voxelize.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [ctypes.c_int] * 3 + [P, P]
        lib.gen_poisson.argtypes = [ctypes.c_long, ctypes.c_long, P, ctypes.c_uint64, ctypes.c_int, P]
        lib.gen_poisson.restype = ctypes.c_uint32
        _LIB = lib
    return _LIB


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def shapes(cfg):
    """Phantom as rows (cx, cy, cz, ax, ay, az, rot_z, increment, 0)."""
    big = 1e6  # 2D shapes extend without limit along z
    d = math.radians
    ph = cfg["phantom"]
    if ph == "c0":
        rows = [(0, 0, 0, 100, 100, big, 0, 1.0),
                (-40, 30, 0, 20, 12, big, d(30), 3.0),
                (45, -20, 0, 15, 10, big, d(-45), 3.0),
                (0, -55, 0, 15, 15, big, 0, -1.0)]
    elif ph == "c0_small":
        rows = [(0, 0, 0, 30, 30, big, 0, 1.0),
                (-10, 8, 0, 8, 5, big, d(30), 3.0),
                (8, -10, 0, 5, 5, big, 0, -1.0)]
    elif ph == "head":
        rows = [(0, 0, 0, 90, 75, 70, 0, 4.0), (0, 0, 0, 80, 65, 60, 0, -3.0)]
        for i, diam in enumerate((5.0, 7.5, 10.0, 12.5, 15.0)):
            ang = d(72 * i)
            rows.append((35 * math.cos(ang), 35 * math.sin(ang), 0, diam / 2, diam / 2, diam / 2, 0, 2.0))
    elif ph == "sim_ellipses":
        # elliptical body inside the 80 mm axial field of the simulated
        # scanner, with hot and cold inserts
        rows = [(0, 0, 0, 130, 90, 36, 0, 1.0),
                (40, 20, 0, 25, 15, 15, d(30), 3.0),
                (-45, -10, 0, 20, 20, 15, 0, -1.0),
                (0, 50, 0, 8, 8, 8, 0, 2.0)]
    elif ph == "head_small":
        rows = [(0, 0, 0, 36, 30, 14, 0, 4.0), (0, 0, 0, 30, 24, 10, 0, -3.0),
                (12, 0, 0, 5, 5, 5, 0, 2.0), (-10, 6, 1, 3, 3, 3, 0, 2.0)]
    else:
        raise ValueError(ph)
    return np.array([r + (0.0,) for r in rows], np.float64)


def voxel_phantom(cfg):
    """Unscaled phantom on the image grid, [nz][ny][nx] FP64."""
    sh = shapes(cfg)
    out = np.zeros((cfg["nz"], cfg["ny"], cfg["nx"]))
    two_d = cfg["kind"] == "parallel2d"
    _lib().gen_voxelize(cfg["nx"], cfg["ny"], cfg["nz"], cfg["vx"], cfg["vy"], cfg["vz"],
                        8 if two_d else 4, 1 if two_d else 4, len(sh), _p(sh), _p(out))
    return out


def _line_tables(cfg, views):
    p1, p2 = scanner.transaxial_endpoints(cfg, views)
    z1, z2 = scanner.plane_z(cfg)
    return (np.ascontiguousarray(p1.reshape(-1, 2)), np.ascontiguousarray(p2.reshape(-1, 2)),
            np.ascontiguousarray(z1), np.ascontiguousarray(z2))


def project_phantom(cfg, views, tof):
    """Exact phantom line integrals for the given views: [V][R][P](x T) float32."""
    p1, p2, z1, z2 = _line_tables(cfg, views)
    sh = shapes(cfg)
    nt = cfg["n_tof"] if tof else 1
    out = np.empty((len(views), cfg["n_rad"], len(z1), nt), np.float32)
    _lib().gen_project(p1.shape[0], _p(p1), _p(p2), len(z1), _p(z1), _p(z2), len(sh), _p(sh),
                       nt, float(cfg["tof_bin"]), float(cfg["tof_sigma"]), float(cfg["tof_nsigma"]), _p(out))
    return out if tof else out[..., 0]


def attenuation_factors(cfg, views=None):
    """a = exp(-mu * chord through the outer shape), [V][R][P] float32."""
    if views is None:
        views = np.arange(cfg["n_views"])
    p1, p2, z1, z2 = _line_tables(cfg, views)
    outer = np.ascontiguousarray(shapes(cfg)[0])
    L = np.empty((len(views), cfg["n_rad"], len(z1)))
    _lib().gen_chord(p1.shape[0], _p(p1), _p(p2), len(z1), _p(z1), _p(z2), _p(outer), _p(L))
    return np.exp(-configs.MU_WATER * L).astype(np.float32)


def seeds(cfg):
    """Independent child seeds: (poisson_key, order_seedseq, batch_seedseq)."""
    ss = np.random.SeedSequence(cfg["seed"])
    kids = ss.spawn(3)
    key = int(kids[0].generate_state(1, np.uint64)[0])
    return key, kids[1], kids[2]


def subset_orders(cfg, n_epochs):
    """One permutation of the subsets per epoch (uniform without replacement)."""
    rng = np.random.Generator(np.random.PCG64(seeds(cfg)[1]))
    return np.stack([rng.permutation(cfg["n_subsets"]) for _ in range(n_epochs)]).astype(np.int32)


def poisson(mean, key, dtype_code, offset=0, out=None):
    """Poisson draws of ``mean``; element j uses counter (key, offset + j)."""
    mean = np.ascontiguousarray(mean, np.float32)
    if out is None:
        out = np.empty(mean.shape, {0: np.uint8, 1: np.uint16, 2: np.float32}[dtype_code])
    mx = _lib().gen_poisson(mean.size, offset, _p(mean), key, dtype_code, _p(out))
    return out, mx


def make_dataset(cfg, chunk_views=16):
    """Build the full dataset for a workload.

    Returns dict with x_true [nz][ny][nx] float32 (scaled), mult [V][R][P]
    float32, r_lor [V][R][P] float32 (background per LOR summed over TOF),
    r [V][R][P][T] float32 (per TOF bin), y [V][R][P][T] (uint8/uint16/float32),
    y_dtype_code (0/1/2), scale.
    """
    V = cfg["n_views"]
    views = np.arange(V)
    nt = cfg["n_tof"]
    p = project_phantom(cfg, views, tof=False)
    a = attenuation_factors(cfg, views)
    ap = a.astype(np.float64) * p
    if cfg["kind"] == "parallel2d":
        scale = cfg["counts_total"] / (ap.sum() * (1.0 + cfg["bg_fraction_of_mean"]))
        ap *= scale
        r_lor = np.full(ap.shape, cfg["bg_fraction_of_mean"] * ap.mean())
    else:
        from scipy.ndimage import gaussian_filter1d
        scale = cfg["counts"] / ap.sum()
        ap *= scale
        sig_bins = 40.0 / (cfg["radius"] * math.pi / cfg["n_crystals"])
        sm = gaussian_filter1d(ap, sig_bins, axis=1, mode="constant")
        sm += 0.01 * sm.max()
        frac = cfg["bg_fraction_of_prompts"]
        r_lor = sm * (frac / (1 - frac)) * ap.sum() / sm.sum()
    r_lor = r_lor.astype(np.float32)
    x_true = (voxel_phantom(cfg) * scale).astype(np.float32)
    key = seeds(cfg)[0]
    if nt == 1:
        mean = (ap.astype(np.float32) + r_lor)[..., None]
        y, mx = poisson(mean, key, 0)
        code = 0
        if mx > 255:
            code = 1 if mx <= 65535 else 2
            y, mx = poisson(mean, key, code)
        r = r_lor[..., None].copy()
    else:
        r = np.repeat(r_lor[..., None] / np.float32(nt), nt, axis=-1)
        per_view = r[0].size
        code = 0
        while True:
            y = np.empty(r.shape, {0: np.uint8, 1: np.uint16, 2: np.float32}[code])
            mx = 0
            for v0 in range(0, V, chunk_views):
                vs = views[v0:v0 + chunk_views]
                pt = project_phantom(cfg, vs, tof=True)
                mean = (pt * np.float32(scale)) * a[vs, ..., None] + r[vs]
                _, m = poisson(mean, key, code, offset=v0 * per_view, out=y[v0:v0 + len(vs)])
                mx = max(mx, m)
            if code == 2 or (code == 0 and mx <= 255) or (code == 1 and mx <= 65535):
                break
            code = 1 if mx <= 65535 else 2
    return dict(x_true=x_true, mult=a, r_lor=r_lor, r=r, y=y, y_dtype_code=code, scale=scale)


def nrmse_region(cfg, scale):
    """Evaluation region and reference level of the convergence NRMSE: the
    voxels whose centres lie inside the phantom's first (outermost) shape, and
    that shape's own value in the scaled phantom (background disc in 2D, grey
    shell in 3D).  Returns (mask [nz][ny][nx] bool, level)."""
    cx, cy, cz, ax, ay, az, rot, inc, _ = shapes(cfg)[0]
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    x = (np.arange(nx) - (nx - 1) / 2.0) * cfg["vx"]
    y = (np.arange(ny) - (ny - 1) / 2.0) * cfg["vy"]
    z = (np.arange(nz) - (nz - 1) / 2.0) * cfg["vz"]
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    c, s = math.cos(rot), math.sin(rot)
    u = (xx - cx) * c + (yy - cy) * s
    v = -(xx - cx) * s + (yy - cy) * c
    w = zz - cz
    mask = (u / ax) ** 2 + (v / ay) ** 2 + (w / az) ** 2 <= 1.0
    return mask, float(inc * scale)


def batch_members(cfg):
    """Member workloads of a batched configuration (kind "batch"): per_cell
    members for each (size, TOF) cell, with counts log-uniform in
    counts_range, beta = (count-scaled rule) x a factor log-uniform in
    beta_factor_range, and a uniform number of subsets in subsets_range, drawn
    from the configuration's batch seed stream; each member has its own data
    seed."""
    rng = np.random.Generator(np.random.PCG64(seeds(cfg)[2]))
    lo, hi = cfg["counts_range"]
    blo, bhi = cfg["beta_factor_range"]
    slo, shi = cfg["subsets_range"]
    out = []
    for size in range(3):
        for tof in (False, True):
            for j in range(cfg["per_cell"]):
                m = configs.batch_size_config(size, tof)
                counts = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
                factor = float(np.exp(rng.uniform(np.log(blo), np.log(bhi))))
                m.update(counts=counts, n_subsets=int(rng.integers(slo, shi + 1)), seed=1000 + len(out),
                         beta_tilde=cfg["beta_tilde"], gamma=cfg["gamma"])
                m["beta"] = configs.beta_value(m) * factor
                m["name"] = f"{m['name']}_{j}"
                out.append(m)
    return out
