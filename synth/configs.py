"""Workload descriptions: image grids, scanner geometries, TOF, counts, prior settings.

Plain parameter records; no arithmetic of the reconstruction method lives here.
Both the oracle and the GPU library read the same records, so a parameter choice
(ring pitch, radial sampling, phantom layout) is made once.

Names: ``c0_2d`` (2D parallel beam), ``c1_3d`` (3D brain-sized non-TOF),
``c2_tof`` (3D TOF, the headline workload), ``c3_diff`` (small 3D used by the
unrolled/differentiable form), plus small ``mini_*`` geometries used by tests so
the FP64 oracle finishes in seconds while still covering ragged shapes.
"""

import math
from copy import deepcopy

FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))

# Water attenuation used for the multiplicative factors a_j = exp(-mu L_j).
MU_WATER = 0.0096  # 1/mm

_C1_PITCH = 71 * 2.03 / 64  # scanner axial FOV equals the image's axial extent

CONFIGS = {
    # 2D parallel-beam, 64x64 image at 4 mm, 91 radial x 60 views over 180 deg.
    "c0_2d": dict(
        name="c0_2d", kind="parallel2d",
        nx=64, ny=64, nz=1, vx=4.0, vy=4.0, vz=4.0,
        n_views=60, n_rad=91, rad_spacing=4.0, half_length=500.0,
        n_tof=1, tof_bin=0.0, tof_sigma=0.0, tof_nsigma=0.0,
        n_subsets=6, phantom="c0", counts_total=1e5, bg_fraction_of_mean=0.1,
        beta=0.01, gamma=2.0, seed=0, epochs=20,
    ),
    # 3D non-TOF brain-sized: 128x128x71, 504-crystal ring of radius 328 mm,
    # 64 rings, span-1 planes with ring difference <= 20 (2204 planes).
    "c1_3d": dict(
        name="c1_3d", kind="cylinder",
        nx=128, ny=128, nz=71, vx=2.086, vy=2.086, vz=2.03,
        radius=328.0, n_crystals=504, n_views=252, n_rad=344,
        n_rings=64, ring_pitch=_C1_PITCH, max_ring_diff=20,
        n_tof=1, tof_bin=0.0, tof_sigma=0.0, tof_nsigma=0.0,
        n_subsets=25, phantom="head", counts=1e7, bg_fraction_of_prompts=0.2,
        beta_tilde=4.0, gamma=2.0, seed=0, epochs=30,
    ),
    # 3D TOF: as c1_3d plus 13 TOF bins of 40 mm, Gaussian 60 mm FWHM, 3 sigma.
    "c2_tof": dict(
        name="c2_tof", kind="cylinder",
        nx=128, ny=128, nz=71, vx=2.086, vy=2.086, vz=2.03,
        radius=328.0, n_crystals=504, n_views=252, n_rad=344,
        n_rings=64, ring_pitch=_C1_PITCH, max_ring_diff=20,
        n_tof=13, tof_bin=40.0, tof_sigma=60.0 * FWHM_TO_SIGMA, tof_nsigma=3.0,
        n_subsets=25, phantom="head", counts=3e7, bg_fraction_of_prompts=0.2,
        beta_tilde=4.0, gamma=2.0, seed=0, epochs=30,
    ),
    # Small 3D geometry of the unrolled form: 96x96x32, 240-crystal ring,
    # 32 rings, ring difference <= 4 (268 planes), 8 subsets.
    "c3_diff": dict(
        name="c3_diff", kind="cylinder",
        nx=96, ny=96, nz=32, vx=128 * 2.086 / 96, vy=128 * 2.086 / 96, vz=4.5,
        radius=328.0, n_crystals=240, n_views=120, n_rad=180,
        n_rings=32, ring_pitch=4.5, max_ring_diff=4,
        n_tof=1, tof_bin=0.0, tof_sigma=0.0, tof_nsigma=0.0,
        n_subsets=8, phantom="head", counts=5e6, bg_fraction_of_prompts=0.2,
        beta_tilde=4.0, gamma=2.0, seed=0, epochs=10,
    ),
    # Batched workload: 24 independent reconstructions, 4 per (size, TOF) cell
    # with sizes {96x96x32 (c3_diff geometry), 128x128x48 (43 rings, ring
    # difference <= 14, 1037 planes), 128x128x71 (c1_3d geometry)}, TOF as
    # c2_tof; counts log-uniform in [1e6, 1e8], beta log-uniform within
    # [0.1, 10] x the count-scaled rule, 8..25 subsets (synth.data.batch_members).
    "c4_batch": dict(
        name="c4_batch", kind="batch", per_cell=4, counts_range=(1e6, 1e8), beta_factor_range=(0.1, 10.0),
        subsets_range=(8, 25), beta_tilde=4.0, gamma=2.0, seed=0, epochs=3,
    ),
    # Test geometries: ragged sizes, several segments, TOF on/off.
    "mini_tof": dict(
        name="mini_tof", kind="cylinder",
        nx=21, ny=19, nz=9, vx=4.0, vy=4.2, vz=3.7,
        radius=90.0, n_crystals=42, n_views=21, n_rad=17,
        n_rings=8, ring_pitch=4.1, max_ring_diff=3,
        n_tof=5, tof_bin=22.0, tof_sigma=14.0, tof_nsigma=3.0,
        n_subsets=4, phantom="head_small", counts=2e4, bg_fraction_of_prompts=0.2,
        beta_tilde=4.0, gamma=2.0, seed=1, epochs=4,
    ),
    "mini_nontof": dict(
        name="mini_nontof", kind="cylinder",
        nx=21, ny=19, nz=9, vx=4.0, vy=4.2, vz=3.7,
        radius=90.0, n_crystals=42, n_views=21, n_rad=17,
        n_rings=8, ring_pitch=4.1, max_ring_diff=3,
        n_tof=1, tof_bin=0.0, tof_sigma=0.0, tof_nsigma=0.0,
        n_subsets=4, phantom="head_small", counts=2e4, bg_fraction_of_prompts=0.2,
        beta_tilde=4.0, gamma=2.0, seed=2, epochs=4,
    ),
    "mini_2d": dict(
        name="mini_2d", kind="parallel2d",
        nx=23, ny=17, nz=1, vx=4.0, vy=4.0, vz=4.0,
        n_views=12, n_rad=31, rad_spacing=3.5, half_length=300.0,
        n_tof=1, tof_bin=0.0, tof_sigma=0.0, tof_nsigma=0.0,
        n_subsets=3, phantom="c0_small", counts_total=5e4, bg_fraction_of_mean=0.1,
        beta=0.01, gamma=2.0, seed=3, epochs=4,
    ),
}

# The paper's own simulation geometry (Section 3.1): 600 mm diameter, 17 rings
# over 80 mm, 36 modules x 12 detectors, span-1 sinograms of 289 planes x 216
# views x 353 radial bins x 25 TOF bins (390 ps), 161x161x33 image at 2.5 mm,
# 4 mm FWHM image-space resolution model, 27 subsets.  The TOF bin width is
# not given; 24 mm makes the 25 bins span the scanner diameter.
CONFIGS["c5_sim"] = dict(
    name="c5_sim", kind="cylinder",
    nx=161, ny=161, nz=33, vx=2.5, vy=2.5, vz=2.5,
    radius=300.0, n_crystals=432, n_views=216, n_rad=353,
    n_rings=17, ring_pitch=80.0 / 17, max_ring_diff=16,
    n_tof=25, tof_bin=24.0, tof_sigma=0.390 * 299.792458 / 2 * FWHM_TO_SIGMA, tof_nsigma=3.0,
    psf_fwhm=4.0,
    n_subsets=27, phantom="sim_ellipses", counts=1e7, bg_fraction_of_prompts=0.2,
    beta_tilde=4.0, gamma=2.0, seed=0, epochs=30,
)
# Test geometry with more TOF bins than a lane holds at once (two bin blocks).
CONFIGS["mini_tof_many"] = dict(CONFIGS["mini_tof"], name="mini_tof_many", n_tof=20, tof_bin=7.0, tof_sigma=6.0)

# Test geometry whose TOF segments hold 37-40 planes (40 rings of 1 mm,
# ring difference <= 3): more than 32 planes per segment, so one plane per lane
# of a segment wave, as on the 3D TOF workload, at a size the oracle finishes
# in seconds.
CONFIGS["mini_tof_seg40"] = dict(CONFIGS["mini_tof"], name="mini_tof_seg40", nz=11, n_rings=40, ring_pitch=1.0,
                                 seed=4)

# Test geometries with the image-space resolution model (Section 3.1): a
# Gaussian of 6 mm FWHM on ~4 mm voxels (kernel radius 3 voxels in x and y).
CONFIGS["mini_tof_psf"] = dict(CONFIGS["mini_tof"], name="mini_tof_psf", psf_fwhm=6.0)
CONFIGS["mini_2d_psf"] = dict(CONFIGS["mini_2d"], name="mini_2d_psf", psf_fwhm=6.0)


MID_PITCH = 48 * 2.03 / 43  # 43 rings spanning the 48-slice image


def batch_size_config(size, tof):
    """Geometry of one batch member: size 0 = c3_diff, 1 = 128x128x48 with 43
    rings (ring difference <= 14), 2 = c1_3d; tof adds c2_tof's 13 bins."""
    base = get("c3_diff") if size == 0 else get("c1_3d")
    if size == 1:
        base.update(nz=48, n_rings=43, ring_pitch=MID_PITCH, max_ring_diff=14)
    if tof:
        t = CONFIGS["c2_tof"]
        base.update(n_tof=t["n_tof"], tof_bin=t["tof_bin"], tof_sigma=t["tof_sigma"], tof_nsigma=t["tof_nsigma"])
    base["name"] = f"c4_{('s', 'm', 'l')[size]}{'_tof' if tof else ''}"
    return base


def get(name, **overrides):
    """Return a copy of the named workload with ``overrides`` applied."""
    cfg = deepcopy(CONFIGS[name])
    cfg.update(overrides)
    return cfg


def n_planes(cfg):
    if cfg["kind"] == "parallel2d":
        return 1
    nr, md = cfg["n_rings"], cfg["max_ring_diff"]
    return nr + 2 * sum(nr - d for d in range(1, md + 1))


def n_bins(cfg):
    return cfg["n_views"] * cfg["n_rad"] * n_planes(cfg) * cfg["n_tof"]


def n_vox(cfg):
    return cfg["nx"] * cfg["ny"] * cfg["nz"]


def subset_views(cfg, i):
    """Views of subset i: every n-th view starting at i (interleaved)."""
    return list(range(i, cfg["n_views"], cfg["n_subsets"]))


def beta_value(cfg):
    """Prior strength: the explicit ``beta`` if given, else the count-scaled rule
    beta = beta_tilde * 2e-4 * counts / 3e7 (Section 3.1, simulation setup)."""
    if "beta" in cfg:
        return float(cfg["beta"])
    return float(cfg["beta_tilde"] * 2e-4 * cfg["counts"] / 3e7)
