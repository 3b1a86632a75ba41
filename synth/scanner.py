"""Scanner description: where each line of response (LOR) starts and ends.

The sinogram bin (view v, radial k, plane p, TOF bin b) is stored at flat index
``((v * n_rad + k) * n_planes + p) * n_tof + b`` (view-major, TOF innermost).

Cylinder (ring) scanners: view v has angle phi_v = pi v / n_views, normal
n = (cos phi, sin phi) and direction t = (-sin phi, cos phi).  The radial
coordinate is not arc-corrected: s_k = R sin(pi (k - (n_rad - 1)/2) / n_crystals),
so neighbouring bins are one crystal-pitch angle apart on the ring.  The
transaxial endpoints are s n -/+ sqrt(R^2 - s^2) t.  A plane is a ring pair
(r1, r2); r1 sits at the first endpoint and r2 at the second, ring r at
z_r = (r - (n_rings - 1)/2) * pitch.  Planes are ordered by segment
d = r2 - r1 = 0, -1, +1, -2, +2, ... and by r1 ascending within a segment.

Parallel-beam 2D: s_k = (k - (n_rad - 1)/2) * spacing and the endpoints are
s n -/+ H t with H larger than the image, so each LOR crosses the whole grid.

The paper delegates the system model to an external projector; these layouts
are this project's reading of the workloads, shared by every consumer.
"""

import numpy as np


def plane_table(cfg):
    """Return (r1, r2, segment_index) int arrays in plane order."""
    if cfg["kind"] == "parallel2d":
        return np.zeros(1, np.int64), np.zeros(1, np.int64), np.zeros(1, np.int64)
    nr, md = cfg["n_rings"], cfg["max_ring_diff"]
    r1s, r2s, segs = [], [], []
    seg_list = [0]
    for d in range(1, md + 1):
        seg_list += [-d, d]
    for si, d in enumerate(seg_list):
        for r1 in range(max(0, -d), min(nr, nr - d)):
            r1s.append(r1)
            r2s.append(r1 + d)
            segs.append(si)
    return np.array(r1s), np.array(r2s), np.array(segs)


def segment_list(cfg):
    if cfg["kind"] == "parallel2d":
        return [0]
    out = [0]
    for d in range(1, cfg["max_ring_diff"] + 1):
        out += [-d, d]
    return out


def ring_z(cfg, r):
    return (np.asarray(r, np.float64) - (cfg["n_rings"] - 1) / 2.0) * cfg["ring_pitch"]


def plane_z(cfg):
    """Axial coordinates (z1, z2) in mm of the two endpoints for every plane."""
    if cfg["kind"] == "parallel2d":
        return np.zeros(1), np.zeros(1)
    r1, r2, _ = plane_table(cfg)
    return ring_z(cfg, r1), ring_z(cfg, r2)


def radial_coords(cfg):
    k = np.arange(cfg["n_rad"], dtype=np.float64)
    if cfg["kind"] == "parallel2d":
        return (k - (cfg["n_rad"] - 1) / 2.0) * cfg["rad_spacing"]
    return cfg["radius"] * np.sin(np.pi * (k - (cfg["n_rad"] - 1) / 2.0) / cfg["n_crystals"])


def transaxial_endpoints(cfg, views=None):
    """Transaxial endpoints for lines (view, radial).

    Returns p1, p2 of shape [len(views), n_rad, 2] (mm, FP64).
    """
    if views is None:
        views = np.arange(cfg["n_views"])
    views = np.asarray(views, np.float64)
    phi = np.pi * views / cfg["n_views"]
    n = np.stack([np.cos(phi), np.sin(phi)], -1)[:, None, :]
    t = np.stack([-np.sin(phi), np.cos(phi)], -1)[:, None, :]
    s = radial_coords(cfg)[None, :, None]
    if cfg["kind"] == "parallel2d":
        h = np.full_like(s, cfg["half_length"])
    else:
        h = np.sqrt(cfg["radius"] ** 2 - s ** 2)
    return s * n - h * t, s * n + h * t


def lor_endpoints(cfg, views, radials, planes):
    """Endpoints of arbitrary LORs given as equal-length index arrays.

    Returns p1, p2 of shape [N, 3] (mm, FP64).
    """
    views = np.asarray(views)
    radials = np.asarray(radials)
    planes = np.asarray(planes)
    p1t, p2t = transaxial_endpoints(cfg, np.arange(cfg["n_views"]))
    z1, z2 = plane_z(cfg)
    p1 = np.empty((views.size, 3))
    p2 = np.empty((views.size, 3))
    p1[:, :2] = p1t[views, radials]
    p2[:, :2] = p2t[views, radials]
    p1[:, 2] = z1[planes]
    p2[:, 2] = z2[planes]
    return p1, p2


def subset_lor_indices(cfg, views):
    """(view, radial, plane) index arrays for all LORs of the given views, in
    sinogram order (view, radial, plane)."""
    npl = len(plane_table(cfg)[0])
    v, k, p = np.meshgrid(np.asarray(views), np.arange(cfg["n_rad"]), np.arange(npl), indexing="ij")
    return v.ravel(), k.ravel(), p.ravel()


def tof_centres(cfg):
    nt = cfg["n_tof"]
    return (np.arange(nt) - (nt - 1) / 2.0) * cfg["tof_bin"]


def voxel_centres(cfg):
    """Voxel-centre coordinates per axis (grid centred on the origin)."""
    out = []
    for n, v in ((cfg["nx"], cfg["vx"]), (cfg["ny"], cfg["vy"]), (cfg["nz"], cfg["vz"])):
        out.append((np.arange(n) - (n - 1) / 2.0) * v)
    return out
