"""Pins for the FP64 Joseph oracle against facts fixed by geometry and
mathematics (hand-computed responses, exact chords, the adjoint identity, the
TOF partition of unity, mass conservation), none of which re-evaluates the
oracle's own formulas."""

import math

import numpy as np
import pytest

from oracle import projector
from synth import configs, data, scanner


def _grid(nx, ny, nz, vx, vy, vz, **kw):
    cfg = dict(nx=nx, ny=ny, nz=nz, vx=vx, vy=vy, vz=vz, n_tof=1, tof_bin=0.0, tof_sigma=1.0, tof_nsigma=0.0)
    cfg.update(kw)
    return cfg


def _centre(cfg, ix, iy, iz):
    return ((ix - (cfg["nx"] - 1) / 2) * cfg["vx"], (iy - (cfg["ny"] - 1) / 2) * cfg["vy"],
            (iz - (cfg["nz"] - 1) / 2) * cfg["vz"])


def test_delta_response_hand_value(oracle_built):
    # Line parallel to x, offset +0.25 voxel in y and -0.5 voxel in z from the
    # centre of voxel (2, 3, 1): bilinear weight (1 - 0.25) * (1 - 0.5) = 0.375,
    # step length vx.  Response = 0.375 * vx = 0.75.
    cfg = _grid(5, 6, 4, 2.0, 3.0, 5.0)
    x = np.zeros((4, 6, 5))
    x[1, 3, 2] = 1.0
    cx, cy, cz = _centre(cfg, 2, 3, 1)
    p1 = np.array([[-50.0, cy + 0.25 * 3.0, cz - 0.5 * 5.0]])
    p2 = np.array([[50.0, cy + 0.25 * 3.0, cz - 0.5 * 5.0]])
    v = projector.fwd(cfg, x, p1, p2)[0, 0]
    assert v == pytest.approx(0.75, rel=1e-14)
    # reversed direction gives the same value
    assert projector.fwd(cfg, x, p2, p1)[0, 0] == pytest.approx(0.75, rel=1e-14)


def test_delta_response_oblique_principal_axis(oracle_built):
    # Oblique line in the x-y plane with |dy| > |dx| (principal axis y), through
    # the delta's centre at y = cy: at that plane the x offset is exactly 0.3 voxel
    # -> weight 0.7; step length = vy * |u| / |u_y|.
    cfg = _grid(7, 7, 1, 2.0, 2.0, 2.0)
    x = np.zeros((1, 7, 7))
    x[0, 3, 3] = 1.0
    cx, cy, _ = _centre(cfg, 3, 3, 0)
    slope = 0.4  # dx/dy
    x0 = cx + 0.3 * 2.0
    p1 = np.array([[x0 - slope * 40.0, cy - 40.0, 0.0]])
    p2 = np.array([[x0 + slope * 40.0, cy + 40.0, 0.0]])
    ell = 2.0 * math.sqrt(1 + slope ** 2)
    # Only the y-plane of row 3 can see the delta; there x sits 0.3 voxel right
    # of column 3.
    v = projector.fwd(cfg, x, p1, p2)[0, 0]
    assert v == pytest.approx(0.7 * ell, rel=1e-13)


def _oblique_line(cfg, centre, direction, offset_vox, half=60.0):
    """Endpoints of a line with the given direction that crosses the principal
    plane of `centre` (principal axis x) at `centre` + offset_vox * (0, vy, vz),
    reaching `half` mm along x on either side; and the crossing point."""
    c = np.array(centre, float)
    hit = c + np.array([0.0, offset_vox[0] * cfg["vy"], offset_vox[1] * cfg["vz"]])
    u = np.array(direction, float) / abs(direction[0])
    return hit - half * u, hit + half * u, hit


def test_delta_response_3d_line_varying_z(oracle_built):
    # A 3D line with a slope in y and z (principal axis x, ring-difference-like
    # tilt): at the x-plane of voxel column 5 it passes 0.2 voxel above the
    # centre of voxel (5, 2, 4) in y and 0.35 voxel below it in z.  Unit deltas
    # at the four voxels around that crossing answer with the bilinear weights
    # (0.8 * 0.65, 0.2 * 0.65, 0.8 * 0.35, 0.2 * 0.35) times the step length
    # l = vx |u| / |u_x|; a delta on the same plane but two voxels away in z
    # answers 0.  The z-coordinate of the sample comes from the line parameter
    # at that plane, so a slip in the axial interpolation changes these values.
    cfg = _grid(9, 8, 7, 2.0, 2.5, 3.0)
    direction = (1.0, 0.21, -0.37)  # |u_x|/vx = 0.5 > |u_z|/vz = 0.123 > |u_y|/vy = 0.084
    p1, p2, _ = _oblique_line(cfg, _centre(cfg, 5, 2, 4), direction, (0.2, -0.35))
    ell = 2.0 * math.sqrt(1.0 + 0.21 ** 2 + 0.37 ** 2)
    want = {(5, 2, 4): 0.8 * 0.65, (5, 3, 4): 0.2 * 0.65, (5, 2, 3): 0.8 * 0.35, (5, 3, 3): 0.2 * 0.35,
            (5, 2, 6): 0.0, (5, 4, 4): 0.0}
    for (ix, iy, iz), w in want.items():
        x = np.zeros((7, 8, 9))
        x[iz, iy, ix] = 1.0
        for a, b in ((p1, p2), (p2, p1)):  # either direction
            v = projector.fwd(cfg, x, a[None], b[None])[0, 0]
            assert v == pytest.approx(w * ell, rel=1e-13, abs=1e-15), (ix, iy, iz)


def test_delta_response_3d_principal_y_negative_slopes(oracle_built):
    # Principal axis y, x and z both decreasing along the line: crossing the
    # y-plane of voxel (3, 6, 2) at +0.45 voxel in x and +0.1 voxel in z gives
    # weights 0.55 * 0.9 at the voxel itself and 0.45 * 0.1 at (4, 6, 3).
    cfg = _grid(8, 10, 6, 2.2, 1.8, 2.6)
    c = np.array(_centre(cfg, 3, 6, 2))
    hit = c + np.array([0.45 * 2.2, 0.0, 0.1 * 2.6])
    u = np.array([-0.3, 1.0, -0.25])
    p1, p2 = hit - 40 * u, hit + 40 * u
    ell = 1.8 * math.sqrt(0.3 ** 2 + 1.0 + 0.25 ** 2)
    for (ix, iy, iz), w in {(3, 6, 2): 0.55 * 0.9, (4, 6, 3): 0.45 * 0.1, (4, 6, 2): 0.45 * 0.9,
                            (3, 6, 3): 0.55 * 0.1}.items():
        x = np.zeros((6, 10, 8))
        x[iz, iy, ix] = 1.0
        assert projector.fwd(cfg, x, p1[None], p2[None])[0, 0] == pytest.approx(w * ell, rel=1e-13)


def test_delta_response_3d_tof_hand_value(oracle_built):
    # The same tilted line with TOF: the crossing point sits at a known signed
    # distance t from the LOR centre (the centre is placed 31 mm before the
    # crossing along the line), so each bin's answer is the bilinear weight,
    # the step length and the bin's truncated-Gaussian mass
    # 1/2 [erf(clamp((t_b + w/2 - t) / (sqrt2 sigma))) - erf(clamp((t_b - w/2 - t) / (sqrt2 sigma)))].
    sig, wb = 9.0, 12.0
    cfg = dict(_grid(9, 8, 7, 2.0, 2.5, 3.0), n_tof=7, tof_bin=wb, tof_sigma=sig, tof_nsigma=3.0)
    direction = np.array([1.0, 0.21, -0.37])
    unit = direction / np.linalg.norm(direction)
    _, _, hit = _oblique_line(cfg, _centre(cfg, 5, 2, 4), direction, (0.2, -0.35))
    mid = hit - 31.0 * unit
    p1, p2 = mid - 70.0 * unit, mid + 70.0 * unit
    ell = 2.0 * math.sqrt(1.0 + 0.21 ** 2 + 0.37 ** 2)
    x = np.zeros((7, 8, 9))
    x[4, 2, 5] = 1.0
    got = projector.fwd(cfg, x, p1[None], p2[None])[0]
    c = 3.0 / math.sqrt(2.0)

    def E(d):
        return math.erf(min(max(d / (math.sqrt(2.0) * sig), -c), c))

    for b in range(7):
        tb = (b - 3) * wb
        w = 0.5 * (E(tb + wb / 2 - 31.0) - E(tb - wb / 2 - 31.0))
        assert got[b] == pytest.approx(0.8 * 0.65 * ell * w, rel=1e-12, abs=1e-15), b
    # bins 3 sigma + half a bin or more away from t = 31 mm receive nothing
    assert got[0] == 0.0 and got[1] == 0.0


def test_constant_image_axis_aligned(oracle_built):
    cfg = _grid(9, 8, 5, 1.5, 2.5, 3.5)
    x = np.full((5, 8, 9), 2.0)
    cx, cy, cz = _centre(cfg, 4, 2, 3)
    # along x through voxel centres: 2 * 9 * 1.5
    vx = projector.fwd(cfg, x, np.array([[-40, cy, cz]]), np.array([[40, cy, cz]]))[0, 0]
    assert vx == pytest.approx(27.0, rel=1e-14)
    # along y: 2 * 8 * 2.5
    vy = projector.fwd(cfg, x, np.array([[cx, -40, cz]]), np.array([[cx, 40, cz]]))[0, 0]
    assert vy == pytest.approx(40.0, rel=1e-14)
    # along z: 2 * 5 * 3.5
    vz = projector.fwd(cfg, x, np.array([[cx, cy, -40]]), np.array([[cx, cy, 40]]))[0, 0]
    assert vz == pytest.approx(35.0, rel=1e-14)


def test_45_degree_ray_c0(oracle_built):
    # The C0 view at 45 degrees through s = 0 runs along the grid diagonal through
    # voxel centres: 64 samples of a constant 1 with step 4 sqrt(2) mm.
    cfg = configs.get("c0_2d")
    x = np.ones((1, 64, 64))
    v15 = 15  # phi = pi * 15 / 60 = 45 deg
    p1, p2 = scanner.lor_endpoints(cfg, [v15], [45], [0])
    assert projector.fwd(cfg, x, p1, p2)[0, 0] == pytest.approx(64 * 4 * math.sqrt(2), rel=1e-12)
    v45 = 45  # 135 deg
    p1, p2 = scanner.lor_endpoints(cfg, [v45], [45], [0])
    assert projector.fwd(cfg, x, p1, p2)[0, 0] == pytest.approx(64 * 4 * math.sqrt(2), rel=1e-12)


@pytest.mark.parametrize("vox", [4.0, 2.0, 1.0])
def test_disc_chords_converge(oracle_built, vox):
    # Uniform disc of radius 50 mm (area-fraction voxelised); the line integral
    # through it at offset s is the chord 2 sqrt(R^2 - s^2).  Rays through the
    # inner half stay within 1%; the RMS error over rays up to R - 2 voxels must
    # fall as the grid is refined (discretisation error, not parity).
    R = 50.0
    n = int(round(128 / vox))
    cfg = dict(_grid(n, n, 1, vox, vox, vox), kind="parallel2d", phantom="disc")
    sh = np.array([[0, 0, 0, R, R, 1e6, 0, 1.0, 0]])
    x = np.zeros((1, n, n))
    data._lib().gen_voxelize(n, n, 1, vox, vox, vox, 8, 1, 1, data._p(sh), data._p(x))
    rng = np.random.default_rng(7)
    s = rng.uniform(-(R - 2 * vox), R - 2 * vox, 40)
    phi = rng.uniform(0, math.pi, 40)
    nrm = np.stack([np.cos(phi), np.sin(phi), 0 * phi], 1)
    t = np.stack([-np.sin(phi), np.cos(phi), 0 * phi], 1)
    p1 = s[:, None] * nrm - 200 * t
    p2 = s[:, None] * nrm + 200 * t
    got = projector.fwd(cfg, x, p1, p2)[:, 0]
    exact = 2 * np.sqrt(R ** 2 - s ** 2)
    rel = np.abs(got - exact) / exact
    assert rel[np.abs(s) < R / 2].max() < 0.01
    assert rel.max() < 0.03
    test_disc_chords_converge.errs = getattr(test_disc_chords_converge, "errs", {})
    test_disc_chords_converge.errs[vox] = np.sqrt(np.mean(rel ** 2))
    if len(test_disc_chords_converge.errs) == 3:
        e = test_disc_chords_converge.errs
        assert e[1.0] < e[2.0] < e[4.0]


@pytest.mark.parametrize("name", ["mini_tof", "mini_nontof", "mini_2d"])
def test_adjoint_identity(oracle_built, name):
    cfg = configs.get(name)
    rng = np.random.default_rng(11)
    views = list(range(cfg["n_views"]))
    p1, p2 = projector.view_lors(cfg, views)
    x = rng.uniform(0, 1, (cfg["nz"], cfg["ny"], cfg["nx"]))
    y = rng.uniform(0, 1, (p1.shape[0], cfg["n_tof"]))
    lhs = np.sum(projector.fwd(cfg, x, p1, p2) * y)
    rhs = np.sum(x * projector.back(cfg, y, p1, p2))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_dense_matrix_linearity(oracle_built):
    # Columns of A from unit images; P x must equal A x and P^T y must equal A^T y.
    cfg = configs.get("mini_tof", nx=5, ny=4, nz=3)
    p1, p2 = projector.view_lors(cfg, [0, 5, 9])
    nv = 5 * 4 * 3
    cols = []
    for j in range(nv):
        e = np.zeros(nv)
        e[j] = 1
        cols.append(projector.fwd(cfg, e, p1, p2).ravel())
    A = np.stack(cols, 1)
    rng = np.random.default_rng(3)
    x = rng.normal(size=nv)
    assert np.allclose(projector.fwd(cfg, x, p1, p2).ravel(), A @ x, rtol=1e-12, atol=1e-12)
    y = rng.normal(size=A.shape[0])
    assert np.allclose(projector.back(cfg, y, p1, p2).ravel(), A.T @ y, rtol=1e-12, atol=1e-12)


def test_tof_partition_of_unity_untruncated(oracle_built):
    # Without truncation and with bins covering the LOR far beyond its ends, the
    # TOF weights of a sample telescope to 1, so sum_b P_tof = P_nontof.
    cfg = configs.get("mini_tof", n_tof=25, tof_nsigma=0.0)
    p1, p2 = projector.view_lors(cfg, [0, 3, 7])
    x = np.random.default_rng(5).uniform(0, 1, (cfg["nz"], cfg["ny"], cfg["nx"]))
    tof = projector.fwd(cfg, x, p1, p2, tof=True)
    nontof = projector.fwd(cfg, x, p1, p2, tof=False)[:, 0]
    assert np.allclose(tof.sum(1), nontof, rtol=1e-12, atol=1e-12 * nontof.max())


def test_tof_truncated_weights_sum_to_erf(oracle_built):
    # The truncated Gaussian (+-3 sigma around the event) integrated over bins
    # that cover its whole window telescopes to the kernel's mass inside the
    # window: sum_b w_b = erf(3 / sqrt 2) exactly, wherever the event sits.
    sig = 60.0 * configs.FWHM_TO_SIGMA
    cfg = dict(_grid(3, 3, 1, 2.0, 2.0, 2.0), n_tof=13, tof_bin=40.0, tof_sigma=sig, tof_nsigma=3.0)
    x = np.zeros((1, 3, 3))
    x[0, 1, 1] = 1.0
    for off in np.linspace(-150, 150, 61):
        p1 = np.array([[-400.0 - off, 0.0, 0.0]])
        p2 = np.array([[400.0 - off, 0.0, 0.0]])
        tof = projector.fwd(cfg, x, p1, p2, tof=True)[0]
        nontof = projector.fwd(cfg, x, p1, p2, tof=False)[0, 0]
        assert tof.sum() / nontof == pytest.approx(math.erf(3 / math.sqrt(2)), rel=1e-13)


def test_tof_kernel_centre_bin_and_support(oracle_built):
    # A source at the LOR centre: bins symmetric about the centre bin; the centre
    # bin holds erf(20 / (sqrt(2) sigma)) (window +-76.4 mm covers the bin);
    # a bin whose nearest edge is farther than 3 sigma (centre 120 mm away,
    # edge at 100 mm) gets nothing; the bins 80 mm away keep their overlap with
    # the window, [60, 76.4] mm.
    sig = 60.0 * configs.FWHM_TO_SIGMA
    cfg = dict(_grid(3, 3, 1, 2.0, 2.0, 2.0), n_tof=13, tof_bin=40.0, tof_sigma=sig, tof_nsigma=3.0)
    x = np.zeros((1, 3, 3))
    x[0, 1, 1] = 1.0
    p1 = np.array([[-300.0, 0.0, 0.0]])
    p2 = np.array([[300.0, 0.0, 0.0]])
    tof = projector.fwd(cfg, x, p1, p2, tof=True)[0] / 2.0  # step length 2 mm
    assert np.allclose(tof, tof[::-1], rtol=1e-13)
    assert tof[6] == pytest.approx(math.erf(20 / (math.sqrt(2) * sig)), rel=1e-13)
    assert tof[3] == 0.0 and tof[9] == 0.0
    gauss_mass_60_to_cut = 0.5 * (math.erf(3 / math.sqrt(2)) - math.erf(60 / (math.sqrt(2) * sig)))
    assert tof[4] == pytest.approx(gauss_mass_60_to_cut, rel=1e-13)
    assert tof.sum() == pytest.approx(math.erf(3 / math.sqrt(2)), rel=1e-13)


def test_parallel_beam_mass_at_grid_angles(oracle_built):
    # At 0 and 90 degrees the C0 rays fall half-way between voxel columns, so the
    # interpolation splits every column evenly between two rays and
    # sum_k p_k * ds equals sum(x) * vx * vy.
    cfg = configs.get("c0_2d")
    x = np.random.default_rng(2).uniform(0, 1, (1, 64, 64))
    for view in (0, 30):
        p1, p2 = projector.view_lors(cfg, [view])
        p = projector.fwd(cfg, x, p1, p2)[:, 0]
        assert p.sum() * 4.0 == pytest.approx(x.sum() * 16.0, rel=1e-13)


def test_scanner_geometry_facts():
    # Cylinder LOR endpoints lie on the ring; the LOR's distance from the axis is
    # |s_k|; plane counts follow the ring-difference limit.
    cfg = configs.get("c1_3d")
    assert configs.n_planes(cfg) == 2204
    assert configs.n_planes(configs.get("c3_diff")) == 268
    p1, p2 = scanner.transaxial_endpoints(cfg, [0, 17, 251])
    assert np.allclose(np.hypot(p1[..., 0], p1[..., 1]), 328.0, rtol=1e-14)
    assert np.allclose(np.hypot(p2[..., 0], p2[..., 1]), 328.0, rtol=1e-14)
    s = scanner.radial_coords(cfg)
    d = np.abs(p1[..., 0] * p2[..., 1] - p1[..., 1] * p2[..., 0]) / np.hypot(*(p2 - p1).transpose(2, 0, 1))
    assert np.allclose(d, np.abs(s)[None, :], atol=1e-10)
    assert s[172] - s[171] == pytest.approx(2 * 328 * math.sin(math.pi / 1008), rel=1e-12)
