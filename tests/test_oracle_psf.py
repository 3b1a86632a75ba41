"""Pins for the oracle's image-space resolution model (Section 3.1): the
separable blur equals scipy.ndimage's Gaussian filter with zero boundaries and
the same truncation, it is symmetric, it keeps the mass of an interior point
source with the kernel's second moment close to sigma^2, a 2D image is blurred
in-plane only, and A = P G with A^T = G P^T passes the adjoint identity."""

import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import psf, recon
from synth import configs, data


def _cfg(fwhm, nz=9, vx=2.0, vy=2.5, vz=3.0):
    return dict(psf_fwhm=fwhm, vx=vx, vy=vy, vz=vz, nz=nz)


@pytest.mark.parametrize("fwhm", [2.0, 4.0, 7.5])
def test_blur_matches_scipy_gaussian_filter(fwhm):
    rng = np.random.default_rng(0)
    x = rng.random((9, 13, 11))
    cfg = _cfg(fwhm)
    s = fwhm / (2 * math.sqrt(2 * math.log(2)))
    ref = x
    for ax, v in ((2, cfg["vx"]), (1, cfg["vy"]), (0, cfg["vz"])):
        ref = ndimage.gaussian_filter1d(ref, s / v, axis=ax, mode="constant", cval=0.0, truncate=4.0)
    assert np.allclose(psf.blur(x, cfg), ref, rtol=1e-13, atol=1e-15)
    # one plane: in-plane only
    x2 = rng.random((1, 13, 11))
    ref2 = x2
    for ax, v in ((2, cfg["vx"]), (1, cfg["vy"])):
        ref2 = ndimage.gaussian_filter1d(ref2, s / v, axis=ax, mode="constant", cval=0.0, truncate=4.0)
    assert np.allclose(psf.blur(x2, cfg), ref2, rtol=1e-13, atol=1e-15)


def test_blur_symmetric_mass_and_width():
    rng = np.random.default_rng(1)
    cfg = _cfg(6.0, nz=15, vx=1.5, vy=1.5, vz=1.5)
    a, b = rng.random((15, 21, 19)), rng.random((15, 21, 19))
    assert float(np.sum(psf.blur(a, cfg) * b)) == pytest.approx(float(np.sum(a * psf.blur(b, cfg))), rel=1e-13)
    d = np.zeros((15, 21, 19))
    d[7, 10, 9] = 1.0
    g = psf.blur(d, cfg)
    assert g.sum() == pytest.approx(1.0, rel=1e-13)
    s_vox = 6.0 / (2 * math.sqrt(2 * math.log(2))) / 1.5
    prof = g.sum(axis=(0, 1))
    var = float(np.sum(prof * (np.arange(19) - 9) ** 2))
    assert var == pytest.approx(s_vox ** 2, rel=1e-3)
    assert np.array_equal(psf.blur(d, _cfg(0.0)), d)


def test_blurred_system_adjoint(oracle_built):
    cfg = configs.get("mini_tof", psf_fwhm=6.0)
    d = data.make_dataset(cfg)
    prob = recon.Problem(cfg, d["y"], d["r"], d["mult"], beta=0.1, gamma=2.0, eps=1e-2)
    rng = np.random.default_rng(2)
    x = rng.random(prob.shape)
    for i in (0, prob.n - 1):
        s = rng.random(prob.y[i].shape)
        lhs = float(np.sum(prob.fwd(x, i) * s))
        rhs = float(np.sum(x * prob.back(s, i)))
        assert lhs == pytest.approx(rhs, rel=1e-12)
    # the blur sits inside the projector: P (G x) with G x computed separately
    p1, p2 = prob.lors[0]
    from oracle import projector
    assert np.allclose(prob.fwd(x, 0), projector.fwd(cfg, psf.blur(x, cfg), p1, p2), rtol=1e-14)
