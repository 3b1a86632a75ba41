"""ORACLE — test infrastructure only.  Image-space resolution model of the
forward operator (Section 3.1: an isotropic Gaussian kernel in image space
models the limited spatial resolution), A = P G, in FP64.

Reading (the paper gives only the kernel's width): 4 mm is the FWHM; G is the
separable convolution with, per axis, sampled Gaussian weights
exp(-d^2 / (2 s^2)) (s = sigma in voxels of that axis) for integer offsets
|d| <= floor(4 s + 1/2), normalised to sum 1, and zero outside the grid; a 2D
image (one plane) is blurred in-plane only.  With zero boundaries and a
symmetric kernel G is a symmetric matrix, so A^T = G P^T.
"""

import math

import numpy as np


def axis_weights(sigma_vox):
    """Weights of offsets -r..r of one axis."""
    r = int(4.0 * sigma_vox + 0.5)
    d = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-0.5 * d * d / (sigma_vox * sigma_vox))
    return w / w.sum()


def blur(x, cfg):
    """G x for an image [nz][ny][nx] of the configuration `cfg`."""
    fwhm = float(cfg.get("psf_fwhm", 0.0))
    x = np.asarray(x, np.float64)
    if fwhm <= 0:
        return x.copy()
    sigma_mm = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    out = x.copy()
    # axes of the [z][y][x] array: x is axis 2, y axis 1, z axis 0
    axes = [(2, cfg["vx"]), (1, cfg["vy"])] + ([(0, cfg["vz"])] if x.shape[0] > 1 else [])
    for ax, v in axes:
        w = axis_weights(sigma_mm / v)
        r = (w.size - 1) // 2
        src = out
        out = np.zeros_like(src)
        n = src.shape[ax]
        for k, wk in enumerate(w):
            d = k - r
            # out[c] += w_d src[c + d] for 0 <= c + d < n
            lo, hi = max(0, -d), min(n, n - d)
            if lo >= hi:
                continue
            dst = [slice(None)] * 3
            srcs = [slice(None)] * 3
            dst[ax] = slice(lo, hi)
            srcs[ax] = slice(lo + d, hi + d)
            out[tuple(dst)] += wk * src[tuple(srcs)]
    return out
