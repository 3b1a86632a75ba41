"""ORACLE — test infrastructure only.  FP64 Joseph projector pair (ctypes over
``joseph.c``) for explicit lists of LORs.

The system model of the paper's problem (eq. (1), Section 1) is
y_bar = A x + r with A = diag(a) P, where P is the line-integral operator
(TOF-resolved when the scanner has TOF bins) and a holds per-LOR multiplicative
factors shared by all TOF bins of a LOR.
"""

import ctypes
import os

import numpy as np

from . import lib
from synth import scanner

_NTHREADS = int(os.environ.get("ORACLE_THREADS", "0"))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tof(cfg, tof):
    if tof and cfg["n_tof"] > 1:
        return cfg["n_tof"], float(cfg["tof_bin"]), float(cfg["tof_sigma"]), float(cfg["tof_nsigma"])
    return 1, 0.0, 1.0, 0.0


def fwd(cfg, x, p1, p2, tof=True):
    """Line integrals P x for LORs (p1[k], p2[k]); returns [N, T] FP64."""
    x = np.ascontiguousarray(x, np.float64).reshape(cfg["nz"], cfg["ny"], cfg["nx"])
    p1 = np.ascontiguousarray(p1, np.float64)
    p2 = np.ascontiguousarray(p2, np.float64)
    nt, tb, sg, ns = _tof(cfg, tof)
    out = np.zeros((p1.shape[0], nt))
    lib().orc_joseph(0, p1.shape[0], _p(p1), _p(p2), cfg["nx"], cfg["ny"], cfg["nz"],
                     cfg["vx"], cfg["vy"], cfg["vz"], nt, tb, sg, ns, _p(x), _p(out), _NTHREADS)
    return out


def back(cfg, s, p1, p2, tof=True):
    """Adjoint P^T s for values s[N, T]; returns image [nz][ny][nx] FP64."""
    nt, tb, sg, ns = _tof(cfg, tof)
    p1 = np.ascontiguousarray(p1, np.float64)
    p2 = np.ascontiguousarray(p2, np.float64)
    s = np.ascontiguousarray(s, np.float64).reshape(p1.shape[0], nt)
    img = np.zeros((cfg["nz"], cfg["ny"], cfg["nx"]))
    lib().orc_joseph(1, p1.shape[0], _p(p1), _p(p2), cfg["nx"], cfg["ny"], cfg["nz"],
                     cfg["vx"], cfg["vy"], cfg["vz"], nt, tb, sg, ns, _p(img), _p(s), _NTHREADS)
    return img


def view_lors(cfg, views):
    """Endpoints of every LOR of the given views, in sinogram order."""
    v, k, p = scanner.subset_lor_indices(cfg, views)
    return scanner.lor_endpoints(cfg, v, k, p)
