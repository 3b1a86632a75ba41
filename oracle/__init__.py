"""ORACLE — test infrastructure only.

A plain, slow, FP64 CPU implementation of what the reconstruction path computes,
written from the paper ("Fast PET Reconstruction with Variance Reduction and
Prior-Aware Preconditioning"): the Joseph projector pair with TOF, the Poisson
(KL) data term and its subset gradients, the relative difference prior (value,
gradient, Hessian diagonal, Hessian-vector product), the harmonic prior-aware
preconditioner, MLEM/OSEM, and the preconditioned SVRG iteration of Algorithm 1.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2506_04976_amd``) and never imports it; the two meet only through the
seeded inputs of ``synth``.
"""

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build(force=False):
    """Compile the FP64 projector with gcc."""
    so = os.path.join(_HERE, "_joseph.so")
    src = os.path.join(_HERE, "joseph.c")
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", so, src, "-lm"])
    return so


def build_native(dest_dir):
    """Compile the same projector source with -O3 -march=native for the host
    it runs on, into dest_dir (for timing the oracle as a CPU baseline; the
    parity tests use build())."""
    so = os.path.join(dest_dir, "_joseph_native.so")
    src = os.path.join(_HERE, "joseph.c")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-o", so, src, "-lm"])
    return so


def use_library(path):
    """Route the oracle's projector calls to another build of joseph.c."""
    global _LIB
    _LIB = _load(path)


def _load(path):
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    L.orc_joseph.argtypes = ([ctypes.c_int, ctypes.c_long, P, P] + [ctypes.c_int] * 3 +
                             [ctypes.c_double] * 3 + [ctypes.c_int] + [ctypes.c_double] * 3 +
                             [P, P, ctypes.c_int])
    L.orc_joseph.restype = None
    return L


def lib():
    global _LIB
    if _LIB is None:
        _LIB = _load(build())
    return _LIB

