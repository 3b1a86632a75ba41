"""ORACLE — test infrastructure only.  Relative difference prior in FP64.

Value (eq. (rdp), Section 1.2):
    S(x) = 1/2 sum_i sum_{j in N_i} w_ij k_i k_j (x_i - x_j)^2 / (x_i + x_j + gamma |x_i - x_j| + eps)
Gradient and Hessian diagonal (Appendix A), with d = x_i - x_j, s = x_i + x_j,
phi = s + gamma |d| + eps:
    dS/dx_i   = sum_j w k_i k_j d (2 phi - (d + gamma |d|)) / phi^2
    d2S/dx_i2 = 2 sum_j w k_i k_j (s - d + eps)^2 / phi^3
Hessian-vector product (derived from the value; not printed in the paper): the
off-diagonal entries are H_ij = -2 w k_i k_j (s - d + eps)(s + d + eps) / phi^3,
i.e. -2 w k k (2 x_j + eps)(2 x_i + eps) / phi^3.

N_i holds the 26 (3D) or 8 (2D, nz == 1) grid neighbours that lie inside the
grid.  Weights are supplied per offset; ``default_weights`` gives the reading
w = v_x / distance (so in-plane face neighbours weigh 1).
"""

import itertools

import numpy as np


def offsets(nz):
    if nz == 1:
        return [(0, dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dy, dx) != (0, 0)]
    return [o for o in itertools.product((-1, 0, 1), repeat=3) if o != (0, 0, 0)]


def default_weights(vx, vy, vz, nz):
    """w[(dz,dy,dx)] = vx / |(dz vz, dy vy, dx vx)| for every neighbour offset."""
    return {o: vx / np.sqrt((o[0] * vz) ** 2 + (o[1] * vy) ** 2 + (o[2] * vx) ** 2) for o in offsets(nz)}


def _pairs(shape, off):
    """Slices (I, J) so that x[I] are voxels i whose neighbour i+off is inside
    the grid, and x[J] are those neighbours."""
    I, J = [], []
    for n, d in zip(shape, off):
        if d == 0:
            I.append(slice(0, n))
            J.append(slice(0, n))
        elif d > 0:
            I.append(slice(0, n - d))
            J.append(slice(d, n))
        else:
            I.append(slice(-d, n))
            J.append(slice(0, n + d))
    return tuple(I), tuple(J)


def _kap(x, kappa):
    return np.ones_like(x) if kappa is None else np.asarray(kappa, np.float64)


def value(x, w, gamma, eps, kappa=None):
    x = np.asarray(x, np.float64)
    k = _kap(x, kappa)
    S = 0.0
    for off, wij in w.items():
        I, J = _pairs(x.shape, off)
        d = x[I] - x[J]
        S += np.sum(wij * k[I] * k[J] * d * d / (x[I] + x[J] + gamma * np.abs(d) + eps))
    return 0.5 * S


def grad(x, w, gamma, eps, kappa=None):
    x = np.asarray(x, np.float64)
    k = _kap(x, kappa)
    g = np.zeros_like(x)
    for off, wij in w.items():
        I, J = _pairs(x.shape, off)
        d = x[I] - x[J]
        phi = x[I] + x[J] + gamma * np.abs(d) + eps
        g[I] += wij * k[I] * k[J] * d * (2 * phi - (d + gamma * np.abs(d))) / phi ** 2
    return g


def hessdiag(x, w, gamma, eps, kappa=None):
    x = np.asarray(x, np.float64)
    k = _kap(x, kappa)
    h = np.zeros_like(x)
    for off, wij in w.items():
        I, J = _pairs(x.shape, off)
        d = x[I] - x[J]
        s = x[I] + x[J]
        phi = s + gamma * np.abs(d) + eps
        h[I] += 2 * wij * k[I] * k[J] * (s - d + eps) ** 2 / phi ** 3
    return h


def hvp(x, v, w, gamma, eps, kappa=None):
    """Hessian of S at x applied to v."""
    x = np.asarray(x, np.float64)
    v = np.asarray(v, np.float64)
    k = _kap(x, kappa)
    out = np.zeros_like(x)
    for off, wij in w.items():
        I, J = _pairs(x.shape, off)
        d = x[I] - x[J]
        s = x[I] + x[J]
        phi = s + gamma * np.abs(d) + eps
        c = 2 * wij * k[I] * k[J] / phi ** 3
        out[I] += c * ((s - d + eps) ** 2 * v[I] - (s - d + eps) * (s + d + eps) * v[J])
    return out
