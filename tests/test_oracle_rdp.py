"""Pins for the FP64 relative-difference-prior oracle: a hand-computed value,
finite differences of the value (gradient, Hessian diagonal, Hessian-vector
product), the constant-image closed forms, 1-homogeneity at eps = 0 and the
total-variation limit (Section 1.2, Appendix A)."""

import math

import numpy as np
import pytest

from oracle import rdp


def test_two_voxel_hand_value():
    # Two voxels side by side in x (2D grid of one row): the pair appears twice in
    # the double sum, so S = w (x1 - x2)^2 / (x1 + x2 + gamma |x1 - x2| + eps)
    # = 4 / (4 + 4 + 0.5) = 8/17.
    x = np.array([[[1.0, 3.0]]])
    w = rdp.default_weights(1.0, 1.0, 1.0, 1)
    assert rdp.value(x, w, gamma=2.0, eps=0.5) == pytest.approx(8.0 / 17.0, rel=1e-15)
    # gradient by hand from S(x1, x2) = (x1 - x2)^2 / (x1 + x2 + 2|x1 - x2| + 0.5):
    # at (1, 3): dS/dx1 = (-4 * 8.5 - 4 * (1 - 2)) / 8.5^2 = -30/72.25 and
    # dS/dx2 = (4 * 8.5 - 4 * (1 + 2)) / 8.5^2 = 22/72.25 (not antisymmetric).
    g = rdp.grad(x, w, gamma=2.0, eps=0.5)
    assert g[0, 0, 0] == pytest.approx(-30.0 / 72.25, rel=1e-15)
    assert g[0, 0, 1] == pytest.approx(22.0 / 72.25, rel=1e-15)


def test_default_weights_reading():
    w = rdp.default_weights(2.0, 2.0, 4.0, 5)
    assert len(w) == 26
    assert w[(0, 0, 1)] == 1.0 and w[(0, 1, 0)] == 1.0
    assert w[(0, 1, 1)] == pytest.approx(1 / math.sqrt(2))
    assert w[(1, 0, 0)] == pytest.approx(0.5)
    assert len(rdp.default_weights(1, 1, 1, 1)) == 8


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.2, 3.0, shape)
    x[0, 0, :2] = 0.0  # include zeros (the boundary of the feasible set)
    return x


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 6, 7)])
def test_gradient_finite_differences(shape):
    x = _rand(shape, 1)
    w = rdp.default_weights(1.0, 1.3, 0.8, shape[0])
    kappa = np.random.default_rng(9).uniform(0.5, 1.5, shape)
    g = rdp.grad(x, w, 2.0, 0.05, kappa)
    h = 1e-6
    rng = np.random.default_rng(2)
    for _ in range(12):
        idx = tuple(rng.integers(0, n) for n in shape)
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (rdp.value(xp, w, 2.0, 0.05, kappa) - rdp.value(xm, w, 2.0, 0.05, kappa)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_hessdiag_and_hvp_finite_differences():
    shape = (3, 4, 5)
    # no equal neighbours: the third derivative jumps at d = 0, which would
    # spoil the finite-difference accuracy there
    x = np.random.default_rng(4).uniform(0.1, 3.0, shape)
    w = rdp.default_weights(1.0, 1.0, 1.2, 3)
    kappa = np.random.default_rng(8).uniform(0.5, 1.5, shape)
    H = rdp.hessdiag(x, w, 2.0, 0.05, kappa)
    h = 1e-5
    rng = np.random.default_rng(3)
    for _ in range(10):
        idx = tuple(rng.integers(0, n) for n in shape)
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (rdp.grad(xp, w, 2.0, 0.05, kappa)[idx] - rdp.grad(xm, w, 2.0, 0.05, kappa)[idx]) / (2 * h)
        assert H[idx] == pytest.approx(fd, rel=1e-6)
    v = np.random.default_rng(5).normal(size=shape)
    Hv = rdp.hvp(x, v, w, 2.0, 0.05, kappa)
    fd = (rdp.grad(x + h * v, w, 2.0, 0.05, kappa) - rdp.grad(x - h * v, w, 2.0, 0.05, kappa)) / (2 * h)
    assert np.allclose(Hv, fd, rtol=1e-6, atol=1e-8)
    # the HVP's diagonal part equals the Hessian diagonal
    e = np.zeros(shape); e[1, 2, 3] = 1.0
    assert rdp.hvp(x, e, w, 2.0, 0.05, kappa)[1, 2, 3] == pytest.approx(H[1, 2, 3], rel=1e-14)


def test_constant_image_closed_forms():
    c, eps, gamma = 1.7, 0.01, 2.0
    x = np.full((4, 5, 6), c)
    w = rdp.default_weights(1.0, 1.0, 1.0, 4)
    assert np.all(rdp.grad(x, w, gamma, eps) == 0.0)
    assert rdp.value(x, w, gamma, eps) == 0.0
    H = rdp.hessdiag(x, w, gamma, eps)
    # interior voxel sees all 26 neighbours: 2 sum(w) (2c + eps)^2 / (2c + eps)^3
    assert H[1, 2, 3] == pytest.approx(2 * sum(w.values()) / (2 * c + eps), rel=1e-14)
    # corner voxel sees 7 neighbours: 3 faces, 3 edge diagonals, 1 corner diagonal
    assert H[0, 0, 0] == pytest.approx(2 * (3 + 3 / math.sqrt(2) + 1 / math.sqrt(3)) / (2 * c + eps), rel=1e-14)


def test_one_homogeneous_at_zero_eps():
    # With eps = 0 every pair term d^2 / (s + gamma |d|) is 1-homogeneous, so
    # Euler's identity gives <x, grad S(x)> = S(x).
    x = _rand((3, 4, 5), 6) + 0.3
    w = rdp.default_weights(1.0, 1.0, 1.0, 3)
    S = rdp.value(x, w, 2.0, 0.0)
    assert np.sum(x * rdp.grad(x, w, 2.0, 0.0)) == pytest.approx(S, rel=1e-13)


def test_total_variation_limit():
    # If gamma |d| dominates s + eps the pair term tends to |d| / gamma
    # (Section 1.2), so gamma * S -> 1/2 sum_i sum_j w |x_i - x_j|.
    x = _rand((2, 3, 4), 7)
    w = rdp.default_weights(1.0, 1.0, 1.0, 2)
    gamma = 1e7
    tv = 0.0
    for off, wij in w.items():
        I, J = rdp._pairs(x.shape, off)
        tv += np.sum(wij * np.abs(x[I] - x[J]))
    assert gamma * rdp.value(x, w, gamma, 1e-9) == pytest.approx(0.5 * tv, rel=1e-5)
