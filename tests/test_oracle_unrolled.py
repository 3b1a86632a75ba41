"""Pins for the oracle's reverse-mode pieces: the FP64 torch prior against the
numpy closed forms, the unrolled forward pass against the oracle's Algorithm 1,
autograd gradients of the unrolled reconstruction (with and without the
image-space resolution model) against central finite differences of its
forward pass, the data-term Hessian-vector product against
finite differences of the data gradient, and the preconditioner's
vector-Jacobian product against finite differences."""

import numpy as np
import pytest
import torch

from oracle import poisson, projector, rdp, recon, unrolled
from synth import configs, data


def _tiny(beta=0.5, n_subsets=3, seed=0, psf_fwhm=0.0):
    cfg = configs.get("mini_2d", nx=8, ny=8, n_views=12, n_rad=15, rad_spacing=4.0,
                      n_subsets=n_subsets, seed=seed, phantom="c0_small", counts_total=5e4, psf_fwhm=psf_fwhm)
    d = data.make_dataset(cfg)
    prob = recon.Problem(cfg, d["y"].astype(np.float64), d["r"], d["mult"], beta=beta,
                         gamma=2.0, eps=1e-2, alpha=1.0, delta=1e-3)
    return cfg, d, prob


def _schedule(cfg, n_epochs):
    n = cfg["n_subsets"]
    orders = data.subset_orders(cfg, n_epochs)
    taus = [[1.0 / (1.0 + 0.02 * (e * n + j) / n) for j in range(n)] for e in range(n_epochs)]
    return orders, taus, set(recon.pc_update_iters(n))


def test_torch_prior_matches_numpy_closed_forms():
    rng = np.random.default_rng(3)
    for shape in ((1, 7, 9), (4, 5, 6)):
        x = rng.uniform(0, 3, shape)
        x[0, 0, :2] = 0.0
        kappa = rng.uniform(0.5, 1.5, shape)
        w = rdp.default_weights(2.0, 2.0, 2.5, shape[0])
        xt, kt = torch.from_numpy(x), torch.from_numpy(kappa)
        g = unrolled.prior_grad(xt, w, 2.0, 0.01, kt).numpy()
        h = unrolled.prior_hessdiag(xt, w, 2.0, 0.01, kt).numpy()
        assert np.allclose(g, rdp.grad(x, w, 2.0, 0.01, kappa), rtol=1e-13, atol=1e-14)
        assert np.allclose(h, rdp.hessdiag(x, w, 2.0, 0.01, kappa), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("psf_fwhm", [0.0, 6.0])
def test_unrolled_forward_matches_algorithm1(psf_fwhm):
    cfg, d, prob = _tiny(psf_fwhm=psf_fwhm)
    n = prob.n
    orders, taus, upd = _schedule(cfg, 3)
    x0 = recon.osem_epoch(prob, np.ones(prob.shape))
    ref = recon.svrg(prob, x0, 3, recon.order_rule(orders), lambda k: taus[k // n][k % n], upd)
    u = unrolled.Unrolled(prob)
    with torch.no_grad():
        got = u.svrg(torch.from_numpy(x0.copy()), torch.tensor(np.log(prob.beta), dtype=torch.float64), 3, orders,
                     taus, upd).numpy()
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("psf_fwhm", [0.0, 6.0])
def test_unrolled_gradient_matches_finite_differences(psf_fwhm):
    # with a resolution model this also pins the blur's adjoint in autograd
    cfg, d, prob = _tiny(psf_fwhm=psf_fwhm)
    orders, taus, upd = _schedule(cfg, 3)
    x0 = recon.osem_epoch(prob, np.ones(prob.shape))
    target = d["x_true"].astype(np.float64)
    lb = np.log(prob.beta)
    L, gx, gb, _ = unrolled.loss_and_grads(prob, x0, lb, target, 3, orders, taus, upd)
    h = 1e-5
    fd_b = (unrolled.loss(prob, x0, lb + h, target, 3, orders, taus, upd)
            - unrolled.loss(prob, x0, lb - h, target, 3, orders, taus, upd)) / (2 * h)
    assert gb == pytest.approx(fd_b, rel=1e-5)
    rng = np.random.default_rng(1)
    for _ in range(2):
        v = rng.standard_normal(x0.shape) * (x0 > 0.05 * x0.max())
        t = 1e-6 * np.linalg.norm(x0) / np.linalg.norm(v)
        fd = (unrolled.loss(prob, x0 + t * v, lb, target, 3, orders, taus, upd)
              - unrolled.loss(prob, x0 - t * v, lb, target, 3, orders, taus, upd)) / (2 * t)
        assert float(np.sum(gx * v)) == pytest.approx(fd, rel=1e-5)


def test_data_hessian_vector_product_matches_finite_differences():
    cfg, d, prob = _tiny()
    rng = np.random.default_rng(2)
    x = recon.osem_epoch(prob, np.ones(prob.shape))
    v = rng.standard_normal(prob.shape)
    for i in range(prob.n):
        p1, p2 = prob.lors[i]
        yb = prob.ybar(x, i)
        hv = projector.back(cfg, prob.a[i] ** 2 * prob.y[i] / yb ** 2 * projector.fwd(cfg, v, p1, p2), p1, p2)
        t = 1e-5 * np.linalg.norm(x) / np.linalg.norm(v)
        fd = (prob.data_grad(x + t * v, i) - prob.data_grad(x - t * v, i)) / (2 * t)
        assert np.linalg.norm(hv - fd) <= 1e-6 * np.linalg.norm(hv)


def test_preconditioner_vjp_matches_finite_differences():
    rng = np.random.default_rng(4)
    shape = (3, 6, 7)
    x = rng.uniform(0.0, 2.0, shape)
    x[1, 2, 3] = 0.0
    sens = rng.uniform(0.5, 2.0, shape)
    w = rdp.default_weights(2.0, 2.0, 2.5, shape[0])
    beta, gamma, eps, alpha, delta = 0.7, 2.0, 0.05, 1.0, 1e-3
    Dbar = rng.standard_normal(shape)
    xt = torch.tensor(x, requires_grad=True)
    bt = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    D = unrolled.preconditioner(xt, torch.from_numpy(sens), bt, w, gamma, eps, alpha, delta)
    (D * torch.from_numpy(Dbar)).sum().backward()

    def Dnp(xx, bb):
        with torch.no_grad():
            return unrolled.preconditioner(torch.from_numpy(xx), torch.from_numpy(sens),
                                           torch.tensor(bb, dtype=torch.float64), w, gamma, eps, alpha,
                                           delta).numpy()

    v = rng.standard_normal(shape)
    t = 1e-6
    fd = np.sum(Dbar * (Dnp(x + t * v, beta) - Dnp(x - t * v, beta))) / (2 * t)
    assert float(np.sum(xt.grad.numpy() * v)) == pytest.approx(fd, rel=1e-6)
    fdb = np.sum(Dbar * (Dnp(x, beta + t) - Dnp(x, beta - t))) / (2 * t)
    assert float(bt.grad) == pytest.approx(fdb, rel=1e-6)
    # closed form of the value itself (eq. (preconditioner))
    h = rdp.hessdiag(x, w, gamma, eps)
    assert np.allclose(Dnp(x, beta), (x + delta) / (sens + alpha * beta * h * (x + delta)), rtol=1e-14)


def test_frozen_clip_finite_differences_match_autograd():
    # Along a direction that moves voxels across the clip, the clipped map has
    # kinks; on the smooth piece selected by the base run's clip decisions its
    # central differences converge to the autograd derivative.
    cfg, d, prob = _tiny(beta=0.05)
    orders, taus, upd = _schedule(cfg, 4)
    x0 = recon.osem_epoch(prob, np.ones(prob.shape))
    target = d["x_true"].astype(np.float64)
    lb = np.log(prob.beta)
    masks = []
    L0 = unrolled.loss(prob, x0, lb, target, 4, orders, taus, upd, record=masks)
    L, gx, gb, _ = unrolled.loss_and_grads(prob, x0, lb, target, 4, orders, taus, upd)
    assert L0 == pytest.approx(L, rel=1e-14)
    assert unrolled.loss(prob, x0, lb, target, 4, orders, taus, upd, clip_masks=masks) == pytest.approx(L, rel=1e-14)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(x0.shape)
    for rel in (1e-5, 1e-6):
        t = rel * np.linalg.norm(x0) / np.linalg.norm(v)
        fd = (unrolled.loss(prob, x0 + t * v, lb, target, 4, orders, taus, upd, clip_masks=masks)
              - unrolled.loss(prob, x0 - t * v, lb, target, 4, orders, taus, upd, clip_masks=masks)) / (2 * t)
        assert float(np.sum(gx * v)) == pytest.approx(fd, rel=1e-6)
