"""GPU parity of the reverse-mode path: the data-term and prior Hessian-vector
products, the preconditioner's vector-Jacobian product, and gradients of a loss
of the unrolled preconditioned-SVRG reconstruction with respect to the initial
image and log(beta), all through the C ABI against the FP64 oracle (torch
autograd over oracle operations), plus central finite differences on the
3D workload of the differentiable configuration.  One case carries the
image-space resolution model (A = P G).

Tolerances: Hessian-vector products (summands of both signs) use a
cancellation-aware denominator, ||hv_gpu - hv_orc|| <= 1e-5 ||sum of |summands|||;
the preconditioner VJP and the unrolled gradients use relative L2 <= 1e-4.
"""

import numpy as np
import pytest
import torch

from oracle import projector, psf, rdp, recon, unrolled
from synth import configs, data

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


class Case:
    def __init__(self, name):
        import paper_2506_04976_amd as pm
        self.pm = pm
        self.cfg = configs.get(name)
        self.d = data.make_dataset(self.cfg)
        self.geom = pm.Geometry(self.cfg)
        self.dev = torch.device("cuda:0")
        rng = np.random.default_rng(7)
        self.x_np = (self.d["x_true"] * rng.uniform(0.7, 1.3, self.d["x_true"].shape) +
                     0.05 * self.d["x_true"].max()).astype(np.float32)
        self.x = torch.from_numpy(self.x_np.ravel()).to(self.dev)
        self.y = torch.from_numpy(self.d["y"].ravel()).to(self.dev)
        self.r = torch.from_numpy(self.d["r"].ravel()).to(self.dev)
        self.a = torch.from_numpy(self.d["mult"].ravel()).to(self.dev)
        self.T = self.cfg["n_tof"]
        self.shape = (self.cfg["nz"], self.cfg["ny"], self.cfg["nx"])
        self.w = rdp.default_weights(self.cfg["vx"], self.cfg["vy"], self.cfg["vz"], self.cfg["nz"])
        self.w27 = pm.rdp_weights27(self.cfg["vx"], self.cfg["vy"], self.cfg["vz"])

    def views(self, subset):
        return list(range(self.cfg["n_views"])) if subset < 0 else configs.subset_views(self.cfg, subset)


@pytest.fixture(scope="module", params=["mini_tof", "mini_nontof", "c0_2d", "mini_tof_psf"])
def case(request):
    _say(f"\n[gpu unrolled case {request.param}]")
    return Case(request.param)


def test_subset_hvp_parity(case):
    pm = case.pm
    rng = np.random.default_rng(11)
    v_np = rng.standard_normal(case.shape).astype(np.float32)
    v = torch.from_numpy(v_np.ravel()).to(case.dev)
    work = torch.zeros(case.geom.n_bins, device=case.dev)
    hv = torch.empty(case.geom.n_vox, device=case.dev)
    for subset in (0, case.cfg["n_subsets"] - 1, -1):
        pm.pet_subset_hvp(case.geom, subset, case.x, v, case.y, case.r, case.a, work, hv)
        views = case.views(subset)
        p1, p2 = projector.view_lors(case.cfg, views)
        a = case.d["mult"][views].reshape(-1, 1).astype(np.float64)
        y = case.d["y"][views].reshape(-1, case.T).astype(np.float64)
        # A = P G with G the resolution model (the identity without one)
        G = lambda img: psf.blur(np.asarray(img, np.float64).reshape(case.shape), case.cfg)  # noqa: E731
        yb = a * projector.fwd(case.cfg, G(case.x_np), p1, p2) + case.d["r"][views].reshape(-1, case.T)
        c = a * a * y / yb ** 2
        ref = G(projector.back(case.cfg, c * projector.fwd(case.cfg, G(v_np), p1, p2), p1, p2)).ravel()
        scale = np.linalg.norm(G(projector.back(case.cfg, c * projector.fwd(case.cfg, G(np.abs(v_np)), p1, p2), p1,
                                                p2)))
        err = np.linalg.norm(hv.cpu().numpy() - ref) / scale
        _say(f"[{case.cfg['name']}] subset {subset} data HVP error {err:.2e}")
        assert err <= 1e-5
    # accumulate mode adds to the output
    base = hv.clone()
    pm.pet_subset_hvp(case.geom, -1, case.x, v, case.y, case.r, case.a, work, hv, accumulate=True)
    assert torch.allclose(hv, 2 * base, rtol=1e-5, atol=1e-6 * float(base.abs().max()))


def test_rdp_hvp_parity(case):
    pm = case.pm
    rng = np.random.default_rng(12)
    v_np = rng.standard_normal(case.shape).astype(np.float32)
    v = torch.from_numpy(v_np.ravel()).to(case.dev)
    beta, gamma, eps = 0.37, 2.0, 1e-3 * float(case.x_np.max())
    hv = torch.empty(case.geom.n_vox, device=case.dev)
    gdot = torch.zeros(1, dtype=torch.float64, device=case.dev)
    pm.pet_rdp_hvp(case.geom, case.x, None, case.w27, beta, gamma, eps, v, hv, gdot_out=gdot)
    x64 = case.x_np.astype(np.float64)
    ref = beta * rdp.hvp(x64, v_np, case.w, gamma, eps)
    h = rdp.hessdiag(x64, case.w, gamma, eps)
    av = np.abs(v_np).astype(np.float64)
    scale = beta * np.linalg.norm(2 * h * av - rdp.hvp(x64, av, case.w, gamma, eps))
    err = np.linalg.norm(hv.cpu().numpy().reshape(case.shape) - ref) / scale
    _say(f"[{case.cfg['name']}] prior HVP error {err:.2e}")
    assert err <= 1e-5
    g = rdp.grad(x64, case.w, gamma, eps)
    assert float(gdot.cpu()) == pytest.approx(float(np.sum(g * v_np)), rel=1e-5,
                                              abs=1e-5 * float(np.sum(np.abs(g * v_np))))


def test_precond_vjp_parity(case):
    pm = case.pm
    rng = np.random.default_rng(13)
    Dbar_np = rng.standard_normal(case.shape).astype(np.float32)
    sens = torch.empty(case.geom.n_vox, device=case.dev)
    pm.pet_back(case.geom, -1, None, case.a, sens)
    beta, gamma, eps, alpha, delta = 0.25, 2.0, 1e-3 * float(case.x_np.max()), 1.0, 1e-3 * float(case.x_np.max())
    xbar = torch.zeros(case.geom.n_vox, device=case.dev)
    bb = torch.zeros(1, dtype=torch.float64, device=case.dev)
    pm.pet_precond_vjp(case.geom, case.x, sens, None, case.w27, beta, gamma, eps, alpha, delta,
                       torch.from_numpy(Dbar_np.ravel()).to(case.dev), xbar, bb)
    xt = torch.tensor(case.x_np.astype(np.float64), requires_grad=True)
    bt = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    st = torch.from_numpy(sens.cpu().numpy().astype(np.float64).reshape(case.shape))
    D = unrolled.preconditioner(xt, st, bt, case.w, gamma, eps, alpha, delta)
    (D * torch.from_numpy(Dbar_np.astype(np.float64))).sum().backward()
    err = _rel(xbar.cpu().numpy().reshape(case.shape), xt.grad.numpy())
    _say(f"[{case.cfg['name']}] preconditioner VJP error {err:.2e}, dbeta {float(bb.cpu()):.6e} vs {float(bt.grad):.6e}")
    assert err <= 1e-4
    assert float(bb.cpu()) == pytest.approx(float(bt.grad), rel=1e-4)


def _unrolled_both(c, n_epochs, x0_np, log_beta, target, eps, delta):
    """GPU and oracle (loss, dL/dx0, dL/dlog beta, final image)."""
    pm = c.pm
    n = c.cfg["n_subsets"]
    orders = data.subset_orders(c.cfg, n_epochs)
    taus = [[1.0 / (1.0 + 0.02 * (e * n + j) / n) for j in range(n)] for e in range(n_epochs)]
    upd_set = set(recon.pc_update_iters(n))
    upd = [[(e * n + j) in upd_set for j in range(n)] for e in range(n_epochs)]
    sens = torch.empty(c.geom.n_vox, device=c.dev)
    pm.pet_back(c.geom, -1, None, c.a, sens)
    prob_g = pm.UnrolledProblem(c.geom, c.y, c.r, c.a, sens, gamma=2.0, eps=eps, alpha=1.0, delta=delta,
                                orders=orders, taus=taus, updates=upd)
    x0 = torch.from_numpy(x0_np.ravel().astype(np.float32)).to(c.dev).requires_grad_(True)
    lb = torch.tensor(log_beta, dtype=torch.float64, device=c.dev, requires_grad=True)
    xf = pm.unrolled_svrg(x0, lb, prob_g)
    tgt = torch.from_numpy(target.ravel().astype(np.float32)).to(c.dev)
    L = ((xf.double() - tgt.double()) ** 2).sum()
    L.backward()
    gpu = (float(L.detach()), x0.grad.cpu().numpy().reshape(c.shape).astype(np.float64), float(lb.grad),
           xf.detach().cpu().numpy().reshape(c.shape))
    prob = recon.Problem(c.cfg, c.d["y"], c.d["r"], c.d["mult"], beta=float(np.exp(log_beta)), gamma=2.0, eps=eps,
                         alpha=1.0, delta=delta)
    orc = unrolled.loss_and_grads(prob, x0_np.astype(np.float64), log_beta, target.astype(np.float64), n_epochs,
                                  orders, taus, upd_set)
    return gpu, orc, (prob, orders, taus, upd_set)


def test_unrolled_gradient_parity(case):
    x0 = case.x_np
    eps = delta = 1e-3 * float(x0.max())
    log_beta = float(np.log(configs.beta_value(case.cfg) * 50.0))
    gpu, orc, _ = _unrolled_both(case, 3, x0, log_beta, case.d["x_true"], eps, delta)
    e_img = _rel(gpu[3], orc[3])
    e_gx = _rel(gpu[1], orc[1])
    _say(f"[{case.cfg['name']}] 3 epochs: image {e_img:.2e}, loss {gpu[0]:.6e} vs {orc[0]:.6e}, dL/dx0 {e_gx:.2e}, "
         f"dL/dlogbeta {gpu[2]:.6e} vs {orc[2]:.6e}")
    assert e_img <= 1e-4
    assert gpu[0] == pytest.approx(orc[0], rel=1e-4)
    assert e_gx <= 1e-4
    assert gpu[2] == pytest.approx(orc[2], rel=1e-4, abs=1e-4 * float(np.linalg.norm(orc[1]) * np.linalg.norm(x0)))


@pytest.mark.timeout(900)
def test_c3_unrolled_gradient_vs_oracle_and_finite_differences():
    """Differentiable configuration: 96x96x32 image, 120 views x 180 radial x
    268 planes, 8 subsets, 10 unrolled epochs from the one-epoch OSEM image,
    L = ||x_10 - x_true||^2.  GPU gradients against the FP64 oracle's autograd
    gradients (relative 1e-4) and against central finite differences of the
    FP64 oracle's forward pass (relative 1e-3) for d/dlog(beta) and three
    seeded directional derivatives in x0.

    The reconstruction clips about 60% of the voxels to 0, so the loss is only
    piecewise smooth in x0: one-sided difference quotients along a random
    direction disagree by 1e-2 at steps of 1e-3 ||x0|| and still by 1e-3 at
    1e-7 ||x0||.  The differences are therefore taken on the smooth piece of the
    base run, with the clip decisions (u > 0) of its 80 iterations held fixed;
    its derivative at the base point is the derivative autograd and the GPU
    compute.  Steps: 1e-4 in log(beta), 1e-5 ||x0|| / ||v|| in x0."""
    c = Case("c3_diff")
    n = c.cfg["n_subsets"]
    _say("[c3] OSEM initial image on the GPU")
    x0 = torch.ones(c.geom.n_vox, device=c.dev)
    xmax = torch.zeros(1, device=c.dev)
    c.pm.pet_osem_epoch(c.geom, x0, c.y, c.r, c.a, list(range(n)), xmax)
    x0_np = x0.cpu().numpy().reshape(c.shape)
    eps = delta = 1e-3 * float(xmax.cpu())
    log_beta = float(np.log(configs.beta_value(c.cfg)))
    E = c.cfg["epochs"]
    _say(f"[c3] GPU and oracle gradients over {E} epochs")
    gpu, orc, (prob, orders, taus, upd) = _unrolled_both(c, E, x0_np, log_beta, c.d["x_true"], eps, delta)
    e_img = _rel(gpu[3], orc[3])
    e_gx = _rel(gpu[1], orc[1])
    _say(f"[c3] image {e_img:.2e}; loss {gpu[0]:.8e} vs {orc[0]:.8e}; dL/dx0 {e_gx:.2e}; "
         f"dL/dlogbeta {gpu[2]:.6e} vs {orc[2]:.6e}")
    assert e_img <= 1e-4
    assert e_gx <= 1e-4
    assert gpu[2] == pytest.approx(orc[2], rel=1e-4)
    tgt = c.d["x_true"].astype(np.float64)
    x0d = x0_np.astype(np.float64)
    masks = []
    L0 = unrolled.loss(prob, x0d, log_beta, tgt, E, orders, taus, upd, record=masks)
    assert L0 == pytest.approx(orc[0], rel=1e-12)

    def Lf(x, lb):
        return unrolled.loss(prob, x, lb, tgt, E, orders, taus, upd, clip_masks=masks)

    h = 1e-4
    fd_b = (Lf(x0d, log_beta + h) - Lf(x0d, log_beta - h)) / (2 * h)
    _say(f"[c3] dL/dlogbeta: finite difference {fd_b:.6e}, GPU {gpu[2]:.6e}, oracle {orc[2]:.6e}")
    assert gpu[2] == pytest.approx(fd_b, rel=1e-3)
    assert orc[2] == pytest.approx(fd_b, rel=1e-3)
    rng = np.random.default_rng(2024)
    for trial in range(3):
        v = rng.standard_normal(c.shape)
        t = 1e-5 * np.linalg.norm(x0d) / np.linalg.norm(v)
        fd = (Lf(x0d + t * v, log_beta) - Lf(x0d - t * v, log_beta)) / (2 * t)
        dg, do = float(np.sum(gpu[1] * v)), float(np.sum(orc[1] * v))
        _say(f"[c3] direction {trial}: finite difference {fd:.6e}, GPU {dg:.6e}, oracle {do:.6e}")
        assert dg == pytest.approx(fd, rel=1e-3)
        assert do == pytest.approx(fd, rel=1e-3)
