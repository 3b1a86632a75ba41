"""GPU parity at the edges of the method and of the geometry, through the C ABI
against the FP64 oracle:

* the largest TOF bin count a geometry may have (32 bins, two bin blocks of the
  line kernel): forward projection and fused subset gradient;
* zero counts (y = 0): the data gradient is then the subset sensitivity
  A_i^T a and the Poisson deviance the sum of the means;
* a zero image (x = 0): the mean data are the additive terms alone;
* one subset (n = 1, every iteration a snapshot) and one view per subset
  (n = number of views), with subsets drawn with replacement: SVRG epochs.

Tolerances as in the other parity tests: cancellation-aware 1e-5 for
gradients, relative L2 1e-5 for projections, 1e-4 for reconstructions.
"""

import numpy as np
import pytest
import torch

from oracle import poisson, recon
from synth import configs, data

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


class Setup:
    def __init__(self, cfg):
        import paper_2506_04976_amd as pm
        self.pm = pm
        self.cfg = cfg
        self.d = data.make_dataset(cfg)
        self.dev = torch.device("cuda:0")
        self.geom = pm.Geometry(cfg)
        self.y = torch.from_numpy(self.d["y"].ravel()).to(self.dev)
        self.r = torch.from_numpy(self.d["r"].ravel()).to(self.dev)
        self.a = torch.from_numpy(self.d["mult"].ravel()).to(self.dev)
        rng = np.random.default_rng(17)
        self.x_np = (self.d["x_true"] * rng.uniform(0.8, 1.2, self.d["x_true"].shape) +
                     0.05 * self.d["x_true"].max()).astype(np.float32)
        self.x = torch.from_numpy(self.x_np.ravel()).to(self.dev)

    def problem(self, y=None, **kw):
        return recon.Problem(self.cfg, self.d["y"] if y is None else y, self.d["r"], self.d["mult"],
                             beta=kw.get("beta", 1e-3), gamma=2.0, eps=kw.get("eps", 1e-3), alpha=1.0,
                             delta=kw.get("delta", 1e-3))


def _grad_check(s, prob, subset, x_t, x_np, y_t):
    g = torch.empty(s.geom.n_vox, device=s.dev)
    kl = torch.zeros(1, dtype=torch.float64, device=s.dev)
    s.pm.pet_subset_grad(s.geom, subset, x_t, y_t, s.r, s.a, g, kl)
    xo = x_np.astype(np.float64)
    ref = prob.data_grad(xo, subset).ravel()
    yb = prob.ybar(xo, subset)
    scale = np.linalg.norm(prob.back(prob.a[subset] * (1 + prob.y[subset] / yb), subset))
    err = np.linalg.norm(g.cpu().double().numpy() - ref) / scale
    kl_ref = float(np.sum(poisson.kl(yb, prob.y[subset])))
    return err, float(kl.cpu()), kl_ref, g


def test_most_tof_bins():
    cfg = configs.get("mini_tof", n_tof=32, tof_bin=4.0, tof_sigma=3.0)
    s = Setup(cfg)
    prob = s.problem()
    subset = 1
    out = torch.empty(s.geom.n_bins, device=s.dev)
    s.pm.pet_fwd(s.geom, subset, s.x, s.a, s.r, out)
    views = configs.subset_views(cfg, subset)
    got = out.view(cfg["n_views"], -1)[views].cpu().double().numpy().reshape(-1, 32)
    ref = prob.ybar(s.x_np.astype(np.float64), subset)
    err_f = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    err_g, kl, kl_ref, _ = _grad_check(s, prob, subset, s.x, s.x_np, s.y)
    _say(f"[32 TOF bins] forward {err_f:.2e}, fused gradient {err_g:.2e}")
    assert err_f <= 1e-5
    assert err_g <= 1e-5
    assert kl == pytest.approx(kl_ref, rel=1e-5)
    s.geom.close()


@pytest.mark.parametrize("name", ["mini_tof", "mini_nontof"])
def test_zero_counts(name):
    s = Setup(configs.get(name))
    y0 = np.zeros_like(s.d["y"])
    prob = s.problem(y=y0)
    y0_t = torch.zeros_like(s.y)
    subset = 0
    err, kl, kl_ref, g = _grad_check(s, prob, subset, s.x, s.x_np, y0_t)
    # with y = 0 the gradient is the subset sensitivity A_i^T a
    sens = torch.empty(s.geom.n_vox, device=s.dev)
    s.pm.pet_back(s.geom, subset, None, s.a, sens)
    rel = float(torch.linalg.norm(g - sens) / torch.linalg.norm(sens))
    _say(f"[{name} y = 0] gradient {err:.2e}, against A_i^T a {rel:.2e}")
    assert err <= 1e-5
    assert rel <= 1e-5
    assert kl == pytest.approx(kl_ref, rel=1e-5)
    s.geom.close()


@pytest.mark.parametrize("name", ["mini_tof", "mini_2d"])
def test_zero_image(name):
    s = Setup(configs.get(name))
    prob = s.problem()
    x0_np = np.zeros_like(s.x_np)
    x0 = torch.zeros_like(s.x)
    subset = 0
    out = torch.empty(s.geom.n_bins, device=s.dev)
    s.pm.pet_fwd(s.geom, subset, x0, s.a, s.r, out)
    views = configs.subset_views(s.cfg, subset)
    got = out.view(s.cfg["n_views"], -1)[views].cpu().double().numpy()
    assert np.array_equal(got, s.d["r"][views].reshape(len(views), -1).astype(np.float64))
    err, kl, kl_ref, _ = _grad_check(s, prob, subset, x0, x0_np, s.y)
    _say(f"[{name} x = 0] fused gradient {err:.2e}")
    assert err <= 1e-5
    assert kl == pytest.approx(kl_ref, rel=1e-5)
    s.geom.close()


def _svrg_pair(cfg, seqs, epochs):
    s = Setup(cfg)
    pm, n = s.pm, cfg["n_subsets"]
    beta = configs.beta_value(cfg)
    x = torch.ones(s.geom.n_vox, device=s.dev)
    xmax = torch.zeros(1, device=s.dev)
    pm.pet_osem_epoch(s.geom, x, s.y, s.r, s.a, list(range(n)), xmax)
    mx = float(xmax.cpu())
    sens = torch.empty(s.geom.n_vox, device=s.dev)
    pm.pet_back(s.geom, -1, None, s.a, sens)
    st = pm.SvrgStateBuffers(s.geom, s.y, s.r, s.a, sens, beta=beta, gamma=2.0, eps=1e-3 * mx, alpha=1.0,
                             delta=1e-3 * mx)
    tau = recon.stepsize_vanishing(1.0, 0.02, n)
    upd = recon.pc_update_iters(n)
    for e in range(epochs):
        ks = [e * n + j for j in range(n)]
        pm.pet_svrg_epoch(s.geom, st, x, seqs[e], [tau(k) for k in ks], [k in upd for k in ks])
    x0 = recon.osem_epoch(s.problem(), np.ones((cfg["nz"], cfg["ny"], cfg["nx"])))
    m0 = float(x0.max())
    prob = recon.Problem(cfg, s.d["y"], s.d["r"], s.d["mult"], beta=beta, gamma=2.0, eps=1e-3 * m0, alpha=1.0,
                         delta=1e-3 * m0)
    x_orc = recon.svrg(prob, x0, epochs, lambda k: int(seqs[k // n][k % n]), tau, upd).ravel()
    err = np.linalg.norm(x.cpu().double().numpy() - x_orc) / np.linalg.norm(x_orc)
    s.geom.close()
    return err


def test_one_subset():
    cfg = configs.get("mini_tof", n_subsets=1)
    err = _svrg_pair(cfg, [[0]] * 4, 4)
    _say(f"[n = 1] 4 epochs: relative L2 {err:.2e}")
    assert err <= 1e-4


def test_one_view_per_subset_with_replacement():
    cfg = configs.get("mini_2d", n_subsets=12)
    rng = np.random.default_rng(5)
    seqs = [rng.integers(0, 12, 12).tolist() for _ in range(3)]
    err = _svrg_pair(cfg, seqs, 3)
    _say(f"[n = views, with replacement] 3 epochs: relative L2 {err:.2e}")
    assert err <= 1e-4
