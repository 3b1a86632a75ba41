"""GPU parity: every entry point of the HIP library through the C ABI against
the FP64 oracle on the same seeded inputs, element by element.

Tolerances (single precision arithmetic on the GPU):
* projections of nonnegative images and backprojections of nonnegative
  sinograms: relative L2 error <= 1e-5 (max-abs / max <= 1e-4);
* gradients with cancelling summands: ||g_gpu - g_orc|| <= 1e-5 ||sum of |summands|||
  (data term: ||P^T(a) + P^T(a y / ybar)||; prior: the norm of the sum of the
  absolute neighbour terms);
* images after a fixed number of iterations: relative L2 <= 1e-4.
Sizes span several workgroups with ragged image dimensions (21x19x9, 23x17,
64x64) and uneven subsets.
"""

import numpy as np
import pytest
import torch

from oracle import projector, psf, rdp, recon, schedules
from synth import configs, data

pytestmark = pytest.mark.gpu

CASES = ["mini_tof", "mini_nontof", "mini_2d", "c0_2d", "mini_tof_psf", "mini_2d_psf", "mini_tof_many",
         "mini_tof_seg40"]


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


class Case:
    def __init__(self, name):
        import paper_2506_04976_amd as pm
        self.pm = pm
        self.cfg = configs.get(name)
        self.d = data.make_dataset(self.cfg)
        self.geom = pm.Geometry(self.cfg)
        dev = torch.device("cuda:0")
        self.dev = dev
        rng = np.random.default_rng(42)
        self.x_np = (self.d["x_true"] * rng.uniform(0.7, 1.3, self.d["x_true"].shape) +
                     0.05 * self.d["x_true"].max()).astype(np.float32)
        self.x = torch.from_numpy(self.x_np.ravel()).to(dev)
        self.y = torch.from_numpy(self.d["y"].ravel()).to(dev)
        self.r = torch.from_numpy(self.d["r"].ravel()).to(dev)
        self.a = torch.from_numpy(self.d["mult"].ravel()).to(dev)
        self.T = self.cfg["n_tof"]
        self.shape4 = (self.cfg["n_views"], self.cfg["n_rad"], configs.n_planes(self.cfg), self.T)
        self.prob = recon.Problem(self.cfg, self.d["y"], self.d["r"], self.d["mult"], beta=configs.beta_value(self.cfg),
                                  gamma=2.0, eps=1e-3 * float(self.x_np.max()), alpha=1.0,
                                  delta=1e-3 * float(self.x_np.max()))

    def views(self, subset):
        return list(range(self.cfg["n_views"])) if subset < 0 else configs.subset_views(self.cfg, subset)


@pytest.fixture(scope="module", params=CASES)
def case(request):
    print(f"\n[gpu case {request.param}]", flush=True)
    return Case(request.param)


def test_fwd_parity(case):
    pm = case.pm
    for subset in (-1, 0, case.cfg["n_subsets"] - 1):
        out = torch.full((case.geom.n_bins,), float("nan"), device=case.dev)
        pm.pet_fwd(case.geom, subset, case.x, case.a, case.r, out)
        got = out.cpu().numpy().reshape(case.shape4)
        views = case.views(subset)
        p1, p2 = projector.view_lors(case.cfg, views)
        ref = (projector.fwd(case.cfg, psf.blur(case.x_np, case.cfg), p1, p2) * case.d["mult"][views].reshape(-1, 1) +
               case.d["r"][views].reshape(-1, case.T)).reshape(len(views), *case.shape4[1:])
        g = got[views]
        assert _rel(g, ref) <= 1e-5
        assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))
        others = sorted(set(range(case.cfg["n_views"])) - set(views))
        assert np.all(np.isnan(got[others])), "bins of other subsets must stay untouched"
    # plain projection (mult, add = NULL)
    out = torch.empty(case.geom.n_bins, device=case.dev)
    pm.pet_fwd(case.geom, -1, case.x, None, None, out)
    p1, p2 = projector.view_lors(case.cfg, case.views(-1))
    ref = projector.fwd(case.cfg, psf.blur(case.x_np, case.cfg), p1, p2).ravel()
    assert _rel(out.cpu().numpy(), ref) <= 1e-5


def test_back_parity(case):
    pm = case.pm
    rng = np.random.default_rng(7)
    sino = rng.uniform(0, 2, case.geom.n_bins).astype(np.float32)
    s_t = torch.from_numpy(sino).to(case.dev)
    for subset in (-1, 1):
        out = torch.empty(case.geom.n_vox, device=case.dev)
        pm.pet_back(case.geom, subset, s_t, case.a, out)
        views = case.views(subset)
        p1, p2 = projector.view_lors(case.cfg, views)
        s_sub = sino.reshape(case.shape4)[views].reshape(-1, case.T) * case.d["mult"][views].reshape(-1, 1)
        ref = psf.blur(projector.back(case.cfg, s_sub, p1, p2), case.cfg).ravel()
        assert _rel(out.cpu().numpy(), ref) <= 1e-5
    # sensitivity (sino = NULL) and accumulate
    sens = torch.empty(case.geom.n_vox, device=case.dev)
    pm.pet_back(case.geom, -1, None, case.a, sens)
    assert _rel(sens.cpu().numpy(), case.prob.sens().ravel()) <= 1e-5
    acc = sens.clone()
    pm.pet_back(case.geom, -1, None, case.a, acc, accumulate=True)
    assert _rel(acc.cpu().numpy(), 2 * case.prob.sens().ravel()) <= 1e-5


def test_back_sensitivity_fold(case):
    # sino = NULL on a TOF geometry: one walk per LOR with the bins' weights
    # summed per sample (they telescope), against the per-bin backprojection of
    # an all-ones sinogram, per subset and over all views
    if case.T == 1:
        pytest.skip("non-TOF: sino = NULL takes the same kernel")
    pm = case.pm
    ones = torch.ones(case.geom.n_bins, device=case.dev)
    for subset in (-1, 0, case.cfg["n_subsets"] - 1):
        fold = torch.full((case.geom.n_vox,), float("nan"), device=case.dev)
        pm.pet_back(case.geom, subset, None, case.a, fold)
        per_bin = torch.empty(case.geom.n_vox, device=case.dev)
        pm.pet_back(case.geom, subset, ones, case.a, per_bin)
        assert _rel(fold.cpu().numpy(), per_bin.cpu().double().numpy()) <= 2e-6
        if subset >= 0:
            ref = case.prob.sens_subset(subset).ravel()
            assert _rel(fold.cpu().numpy(), ref) <= 1e-5


def test_back_gather_parity(case):
    # the cell-driven gather adjoint gives the scatter's (sample, weight) pairs:
    # against the oracle (relative L2 <= 1e-5) and against the scatter
    pm = case.pm
    rng = np.random.default_rng(17)
    sino = rng.uniform(0, 2, case.geom.n_bins).astype(np.float32)
    s_t = torch.from_numpy(sino).to(case.dev)
    for subset in (-1, 2 % case.cfg["n_subsets"]):
        out = torch.full((case.geom.n_vox,), float("nan"), device=case.dev)
        pm.pet_back(case.geom, subset, s_t, case.a, out, algo=pm.PET_BACK_GATHER)
        sc = torch.empty(case.geom.n_vox, device=case.dev)
        pm.pet_back(case.geom, subset, s_t, case.a, sc, algo=pm.PET_BACK_SCATTER)
        views = case.views(subset)
        p1, p2 = projector.view_lors(case.cfg, views)
        s_sub = sino.reshape(case.shape4)[views].reshape(-1, case.T) * case.d["mult"][views].reshape(-1, 1)
        ref = psf.blur(projector.back(case.cfg, s_sub, p1, p2), case.cfg).ravel()
        assert _rel(out.cpu().numpy(), ref) <= 1e-5
        assert _rel(out.cpu().numpy(), sc.cpu().double().numpy()) <= 2e-6
    sens = torch.empty(case.geom.n_vox, device=case.dev)
    pm.pet_back(case.geom, -1, None, case.a, sens, algo=pm.PET_BACK_GATHER)
    assert _rel(sens.cpu().numpy(), case.prob.sens().ravel()) <= 1e-5
    # accumulate = 1 adds
    acc = sens.clone()
    pm.pet_back(case.geom, -1, None, case.a, acc, accumulate=True, algo=pm.PET_BACK_GATHER)
    assert _rel(acc.cpu().numpy(), 2 * case.prob.sens().ravel()) <= 1e-5


def test_gpu_adjoint_identity(case):
    pm = case.pm
    rng = np.random.default_rng(3)
    xv = torch.from_numpy(rng.uniform(0, 1, case.geom.n_vox).astype(np.float32)).to(case.dev)
    yv = torch.from_numpy(rng.uniform(0, 1, case.geom.n_bins).astype(np.float32)).to(case.dev)
    px = torch.empty(case.geom.n_bins, device=case.dev)
    pm.pet_fwd(case.geom, -1, xv, None, None, px)
    pty = torch.empty(case.geom.n_vox, device=case.dev)
    pm.pet_back(case.geom, -1, yv, None, pty)
    lhs = float(torch.dot(px.double(), yv.double()))
    rhs = float(torch.dot(xv.double(), pty.double()))
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


def test_subset_grad_and_kl_parity(case):
    pm = case.pm
    n = case.cfg["n_subsets"]
    for subset in range(n):
        g = torch.empty(case.geom.n_vox, device=case.dev)
        kl = torch.zeros(1, dtype=torch.float64, device=case.dev)
        pm.pet_subset_grad(case.geom, subset, case.x, case.y, case.r, case.a, g, kl)
        xo = case.x_np.astype(np.float64)
        ref = case.prob.data_grad(xo, subset).ravel()
        yb = case.prob.ybar(xo, subset)
        scale = np.linalg.norm(case.prob.back(case.prob.a[subset] * (1 + case.prob.y[subset] / yb), subset))
        err = np.linalg.norm(g.cpu().numpy() - ref) / scale
        assert err <= 1e-5, f"subset {subset}: {err:.3e}"
        from oracle import poisson
        kl_ref = float(np.sum(poisson.kl(yb, case.prob.y[subset])))
        assert float(kl.cpu()) == pytest.approx(kl_ref, rel=1e-5)


def test_count_dtypes_agree(case):
    # the same counts stored as uint8 (when they fit), uint16 and float32 give
    # the same fused gradient and KL (the kernels convert every count to FP32)
    pm = case.pm
    y_np = case.d["y"].ravel()
    ys = {"u16": torch.from_numpy(y_np.astype(np.uint16)).to(case.dev),
          "f32": torch.from_numpy(y_np.astype(np.float32)).to(case.dev)}
    if y_np.max() <= 255:
        ys["u8"] = torch.from_numpy(y_np.astype(np.uint8)).to(case.dev)
    subset = case.cfg["n_subsets"] - 1
    out = {}
    for name, y in ys.items():
        g = torch.empty(case.geom.n_vox, device=case.dev)
        kl = torch.zeros(1, dtype=torch.float64, device=case.dev)
        pm.pet_subset_grad(case.geom, subset, case.x, y, case.r, case.a, g, kl)
        out[name] = (g.cpu().double().numpy(), float(kl.cpu()))
    g0, kl0 = out["f32"]
    for name, (g, kl) in out.items():
        assert np.linalg.norm(g - g0) <= 1e-6 * np.linalg.norm(g0), name
        assert kl == pytest.approx(kl0, rel=1e-9), name


def test_rdp_parity(case):
    pm = case.pm
    w27 = pm.rdp_weights27(case.cfg["vx"], case.cfg["vy"], case.cfg["vz"])
    beta, gamma, eps = 0.37, 2.0, 1e-3 * float(case.x_np.max())
    kappa_np = np.random.default_rng(1).uniform(0.5, 1.5, case.x_np.shape).astype(np.float32)
    for kap in (None, kappa_np):
        kt = None if kap is None else torch.from_numpy(kap.ravel()).to(case.dev)
        g = torch.empty(case.geom.n_vox, device=case.dev)
        h = torch.empty(case.geom.n_vox, device=case.dev)
        val = torch.zeros(1, dtype=torch.float64, device=case.dev)
        pm.pet_rdp_grad_hessdiag(case.geom, case.x, kt, w27, beta, gamma, eps, g, h, val)
        w = rdp.default_weights(case.cfg["vx"], case.cfg["vy"], case.cfg["vz"], case.cfg["nz"])
        xo = case.x_np.astype(np.float64)
        ko = None if kap is None else kap.astype(np.float64)
        gref = beta * rdp.grad(xo, w, gamma, eps, ko)
        # cancellation-aware scale: sum over neighbours of |terms|
        absg = np.zeros_like(xo)
        kk = np.ones_like(xo) if ko is None else ko
        for off, wij in w.items():
            I, J = rdp._pairs(xo.shape, off)
            dd = xo[I] - xo[J]
            phi = xo[I] + xo[J] + gamma * np.abs(dd) + eps
            absg[I] += np.abs(wij * kk[I] * kk[J] * dd * (2 * phi - (dd + gamma * np.abs(dd))) / phi ** 2)
        assert np.linalg.norm(g.cpu().numpy() - gref.ravel()) <= 1e-5 * np.linalg.norm(beta * absg)
        href = beta * rdp.hessdiag(xo, w, gamma, eps, ko)
        assert _rel(h.cpu().numpy(), href.ravel()) <= 1e-5
        assert float(val.cpu()) == pytest.approx(beta * rdp.value(xo, w, gamma, eps, ko), rel=1e-5)


def test_precond_parity(case):
    pm = case.pm
    sens = torch.empty(case.geom.n_vox, device=case.dev)
    pm.pet_back(case.geom, -1, None, case.a, sens)
    hess = torch.from_numpy(np.random.default_rng(4).uniform(0, 3, case.geom.n_vox).astype(np.float32)).to(case.dev)
    hess[:5] = 0
    D = torch.empty(case.geom.n_vox, device=case.dev)
    pm.pet_precond(case.geom, case.x, sens, hess, 1.3, 0.02, D)
    ref = recon.precond_harmonic(case.x_np.ravel(), sens.cpu().double().numpy(), hess.cpu().double().numpy(), 1.3, 0.02)
    assert _rel(D.cpu().numpy(), ref) <= 1e-6


def test_osem_and_objective_parity(case):
    pm = case.pm
    n = case.cfg["n_subsets"]
    order = list(range(n))[::-1]
    x = torch.ones(case.geom.n_vox, device=case.dev)
    xmax = torch.zeros(1, device=case.dev)
    pm.pet_osem_epoch(case.geom, x, case.y, case.r, case.a, order, xmax)
    ref = recon.osem_epoch(case.prob, np.ones(case.prob.shape), order).ravel()
    assert _rel(x.cpu().numpy(), ref) <= 1e-5
    assert float(xmax.cpu()) == pytest.approx(ref.max(), rel=1e-5)
    w27 = pm.rdp_weights27(case.cfg["vx"], case.cfg["vy"], case.cfg["vz"])
    out = torch.zeros(1, dtype=torch.float64, device=case.dev)
    pm.pet_objective(case.geom, case.x, case.y, case.r, case.a, None, w27, case.prob.beta, case.prob.gamma,
                     case.prob.eps, out)
    assert float(out.cpu()) == pytest.approx(case.prob.objective(case.x_np.astype(np.float64)), rel=1e-5)


def _svrg_pair(case, epochs, algo="svrg"):
    """Run OSEM init + `epochs` epochs of SVRG, SAGA or SGD on the GPU and in
    the oracle."""
    pm = case.pm
    cfg, n = case.cfg, case.cfg["n_subsets"]
    beta = configs.beta_value(cfg)
    # GPU
    x = torch.ones(case.geom.n_vox, device=case.dev)
    xmax = torch.zeros(1, device=case.dev)
    pm.pet_osem_epoch(case.geom, x, case.y, case.r, case.a, list(range(n)), xmax)
    mx = float(xmax.cpu())
    sens = torch.empty(case.geom.n_vox, device=case.dev)
    pm.pet_back(case.geom, -1, None, case.a, sens)
    st = pm.SvrgStateBuffers(case.geom, case.y, case.r, case.a, sens, beta=beta, gamma=2.0, eps=1e-3 * mx,
                             alpha=1.0, delta=1e-3 * mx)
    orders = data.subset_orders(cfg, epochs)
    tau_rule = recon.stepsize_vanishing(0.3, 0.5, n) if algo == "sgd" else recon.stepsize_vanishing(1.0, 0.02, n)
    upd = recon.pc_update_iters(n)
    epoch_fn = {"svrg": pm.pet_svrg_epoch, "saga": pm.pet_saga_epoch, "sgd": pm.pet_sgd_epoch}[algo]
    for e in range(epochs):
        ks = [e * n + j for j in range(n)]
        epoch_fn(case.geom, st, x, orders[e], [tau_rule(k) for k in ks], [k in upd for k in ks])
    x_gpu = x.cpu().double().numpy()
    # oracle
    x0 = recon.osem_epoch(case.prob, np.ones(case.prob.shape))
    m0 = float(x0.max())
    prob = recon.Problem(cfg, case.d["y"], case.d["r"], case.d["mult"], beta=beta, gamma=2.0, eps=1e-3 * m0,
                         alpha=1.0, delta=1e-3 * m0)
    x_orc = getattr(recon, algo)(prob, x0, epochs, recon.order_rule(orders), tau_rule, upd)
    return x_gpu, x_orc.ravel()


def test_svrg_reconstruction_parity(case):
    epochs = case.cfg["epochs"]
    x_gpu, x_orc = _svrg_pair(case, epochs)
    err = _rel(x_gpu, x_orc)
    print(f"[{case.cfg['name']}] {epochs} epochs: relative L2 {err:.2e}", flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("algo", ["saga", "sgd"])
def test_saga_sgd_reconstruction_parity(case, algo):
    epochs = case.cfg["epochs"]
    x_gpu, x_orc = _svrg_pair(case, epochs, algo)
    err = _rel(x_gpu, x_orc)
    print(f"[{case.cfg['name']}] {algo} {epochs} epochs: relative L2 {err:.2e}", flush=True)
    assert err <= 1e-4


def _gpu_start(case, bb=False, gnorm=False):
    pm = case.pm
    cfg, n = case.cfg, case.cfg["n_subsets"]
    beta = configs.beta_value(cfg)
    x = torch.ones(case.geom.n_vox, device=case.dev)
    xmax = torch.zeros(1, device=case.dev)
    pm.pet_osem_epoch(case.geom, x, case.y, case.r, case.a, list(range(n)), xmax)
    mx = float(xmax.cpu())
    sens = torch.empty(case.geom.n_vox, device=case.dev)
    pm.pet_back(case.geom, -1, None, case.a, sens)
    st = pm.SvrgStateBuffers(case.geom, case.y, case.r, case.a, sens, beta=beta, gamma=2.0, eps=1e-3 * mx,
                             alpha=1.0, delta=1e-3 * mx, bb=bb, gnorm=gnorm)
    x0 = recon.osem_epoch(case.prob, np.ones(case.prob.shape))
    m0 = float(x0.max())
    prob = recon.Problem(cfg, case.d["y"], case.d["r"], case.d["mult"], beta=beta, gamma=2.0, eps=1e-3 * m0,
                         alpha=1.0, delta=1e-3 * m0)
    return x, st, x0, prob


def test_alg2_bb_parity(case):
    # ALG2: preconditioner updates at the start of epochs 1, 2, 4, 6; short BB
    # step at the end of epochs 2 and 4 (snapshots), capped by the schedule
    pm = case.pm
    cfg, n = case.cfg, case.cfg["n_subsets"]
    epochs = 6
    x, st, x0, prob = _gpu_start(case, bb=True)
    orders = data.subset_orders(cfg, epochs)
    upd = {0, n, 3 * n, 5 * n}
    bb_it = {2 * n, 4 * n}
    cap = lambda k: schedules.alg2_cap(k, n)  # noqa: E731
    x_end = {}
    for e in range(epochs):
        ks = [e * n + j for j in range(n)]
        pm.pet_svrg_epoch(case.geom, st, x, orders[e], [cap(k) for k in ks], [k in upd for k in ks],
                          bb_update=[k in bb_it for k in ks])
        x_end[(e + 1) * n] = x.cpu().double().numpy().reshape(prob.shape)
    rec = []
    x_orc = recon.svrg(prob, x0, epochs, recon.order_rule(orders), cap, upd, bb_iters=bb_it, record=rec)
    bbs = [r for r in rec if r[0] == "bb"]
    assert [r[1] for r in bbs] == sorted(bb_it)
    bb_gpu = st.bb.cpu().numpy()
    assert bb_gpu[3] == len(bb_it)
    # the short BB step of the GPU's own snapshots (k = 2n, 4n) with the
    # preconditioner of its last update (k = 3n), in FP64
    xa, xb = x_end[2 * n], x_end[4 * n]
    D = recon.precond_harmonic(x_end[3 * n], prob.sens(), prob.prior_hessdiag(x_end[3 * n]), prob.alpha, prob.delta)
    p = xb - xa
    q = prob.full_grad(xb) - prob.full_grad(xa)
    tau_ref = float(np.sum(p * q) / np.sum(q * D * q))
    print(f"[{cfg['name']}] tau_bb gpu {bb_gpu[2]:.7g}, of the gpu snapshots {tau_ref:.7g}, "
          f"oracle run {bbs[-1][4]:.7g}", flush=True)
    assert bb_gpu[2] == pytest.approx(tau_ref, rel=1e-4)
    err = _rel(x.cpu().double().numpy(), x_orc.ravel())
    print(f"[{cfg['name']}] ALG2 {epochs} epochs: relative L2 {err:.2e}", flush=True)
    assert err <= 1e-4


def test_importance_sampling_parity(case):
    pm = case.pm
    cfg, n = case.cfg, case.cfg["n_subsets"]
    epochs = 4
    x, st, x0, prob = _gpu_start(case, gnorm=True)
    u = np.random.default_rng(11).random(epochs * n)
    rec = []
    x_orc = recon.svrg(prob, x0, epochs, None, recon.stepsize_vanishing(1.0, 0.02, n), recon.pc_update_iters(n),
                       importance_u=u, record=rec)
    draws = {r[1]: (r[2], r[3]) for r in rec if r[0] == "sample"}
    snaps = {r[1]: r[2] for r in rec if r[0] == "snapshot"}
    tau_rule = recon.stepsize_vanishing(1.0, 0.02, n)
    upd = recon.pc_update_iters(n)
    for e in range(epochs):
        ks = [e * n + j for j in range(n)]
        seq = [draws[k][0] if k in draws else 0 for k in ks]
        w = [draws[k][1] if k in draws else float(n) for k in ks]
        pm.pet_svrg_epoch(case.geom, st, x, seq, [tau_rule(k) for k in ks], [k in upd for k in ks], weight=w)
        if e * n in snaps:
            got = st.gnorm.cpu().numpy()
            ref = np.asarray(snaps[e * n])
            assert np.max(np.abs(got - ref) / ref) <= 1e-5
            # the GPU norms give the same draws, except for a uniform within
            # rounding of a boundary of the cumulative distribution
            pr = recon.importance_probabilities(list(got))
            c = np.cumsum(recon.importance_probabilities(list(ref)))
            for k in range(e * n + 1, min(e * n + 2 * n, epochs * n)):
                if np.min(np.abs(c - u[k])) > 1e-4:
                    assert recon.sample_inverse_cdf(pr, u[k]) == draws[k][0]
    err = _rel(x.cpu().double().numpy(), x_orc.ravel())
    print(f"[{cfg['name']}] importance-sampled SVRG {epochs} epochs: relative L2 {err:.2e}", flush=True)
    assert err <= 1e-4
