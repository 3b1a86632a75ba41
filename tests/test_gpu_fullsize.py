"""GPU parity at the full workload sizes, in the launch configuration the
benchmark uses (whole subsets of the 3D geometries).

* Forward projections of a subset: sampled LORs recomputed one by one by the
  FP64 oracle (relative L2 <= 1e-5 over the sample).
* Fused subset gradient: the multiplicative factors of every view but one are
  zeroed, so the GPU subset gradient equals the gradient of that one view, which
  the oracle computes in full (cancellation-aware error <= 1e-5).
* Whole-subset gradient (every view of one subset, the data's own factors),
  dense and zero-count-aware, against the oracle computed view by view.
* The 3D non-TOF image after OSEM + 2 SVRG epochs (dense and zero-count-aware)
  against a stored oracle image of the same schedule (relative L2 <= 1e-4).
* 3D image after 10 SVRG epochs on the small 3D geometry (96x96x32, 268 planes,
  8 subsets): relative L2 <= 1e-4 against the oracle.
* The GPU adjoint identity on a whole TOF subset.

The cases are the non-TOF and TOF brain-sized workloads and the paper's own
simulation geometry (17 rings, 25 TOF bins, 4 mm resolution model): with a
resolution model the references use A = P G.
"""

import numpy as np
import pytest
import torch

from oracle import poisson, projector, psf, recon
from synth import configs, data, scanner

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module", params=["c1_3d", "c2_tof", "c5_sim"])
def big(request):
    import paper_2506_04976_amd as pm
    name = request.param
    _say(f"\n[fullsize {name}] generating data")
    cfg = configs.get(name)
    d = data.make_dataset(cfg)
    dev = torch.device("cuda:0")
    geom = pm.Geometry(cfg)
    out = dict(pm=pm, cfg=cfg, d=d, geom=geom, dev=dev,
               y=torch.from_numpy(d["y"].reshape(-1)).to(dev),
               r=torch.from_numpy(d["r"].reshape(-1)).to(dev),
               a=torch.from_numpy(d["mult"].reshape(-1)).to(dev))
    rng = np.random.default_rng(5)
    x = d["x_true"] * rng.uniform(0.8, 1.2, d["x_true"].shape) + 0.05 * d["x_true"].max()
    out["x_np"] = x.astype(np.float32)
    out["x"] = torch.from_numpy(out["x_np"].ravel()).to(dev)
    # G x in FP64 (the image itself without a resolution model)
    out["gx"] = psf.blur(out["x_np"].astype(np.float64), cfg)
    yield out
    geom.close()


def test_fullsize_fwd_sampled(big):
    cfg, pm = big["cfg"], big["pm"]
    T = cfg["n_tof"]
    n_pl = configs.n_planes(cfg)
    subset = 3
    out = torch.full((big["geom"].n_bins,), float("nan"), device=big["dev"])
    pm.pet_fwd(big["geom"], subset, big["x"], big["a"], big["r"], out)
    got = out.view(cfg["n_views"], cfg["n_rad"], n_pl, T)
    views = configs.subset_views(cfg, subset)
    rng = np.random.default_rng(11)
    ns = 3000
    v = rng.choice(views, ns)
    k = rng.integers(0, cfg["n_rad"], ns)
    p = rng.integers(0, n_pl, ns)
    p1, p2 = scanner.lor_endpoints(cfg, v, k, p)
    ref = projector.fwd(cfg, big["gx"], p1, p2) * big["d"]["mult"][v, k, p][:, None] + big["d"]["r"][v, k, p]
    g = got[torch.from_numpy(v), torch.from_numpy(k), torch.from_numpy(p)].cpu().numpy()
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    _say(f"[{cfg['name']}] sampled fwd relative L2 {err:.2e}")
    assert err <= 1e-5
    # the other subsets' bins are untouched
    other = configs.subset_views(cfg, (subset + 1) % cfg["n_subsets"])[0]
    assert torch.isnan(got[other]).all()


def test_fullsize_subset_grad_one_view(big):
    cfg, pm, d = big["cfg"], big["pm"], big["d"]
    subset = 1
    view = configs.subset_views(cfg, subset)[2]
    mult = np.zeros_like(d["mult"])
    mult[view] = d["mult"][view]
    a1 = torch.from_numpy(mult.reshape(-1)).to(big["dev"])
    g = torch.empty(big["geom"].n_vox, device=big["dev"])
    kl = torch.zeros(1, dtype=torch.float64, device=big["dev"])
    pm.pet_subset_grad(big["geom"], subset, big["x"], big["y"], big["r"], a1, g, kl)
    g_gpu = g.cpu().double().numpy()
    T = cfg["n_tof"]
    p1, p2 = projector.view_lors(cfg, [view])
    a = d["mult"][view].reshape(-1, 1).astype(np.float64)
    r = d["r"][view].reshape(-1, T).astype(np.float64)
    y = d["y"][view].reshape(-1, T).astype(np.float64)
    yb = a * projector.fwd(cfg, big["gx"], p1, p2) + r
    ref = psf.blur(projector.back(cfg, a * (1.0 - y / yb), p1, p2), cfg).ravel()
    scale = np.linalg.norm(psf.blur(projector.back(cfg, a * (1.0 + y / yb), p1, p2), cfg))
    err = np.linalg.norm(g_gpu - ref) / scale
    _say(f"[{cfg['name']}] one-view fused gradient, cancellation-aware error {err:.2e}")
    assert err <= 1e-5
    # KL over the subset: the zeroed views contribute d(r, y), the kept view d(ybar, y)
    views = configs.subset_views(cfg, subset)
    kl_ref = float(np.sum(poisson.kl(yb, y)))
    for vv in views:
        if vv != view:
            kl_ref += float(np.sum(poisson.kl(d["r"][vv].astype(np.float64), d["y"][vv].astype(np.float64))))
    assert float(kl.cpu()) == pytest.approx(kl_ref, rel=1e-6)


def test_fullsize_whole_subset_gradient(big):
    # One whole subset (every view, the data's own mult): the dense fused
    # gradient and the zero-count-aware gradient against the FP64 oracle's
    # subset gradient, computed view by view (cancellation-aware <= 1e-5), and
    # the subset KL (relative 1e-6).
    cfg, pm, d, dev = big["cfg"], big["pm"], big["d"], big["dev"]
    subset = 2
    geom = big["geom"]
    g = torch.empty(geom.n_vox, device=dev)
    kl = torch.zeros(1, dtype=torch.float64, device=dev)
    pm.pet_subset_grad(geom, subset, big["x"], big["y"], big["r"], big["a"], g, kl)
    cnt = pm.Counts(geom, big["y"], big["r"], big["a"])
    sens = torch.empty(geom.n_vox, device=dev)
    pm.pet_back(geom, subset, None, big["a"], sens)
    gc = torch.empty(geom.n_vox, device=dev)
    klc = torch.zeros(1, dtype=torch.float64, device=dev)
    pm.pet_subset_grad_counts(geom, cnt, subset, big["x"], sens, gc, klc)
    g_gpu, gc_gpu = g.cpu().double().numpy(), gc.cpu().double().numpy()
    cnt.close()
    T = cfg["n_tof"]
    ref = np.zeros(geom.n_vox)
    absref = np.zeros(geom.n_vox)
    kl_ref = 0.0
    views = configs.subset_views(cfg, subset)
    for j, view in enumerate(views):
        p1, p2 = projector.view_lors(cfg, [view])
        a = d["mult"][view].reshape(-1, 1).astype(np.float64)
        r = d["r"][view].reshape(-1, T).astype(np.float64)
        y = d["y"][view].reshape(-1, T).astype(np.float64)
        yb = a * projector.fwd(cfg, big["gx"], p1, p2) + r
        ref += projector.back(cfg, a * (1.0 - y / yb), p1, p2).ravel()
        absref += projector.back(cfg, a * (1.0 + y / yb), p1, p2).ravel()
        kl_ref += float(np.sum(poisson.kl(yb, y)))
        _say(f"[{cfg['name']}] oracle view {j + 1}/{len(views)}")
    ref = psf.blur(ref.reshape(geom.shape), cfg).ravel()
    scale = np.linalg.norm(psf.blur(absref.reshape(geom.shape), cfg))
    err = np.linalg.norm(g_gpu - ref) / scale
    err_c = np.linalg.norm(gc_gpu - ref) / scale
    _say(f"[{cfg['name']}] whole-subset gradient, cancellation-aware error: dense {err:.2e}, "
         f"zero-count-aware {err_c:.2e}")
    assert err <= 1e-5
    assert err_c <= 1e-5
    assert float(kl.cpu()) == pytest.approx(kl_ref, rel=1e-6)
    assert float(klc.cpu()) == pytest.approx(kl_ref, rel=1e-6)


def test_fullsize_sensitivity_fold_and_counts_osem(big):
    # At full size, GPU against GPU (the oracle pins both forms on the small
    # workloads): on TOF geometries the sensitivity from the bins' weights
    # summed per sample against the per-bin backprojection of an all-ones
    # sinogram (relative L2 <= 2e-6); one OSEM epoch from the compacted bins
    # against the dense epoch (<= 1e-5).
    cfg, pm, dev, geom = big["cfg"], big["pm"], big["dev"], big["geom"]
    if cfg["n_tof"] > 1:
        fold = torch.empty(geom.n_vox, device=dev)
        pm.pet_back(geom, 2, None, big["a"], fold)
        ones = torch.ones(geom.n_bins, device=dev)
        per_bin = torch.empty(geom.n_vox, device=dev)
        pm.pet_back(geom, 2, ones, big["a"], per_bin)
        del ones
        e = float((fold.double() - per_bin.double()).norm() / per_bin.double().norm())
        _say(f"[{cfg['name']}] sensitivity, summed bin weights against per bin: {e:.2e}")
        assert e <= 2e-6
    cnt = pm.Counts(geom, big["y"], big["r"], big["a"])
    n = cfg["n_subsets"]
    xc = torch.ones(geom.n_vox, device=dev)
    xd = torch.ones(geom.n_vox, device=dev)
    pm.pet_osem_epoch_counts(geom, cnt, xc, big["a"], list(range(n)))
    pm.pet_osem_epoch(geom, xd, big["y"], big["r"], big["a"], list(range(n)))
    cnt.close()
    e = float((xc.double() - xd.double()).norm() / xd.double().norm())
    _say(f"[{cfg['name']}] OSEM epoch, compacted bins against dense: {e:.2e}")
    assert e <= 1e-5


def test_fullsize_adjoint_identity(big):
    pm, geom, dev = big["pm"], big["geom"], big["dev"]
    gen = torch.Generator(device=dev).manual_seed(3)
    xv = torch.rand(geom.n_vox, device=dev, generator=gen)
    yv = torch.rand(geom.n_bins, device=dev, generator=gen)
    px = torch.zeros(geom.n_bins, device=dev)
    pm.pet_fwd(geom, 0, xv, None, None, px)
    pty = torch.empty(geom.n_vox, device=dev)
    views = configs.subset_views(big["cfg"], 0)
    mask = torch.zeros(big["cfg"]["n_views"], device=dev)
    mask[views] = 1.0
    ym = (yv.view(big["cfg"]["n_views"], -1) * mask[:, None]).reshape(-1)
    pm.pet_back(geom, 0, ym, None, pty)
    V = big["cfg"]["n_views"]
    lhs = sum(float(torch.dot(px.view(V, -1)[v].double(), ym.view(V, -1)[v].double())) for v in views)
    rhs = float(torch.dot(xv.double(), pty.double()))
    _say(f"[{big['cfg']['name']}] adjoint identity relative gap {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


def test_c1_osem_two_epochs_against_golden():
    # The 3D non-TOF brain-sized workload after one OSEM epoch from x = 1 and
    # two epochs of preconditioned SVRG, dense and zero-count-aware, against
    # the FP64 oracle's image of the same schedule (stored by
    # tests/golden/make_c1_osem_2epochs.py, which runs the oracle alone).
    import os
    import paper_2506_04976_amd as pm
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_3d_osem_2epochs.npz")
    gold = np.load(path)
    cfg = configs.get("c1_3d")
    n, epochs = cfg["n_subsets"], int(gold["epochs"])
    _say("\n[c1 golden] generating data")
    d = data.make_dataset(cfg)
    dev = torch.device("cuda:0")
    geom = pm.Geometry(cfg)
    y = torch.from_numpy(d["y"].reshape(-1)).to(dev)
    r = torch.from_numpy(d["r"].reshape(-1)).to(dev)
    a = torch.from_numpy(d["mult"].reshape(-1)).to(dev)
    del d
    beta = configs.beta_value(cfg)
    assert beta == pytest.approx(float(gold["beta"]), rel=1e-12)
    orders = data.subset_orders(cfg, epochs)
    assert np.array_equal(np.asarray(orders), gold["orders"])
    sens = torch.empty(geom.n_vox, device=dev)
    pm.pet_back(geom, -1, None, a, sens)
    cnt = pm.Counts(geom, y, r, a)
    x_ref = gold["x"].astype(np.float64).ravel()
    tau = recon.stepsize_vanishing(1.0, 0.02, n)
    upd = recon.pc_update_iters(n)
    for name, c in (("dense", None), ("zero-count-aware", cnt)):
        x = torch.ones(geom.n_vox, device=dev)
        xmax = torch.zeros(1, device=dev)
        pm.pet_osem_epoch(geom, x, y, r, a, list(range(n)), xmax)
        mx = float(xmax.cpu())
        assert mx == pytest.approx(float(gold["x_osem_max"]), rel=1e-5)
        st = pm.SvrgStateBuffers(geom, y, r, a, sens, beta=beta, gamma=2.0, eps=1e-3 * mx, alpha=1.0,
                                 delta=1e-3 * mx, counts=c)
        for e in range(epochs):
            ks = [e * n + j for j in range(n)]
            pm.pet_svrg_epoch(geom, st, x, orders[e], [tau(k) for k in ks], [k in upd for k in ks])
        err = np.linalg.norm(x.cpu().double().numpy() - x_ref) / np.linalg.norm(x_ref)
        _say(f"[c1 golden] {name}: OSEM + {epochs} epochs, relative L2 {err:.2e}")
        assert err <= 1e-4
    cnt.close()
    geom.close()


def test_c3_reconstruction_parity():
    import paper_2506_04976_amd as pm
    cfg = configs.get("c3_diff")
    n, epochs = cfg["n_subsets"], cfg["epochs"]
    _say("\n[c3] generating data")
    d = data.make_dataset(cfg)
    dev = torch.device("cuda:0")
    geom = pm.Geometry(cfg)
    y = torch.from_numpy(d["y"].reshape(-1)).to(dev)
    r = torch.from_numpy(d["r"].reshape(-1)).to(dev)
    a = torch.from_numpy(d["mult"].reshape(-1)).to(dev)
    beta = configs.beta_value(cfg)
    x = torch.ones(geom.n_vox, device=dev)
    xmax = torch.zeros(1, device=dev)
    pm.pet_osem_epoch(geom, x, y, r, a, list(range(n)), xmax)
    mx = float(xmax.cpu())
    sens = torch.empty(geom.n_vox, device=dev)
    pm.pet_back(geom, -1, None, a, sens)
    st = pm.SvrgStateBuffers(geom, y, r, a, sens, beta=beta, gamma=2.0, eps=1e-3 * mx, alpha=1.0, delta=1e-3 * mx)
    orders = data.subset_orders(cfg, epochs)
    tau = recon.stepsize_vanishing(1.0, 0.02, n)
    upd = recon.pc_update_iters(n)
    for e in range(epochs):
        ks = [e * n + j for j in range(n)]
        pm.pet_svrg_epoch(geom, st, x, orders[e], [tau(k) for k in ks], [k in upd for k in ks])
    x_gpu = x.cpu().double().numpy()
    _say("[c3] GPU done; oracle OSEM + SVRG")
    prob0 = recon.Problem(cfg, d["y"], d["r"], d["mult"], beta=beta, gamma=2.0, eps=1.0, alpha=1.0, delta=1.0)
    x0 = recon.osem_epoch(prob0, np.ones(prob0.shape))
    m0 = float(x0.max())
    assert m0 == pytest.approx(mx, rel=1e-5)
    prob = recon.Problem(cfg, d["y"], d["r"], d["mult"], beta=beta, gamma=2.0, eps=1e-3 * m0, alpha=1.0,
                         delta=1e-3 * m0)
    prob._sens_i = prob0._sens_i
    x_orc = recon.svrg(prob, x0, epochs, recon.order_rule(orders), tau, upd).ravel()
    err = np.linalg.norm(x_gpu - x_orc) / np.linalg.norm(x_orc)
    _say(f"[c3] {epochs} epochs: relative L2 {err:.2e}")
    assert err <= 1e-4
    geom.close()
