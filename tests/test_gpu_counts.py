"""GPU parity of the zero-count-aware path (pet_counts_*, pet_subset_grad_counts,
pet_objective_counts, pet_svrg_epoch with state->counts) through the C ABI
against the FP64 oracle, which evaluates the dense formulas over every bin
(Section 1.2's d(s, t), eq. (svrg)).  The identity the path rests on,
grad D_i = P_i^T mult - P_i^T[mult y / ybar], is therefore checked against an
oracle that never splits the sum.  Tolerances as in the dense parity tests:
cancellation-aware 1e-5 for gradients, 1e-5 relative for objectives, 1e-4 for
images after the workload's epochs."""

import numpy as np
import pytest
import torch

from oracle import poisson, recon
from synth import configs, data

pytestmark = pytest.mark.gpu

CASES = ["mini_tof", "mini_nontof", "mini_2d", "c0_2d", "mini_tof_psf", "mini_tof_many", "mini_tof_seg40"]


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


class CountsCase:
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
        self.counts = pm.Counts(self.geom, self.y, self.r, self.a)
        self.T = self.cfg["n_tof"]
        self.prob = recon.Problem(self.cfg, self.d["y"], self.d["r"], self.d["mult"],
                                  beta=configs.beta_value(self.cfg), gamma=2.0, eps=1e-3 * float(self.x_np.max()),
                                  alpha=1.0, delta=1e-3 * float(self.x_np.max()))

    def sens_subset(self, subset):
        s = torch.empty(self.geom.n_vox, device=self.dev)
        self.pm.pet_back(self.geom, subset, None, self.a, s)
        return s


@pytest.fixture(scope="module", params=CASES)
def case(request):
    print(f"\n[gpu counts case {request.param}]", flush=True)
    return CountsCase(request.param)


def test_counts_index(case):
    # the compacted bins are exactly the bins with y > 0, per subset; the FP64
    # sums over every bin of the subset match numpy's
    y = case.d["y"].astype(np.float64)
    r = case.d["r"].astype(np.float64)
    for subset in list(range(case.cfg["n_subsets"])) + [-1]:
        views = list(range(case.cfg["n_views"])) if subset < 0 else configs.subset_views(case.cfg, subset)
        n_items, sy, sa = case.counts.info(subset)
        assert n_items == int(np.count_nonzero(y[views]))
        assert sy == pytest.approx(float(y[views].sum()), rel=1e-12)
        assert sa == pytest.approx(float(r[views].sum()), rel=1e-12)


def test_counts_subset_grad_and_kl_parity(case):
    pm = case.pm
    xo = case.x_np.astype(np.float64)
    for subset in range(case.cfg["n_subsets"]):
        sens = case.sens_subset(subset)
        g = torch.full((case.geom.n_vox,), float("nan"), device=case.dev)
        kl = torch.zeros(1, dtype=torch.float64, device=case.dev)
        pm.pet_subset_grad_counts(case.geom, case.counts, subset, case.x, sens, g, kl)
        ref = case.prob.data_grad(xo, subset).ravel()
        yb = case.prob.ybar(xo, subset)
        scale = np.linalg.norm(case.prob.back(case.prob.a[subset] * (1 + case.prob.y[subset] / yb), subset))
        err = np.linalg.norm(g.cpu().double().numpy() - ref) / scale
        assert err <= 1e-5, f"subset {subset}: {err:.3e}"
        kl_ref = float(np.sum(poisson.kl(yb, case.prob.y[subset])))
        assert float(kl.cpu()) == pytest.approx(kl_ref, rel=1e-5)
        # the part that depends on x alone: grad - sens_i
        h = torch.empty(case.geom.n_vox, device=case.dev)
        pm.pet_subset_grad_counts(case.geom, case.counts, subset, case.x, None, h)
        err_h = np.linalg.norm((h + sens).cpu().double().numpy() - ref) / scale
        assert err_h <= 1e-5, f"subset {subset}: {err_h:.3e}"


def test_counts_signed_sheets(case):
    # PET_SIGNED_SHEETS: every chunk accumulates its fixed-point sheet in the
    # signed form (low word with borrow) that chunks with a negative factor
    # take; on the same well-conditioned data, the same oracle bar.
    pm = case.pm
    xo = case.x_np.astype(np.float64)
    pm.pet_geom_set_flags(case.geom, pm.PET_SIGNED_SHEETS)
    try:
        for subset in range(case.cfg["n_subsets"]):
            sens = case.sens_subset(subset)
            g = torch.full((case.geom.n_vox,), float("nan"), device=case.dev)
            pm.pet_subset_grad_counts(case.geom, case.counts, subset, case.x, sens, g)
            ref = case.prob.data_grad(xo, subset).ravel()
            yb = case.prob.ybar(xo, subset)
            scale = np.linalg.norm(case.prob.back(case.prob.a[subset] * (1 + case.prob.y[subset] / yb), subset))
            err = np.linalg.norm(g.cpu().double().numpy() - ref) / scale
            assert err <= 1e-5, f"subset {subset}: {err:.3e}"
    finally:
        pm.pet_geom_set_flags(case.geom, 0)


def test_counts_negative_means(case):
    # Negative means lie outside the domain (d = inf for s <= 0 < t), but
    # without PET_CHECK the kernels still evaluate the formulas.  With x < 0
    # and add < 0 every bin has ybar <= add < 0, so every factor Q is negative
    # and each chunk switches to the signed fixed-point sheet by itself; |ybar|
    # stays >= |add|, so the data are as well conditioned as for x >= 0 and the
    # oracle bar is the same.
    pm = case.pm
    xn = (-case.x_np).astype(np.float32)
    xo = xn.astype(np.float64)
    x = torch.from_numpy(xn.ravel()).to(case.dev)
    neg_r = -case.r
    cnt = pm.Counts(case.geom, case.y, neg_r, case.a)
    prob = recon.Problem(case.cfg, case.d["y"], -case.d["r"], case.d["mult"], beta=1.0, gamma=2.0, eps=1.0)
    try:
        for subset in range(case.cfg["n_subsets"]):
            yb = prob.ybar(xo, subset)
            yy = prob.y[subset]
            assert np.all(yb[yy > 0] < 0)
            sens = case.sens_subset(subset)
            g = torch.full((case.geom.n_vox,), float("nan"), device=case.dev)
            pm.pet_subset_grad_counts(case.geom, cnt, subset, x, sens, g)
            ref = prob.data_grad(xo, subset).ravel()
            scale = np.linalg.norm(prob.back(prob.a[subset] * (1 + yy / np.abs(yb)), subset))
            err = np.linalg.norm(g.cpu().double().numpy() - ref) / scale
            assert err <= 1e-5, f"subset {subset}: {err:.3e}"
    finally:
        cnt.close()


def test_counts_chunked_grad_parity(case):
    # PET_SMALL_CHUNKS cuts every line's bins into chunks of 16, each with its
    # own fixed-point scale and sheet readout: same oracle bar as above
    pm = case.pm
    y = case.d["y"]
    per_line = np.count_nonzero(y.reshape(y.shape[0] * y.shape[1], -1), axis=1)
    xo = case.x_np.astype(np.float64)
    pm.pet_geom_set_flags(case.geom, pm.PET_SMALL_CHUNKS)
    try:
        for subset in range(case.cfg["n_subsets"]):
            sens = case.sens_subset(subset)
            g = torch.full((case.geom.n_vox,), float("nan"), device=case.dev)
            pm.pet_subset_grad_counts(case.geom, case.counts, subset, case.x, sens, g)
            ref = case.prob.data_grad(xo, subset).ravel()
            yb = case.prob.ybar(xo, subset)
            scale = np.linalg.norm(case.prob.back(case.prob.a[subset] * (1 + case.prob.y[subset] / yb), subset))
            err = np.linalg.norm(g.cpu().double().numpy() - ref) / scale
            assert err <= 1e-5, f"subset {subset}: {err:.3e}"
    finally:
        pm.pet_geom_set_flags(case.geom, 0)
    if case.cfg["kind"] != "parallel2d":  # (2D lines hold one bin each)
        assert per_line.max() > 16, "no line has more than one chunk"


def test_counts_objective_parity(case):
    pm = case.pm
    sens = case.sens_subset(-1)
    w27 = pm.rdp_weights27(case.cfg["vx"], case.cfg["vy"], case.cfg["vz"])
    out = torch.zeros(1, dtype=torch.float64, device=case.dev)
    pm.pet_objective_counts(case.geom, case.counts, case.x, sens, None, w27, case.prob.beta, case.prob.gamma,
                            case.prob.eps, out)
    assert float(out.cpu()) == pytest.approx(case.prob.objective(case.x_np.astype(np.float64)), rel=1e-5)


def test_counts_osem_epoch_parity(case):
    # one OSEM epoch from the compacted bins (the numerator from the bins with
    # counts alone; on TOF geometries P_i^T mult from the summed bin weights),
    # in a shuffled subset order, against the FP64 oracle's dense epoch and the
    # GPU's dense epoch
    pm = case.pm
    n = case.cfg["n_subsets"]
    order = [int(v) for v in np.random.default_rng(3).permutation(n)]
    x = torch.ones(case.geom.n_vox, device=case.dev)
    xmax = torch.zeros(1, device=case.dev)
    sens = torch.full((case.geom.n_vox,), float("nan"), device=case.dev)
    pm.pet_osem_epoch_counts(case.geom, case.counts, x, case.a, order, xmax, sens_out=sens)
    got = x.cpu().double().numpy()
    ref = recon.osem_epoch(case.prob, np.ones(case.prob.shape), order).ravel()
    assert _rel(got, ref) <= 1e-5
    assert float(xmax.cpu()) == float(got.max())
    # the sensitivity summed over the epoch's subsets: the oracle's A^T 1
    assert _rel(sens.cpu().numpy(), case.prob.sens().ravel()) <= 1e-5
    xd = torch.ones(case.geom.n_vox, device=case.dev)
    pm.pet_osem_epoch(case.geom, xd, case.y, case.r, case.a, order, None)
    assert _rel(got, xd.cpu().double().numpy()) <= 1e-5
    # a second epoch from there (x no longer uniform)
    pm.pet_osem_epoch_counts(case.geom, case.counts, x, case.a, order, None)
    ref2 = recon.osem_epoch(case.prob, ref.reshape(case.prob.shape), order).ravel()
    assert _rel(x.cpu().double().numpy(), ref2) <= 1e-5


def test_counts_osem_epoch_errors(case):
    pm = case.pm
    n = case.cfg["n_subsets"]
    x = torch.ones(case.geom.n_vox, device=case.dev)
    other = pm.Geometry(case.cfg)
    try:
        with pytest.raises(pm.PetError, match="another geometry"):
            pm.pet_osem_epoch_counts(other, case.counts, x, case.a, list(range(n)))
    finally:
        other.close()
    with pytest.raises(pm.PetError, match="order entry out of range"):
        pm.pet_osem_epoch_counts(case.geom, case.counts, x, case.a, [n] + list(range(n - 1)))


def _svrg(case, counts, epochs, algo="svrg"):
    pm = case.pm
    cfg, n = case.cfg, case.cfg["n_subsets"]
    beta = configs.beta_value(cfg)
    x = torch.ones(case.geom.n_vox, device=case.dev)
    xmax = torch.zeros(1, device=case.dev)
    pm.pet_osem_epoch(case.geom, x, case.y, case.r, case.a, list(range(n)), xmax)
    mx = float(xmax.cpu())
    sens = case.sens_subset(-1)
    st = pm.SvrgStateBuffers(case.geom, case.y, case.r, case.a, sens, beta=beta, gamma=2.0, eps=1e-3 * mx,
                             alpha=1.0, delta=1e-3 * mx, counts=case.counts if counts else None)
    orders = data.subset_orders(cfg, epochs)
    tau_rule = recon.stepsize_vanishing(0.3, 0.5, n) if algo == "sgd" else recon.stepsize_vanishing(1.0, 0.02, n)
    upd = recon.pc_update_iters(n)
    obj = torch.zeros(1, dtype=torch.float64, device=case.dev)
    epoch_fn = {"svrg": pm.pet_svrg_epoch, "saga": pm.pet_saga_epoch, "sgd": pm.pet_sgd_epoch}[algo]
    for e in range(epochs):
        ks = [e * n + j for j in range(n)]
        epoch_fn(case.geom, st, x, orders[e], [tau_rule(k) for k in ks], [k in upd for k in ks], obj)
    return x.cpu().double().numpy(), float(obj.cpu()), (orders, tau_rule, upd, beta)


def test_counts_svrg_reconstruction_parity(case):
    epochs = case.cfg["epochs"]
    x_cnt, obj_cnt, (orders, tau_rule, upd, beta) = _svrg(case, True, epochs)
    x0 = recon.osem_epoch(case.prob, np.ones(case.prob.shape))
    m0 = float(x0.max())
    prob = recon.Problem(case.cfg, case.d["y"], case.d["r"], case.d["mult"], beta=beta, gamma=2.0, eps=1e-3 * m0,
                         alpha=1.0, delta=1e-3 * m0)
    x_orc = recon.svrg(prob, x0, epochs, recon.order_rule(orders), tau_rule, upd).ravel()
    err = _rel(x_cnt, x_orc)
    print(f"[{case.cfg['name']}] zero-count-aware SVRG, {epochs} epochs: relative L2 {err:.2e}", flush=True)
    assert err <= 1e-4
    assert obj_cnt == pytest.approx(prob.objective(x_cnt.reshape(prob.shape)), rel=1e-5)
    # and the dense GPU path on the same schedule
    x_dense, obj_dense, _ = _svrg(case, False, epochs)
    assert _rel(x_cnt, x_dense) <= 1e-4
    assert obj_cnt == pytest.approx(obj_dense, rel=1e-5)


@pytest.mark.parametrize("algo", ["saga", "sgd"])
def test_counts_saga_sgd_reconstruction_parity(case, algo):
    # SAGA (table of h_i + (beta/n) grad S, sum from the sensitivity) and SGD
    # (subset sensitivities in state->ghat_i) on the zero-count-aware path,
    # against the FP64 oracle's dense iteration and against the GPU's dense
    # path on the same schedule (eq. (saga), Section 2.1).
    epochs = case.cfg["epochs"]
    x_cnt, obj_cnt, (orders, tau_rule, upd, beta) = _svrg(case, True, epochs, algo)
    x0 = recon.osem_epoch(case.prob, np.ones(case.prob.shape))
    m0 = float(x0.max())
    prob = recon.Problem(case.cfg, case.d["y"], case.d["r"], case.d["mult"], beta=beta, gamma=2.0, eps=1e-3 * m0,
                         alpha=1.0, delta=1e-3 * m0)
    x_orc = getattr(recon, algo)(prob, x0, epochs, recon.order_rule(orders), tau_rule, upd).ravel()
    err = _rel(x_cnt, x_orc)
    print(f"[{case.cfg['name']}] zero-count-aware {algo}, {epochs} epochs: relative L2 {err:.2e}", flush=True)
    assert err <= 1e-4
    assert obj_cnt == pytest.approx(prob.objective(x_cnt.reshape(prob.shape)), rel=1e-5)
    x_dense, obj_dense, _ = _svrg(case, False, epochs, algo)
    assert _rel(x_cnt, x_dense) <= 1e-4
    assert obj_cnt == pytest.approx(obj_dense, rel=1e-5)


def test_counts_argument_errors(case):
    pm = case.pm
    other = pm.Geometry(case.cfg)
    g = torch.empty(case.geom.n_vox, device=case.dev)
    with pytest.raises(pm.PetError, match="another geometry") as ei:
        pm.pet_subset_grad_counts(other, case.counts, 0, case.x, None, g)
    assert ei.value.status == 1
    with pytest.raises(pm.PetError, match="sens_subset"):
        pm.pet_subset_grad_counts(case.geom, case.counts, 0, case.x, None, g,
                                  torch.zeros(1, dtype=torch.float64, device=case.dev))
    n = case.cfg["n_subsets"]
    sens = case.sens_subset(-1)
    seq, tau, upd = list(range(n)), [1.0] * n, [True] + [False] * (n - 1)
    other_counts = pm.Counts(other, case.y, case.r, case.a)
    st_other = pm.SvrgStateBuffers(case.geom, case.y, case.r, case.a, sens, beta=0.1, gamma=2.0, eps=1e-3,
                                   counts=other_counts)
    for fn in (pm.pet_svrg_epoch, pm.pet_saga_epoch, pm.pet_sgd_epoch):
        with pytest.raises(pm.PetError, match="another geometry"):
            fn(case.geom, st_other, case.x.clone(), seq, tau, upd)
    del st_other
    other_counts.close()
    stg = pm.SvrgStateBuffers(case.geom, case.y, case.r, case.a, sens, beta=0.1, gamma=2.0, eps=1e-3,
                              counts=case.counts, gnorm=True)
    with pytest.raises(pm.PetError, match="gnorm"):
        pm.pet_svrg_epoch(case.geom, stg, case.x.clone(), seq, tau, upd)
    torch.cuda.synchronize()
    other.close()


def test_snapshot_objective(case):
    # the objective at each snapshot, summed from the snapshot's own passes
    # (dense and zero-count-aware), against the oracle's objective at xhat
    pm = case.pm
    cfg, n = case.cfg, case.cfg["n_subsets"]
    beta = configs.beta_value(cfg)
    sens = case.sens_subset(-1)
    x0 = torch.ones(case.geom.n_vox, device=case.dev)
    xmax = torch.zeros(1, device=case.dev)
    pm.pet_osem_epoch(case.geom, x0, case.y, case.r, case.a, list(range(n)), xmax)
    eps = 1e-3 * float(xmax.cpu())
    prob = recon.Problem(cfg, case.d["y"], case.d["r"], case.d["mult"], beta=beta, gamma=2.0, eps=eps)
    orders = data.subset_orders(cfg, 3)
    for counts in (None, case.counts):
        x = x0.clone()
        st = pm.SvrgStateBuffers(case.geom, case.y, case.r, case.a, sens, beta=beta, gamma=2.0, eps=eps,
                                 alpha=1.0, delta=eps, counts=counts, snap_objective=True)
        for e in range(3):
            ks = [e * n + j for j in range(n)]
            pm.pet_svrg_epoch(case.geom, st, x, orders[e], [1.0] * n, [k in (0, n, 2 * n) for k in ks])
            if e % 2 == 0:  # epochs 0 and 2 start with a snapshot
                got = float(st.snap_objective.cpu())
                ref = prob.objective(st.x_snap.cpu().double().numpy().reshape(prob.shape))
                assert got == pytest.approx(ref, rel=1e-5), (counts is not None, e)


@pytest.mark.parametrize("n_rings,counts", [(18, 4e7), (20, 5e8)])
def test_counts_many_bins_per_line(n_rings, counts):
    # Lines with more bins with counts than the workgroup has threads: phase
    # two keeps up to four rounds of bins per thread in registers, and a line
    # with more than 2048 takes a second chunk (the image sheet rebuilt).  A
    # small TOF geometry with many planes and high counts; the subset gradient
    # and KL against the FP64 oracle's dense formulas.
    import paper_2506_04976_amd as pm
    cfg = configs.get("mini_tof_many", n_rings=n_rings, counts=counts)
    d = data.make_dataset(cfg)
    per_line = (d["y"] > 0).reshape(cfg["n_views"], cfg["n_rad"], -1).sum(-1)
    assert per_line.max() > (2048 if counts > 1e8 else 1024)
    dev = torch.device("cuda:0")
    geom = pm.Geometry(cfg)
    y = torch.from_numpy(d["y"].ravel()).to(dev)
    r = torch.from_numpy(d["r"].ravel()).to(dev)
    a = torch.from_numpy(d["mult"].ravel()).to(dev)
    cnt = pm.Counts(geom, y, r, a)
    rng = np.random.default_rng(8)
    x_np = (d["x_true"] * rng.uniform(0.7, 1.3, d["x_true"].shape) + 0.05 * d["x_true"].max()).astype(np.float32)
    x = torch.from_numpy(x_np.ravel()).to(dev)
    prob = recon.Problem(cfg, d["y"], d["r"], d["mult"], beta=0.0, gamma=2.0, eps=1e-3)
    xo = x_np.astype(np.float64)
    try:
        for subset in (0, cfg["n_subsets"] - 1):
            sens = torch.empty(geom.n_vox, device=dev)
            pm.pet_back(geom, subset, None, a, sens)
            g = torch.full((geom.n_vox,), float("nan"), device=dev)
            kl = torch.zeros(1, dtype=torch.float64, device=dev)
            pm.pet_subset_grad_counts(geom, cnt, subset, x, sens, g, kl)
            ref = prob.data_grad(xo, subset).ravel()
            yb = prob.ybar(xo, subset)
            scale = np.linalg.norm(prob.back(prob.a[subset] * (1 + prob.y[subset] / yb), subset))
            err = np.linalg.norm(g.cpu().double().numpy() - ref) / scale
            print(f"[mini_tof_many, {n_rings} rings, {counts:.0e} counts] subset {subset}: {err:.2e}", flush=True)
            assert err <= 1e-5
            assert float(kl.cpu()) == pytest.approx(float(np.sum(poisson.kl(yb, prob.y[subset]))), rel=1e-5)
    finally:
        cnt.close()
        geom.close()


def test_counts_alg2_bb_parity(case):
    # ALG2 on the zero-count-aware path: preconditioner updates at the start
    # of epochs 1, 2, 4, 6, short BB step at the snapshots of epochs 3 and 5
    # (the snapshot's full gradient from the compacted bins, in one launch
    # where the fused step serves the geometry), capped by the schedule;
    # against the FP64 oracle's dense iteration (Algorithm 1 with the short BB
    # step of Section 2.2)
    from oracle import schedules
    pm = case.pm
    cfg, n = case.cfg, case.cfg["n_subsets"]
    epochs = 6
    beta = configs.beta_value(cfg)
    x = torch.ones(case.geom.n_vox, device=case.dev)
    xmax = torch.zeros(1, device=case.dev)
    pm.pet_osem_epoch_counts(case.geom, case.counts, x, case.a, list(range(n)), xmax)
    mx = float(xmax.cpu())
    sens = case.sens_subset(-1)
    st = pm.SvrgStateBuffers(case.geom, case.y, case.r, case.a, sens, beta=beta, gamma=2.0, eps=1e-3 * mx,
                             alpha=1.0, delta=1e-3 * mx, bb=True, counts=case.counts)
    orders = data.subset_orders(cfg, epochs)
    upd = {0, n, 3 * n, 5 * n}
    bb_it = {2 * n, 4 * n}
    cap = lambda k: schedules.alg2_cap(k, n)  # noqa: E731
    for e in range(epochs):
        ks = [e * n + j for j in range(n)]
        pm.pet_svrg_epoch(case.geom, st, x, orders[e], [cap(k) for k in ks], [k in upd for k in ks],
                          bb_update=[k in bb_it for k in ks])
    x0 = recon.osem_epoch(case.prob, np.ones(case.prob.shape))
    m0 = float(x0.max())
    prob = recon.Problem(cfg, case.d["y"], case.d["r"], case.d["mult"], beta=beta, gamma=2.0, eps=1e-3 * m0,
                         alpha=1.0, delta=1e-3 * m0)
    rec = []
    x_orc = recon.svrg(prob, x0, epochs, recon.order_rule(orders), cap, upd, bb_iters=bb_it, record=rec)
    assert st.bb.cpu().numpy()[3] == len(bb_it)
    err = _rel(x.cpu().double().numpy(), x_orc.ravel())
    print(f"[{cfg['name']}] zero-count-aware ALG2, {epochs} epochs: relative L2 {err:.2e}", flush=True)
    assert err <= 1e-4
