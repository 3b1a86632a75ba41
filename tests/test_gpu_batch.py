"""GPU: batches of reconstructions.  Members of different geometries, sizes,
TOF settings, count levels, beta and subset counts advanced by pet_batch_epochs
(persistent subset-gradient launch, with and without HIP-graph replay) match
the same members advanced one by one with pet_svrg_epoch on the same schedule
(relative L2 <= 1e-5 per member; the two differ only in the summation order
of floating-point atomics), and members with and without the image-space
resolution model match the FP64 oracle's Algorithm 1 (relative L2 <= 1e-4)."""

import numpy as np
import pytest
import torch

from oracle import recon
from synth import configs, data

pytestmark = pytest.mark.gpu

# the last two carry the image-space resolution model (3D: three passes, 2D: two)
MEMBERS = [("mini_tof", 1.0), ("mini_nontof", 3.0), ("mini_2d", 0.5), ("c0_2d", 1.0), ("mini_tof_psf", 1.0),
           ("mini_2d_psf", 2.0)]


def _say(msg):
    print(msg, flush=True)


class Member:
    def __init__(self, name, beta_factor):
        import paper_2506_04976_amd as pm
        self.pm = pm
        self.cfg = configs.get(name) if isinstance(name, str) else dict(name)
        self.d = data.make_dataset(self.cfg)
        dev = torch.device("cuda:0")
        self.dev = dev
        self.y = torch.from_numpy(self.d["y"].ravel()).to(dev)
        self.r = torch.from_numpy(self.d["r"].ravel()).to(dev)
        self.a = torch.from_numpy(self.d["mult"].ravel()).to(dev)
        self.beta = configs.beta_value(self.cfg) * beta_factor
        g = pm.Geometry(self.cfg)
        self.sens = torch.empty(g.n_vox, device=dev)
        pm.pet_back(g, -1, None, self.a, self.sens)
        x = torch.ones(g.n_vox, device=dev)
        xmax = torch.zeros(1, device=dev)
        pm.pet_osem_epoch(g, x, self.y, self.r, self.a, list(range(self.cfg["n_subsets"])), xmax)
        self.x0 = x
        self.eps = 1e-3 * float(xmax.cpu())
        g.close()

    def runner(self):
        g = self.pm.Geometry(self.cfg)
        st = self.pm.SvrgStateBuffers(g, self.y, self.r, self.a, self.sens, beta=self.beta, gamma=2.0, eps=self.eps,
                                      alpha=1.0, delta=self.eps)
        return g, st, self.x0.clone()

    def schedule(self, n_epochs):
        n = self.cfg["n_subsets"]
        orders = data.subset_orders(self.cfg, n_epochs)
        taus = [[1.0 / (1.0 + 0.02 * (e * n + j) / n) for j in range(n)] for e in range(n_epochs)]
        upd = [[(e * n + j) in (0, n, 2 * n) for j in range(n)] for e in range(n_epochs)]
        return orders, taus, upd


@pytest.fixture(scope="module")
def members():
    _say("\n[batch] building members")
    return [Member(n, f) for n, f in MEMBERS]


def _rel(a, b):
    return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_individual_runs(members, use_graph):
    pm = members[0].pm
    E = 3
    singles, batched = [], []
    for m in members:
        g, st, x = m.runner()
        orders, taus, upd = m.schedule(E)
        for e in range(E):
            pm.pet_svrg_epoch(g, st, x, orders[e], taus[e], upd[e])
        singles.append((g, st, x))
        batched.append(m.runner())
    b = pm.Batch(batched)
    scheds = [m.schedule(E) for m in members]
    # one round, then two more (schedule refresh between graph replays)
    for lo, hi in ((0, 1), (1, E)):
        b.epochs([[int(v) for e in range(lo, hi) for v in s[0][e]] for s in scheds],
                 [[v for e in range(lo, hi) for v in s[1][e]] for s in scheds],
                 [[v for e in range(lo, hi) for v in s[2][e]] for s in scheds], use_graph=use_graph)
    torch.cuda.synchronize()
    for m, (g1, st1, x1), (g2, st2, x2) in zip(members, singles, batched):
        err = _rel(x2, x1)
        _say(f"[batch graph={use_graph}] {m.cfg['name']}: batched vs single relative L2 {err:.2e}")
        assert err <= 1e-5
        assert st2.k == st1.k == E * m.cfg["n_subsets"]
    b.close()


def test_batch_single_rounds_match_individual_runs(members):
    # pet_batch_epoch: one round per call, the schedule refreshed between calls
    pm = members[0].pm
    E = 2
    ref = [m.runner() for m in members]
    for m, (g, st, x) in zip(members, ref):
        orders, taus, upd = m.schedule(E)
        for e in range(E):
            pm.pet_svrg_epoch(g, st, x, orders[e], taus[e], upd[e])
    runs = [m.runner() for m in members]
    b = pm.Batch(runs)
    scheds = [m.schedule(E) for m in members]
    for e in range(E):
        b.epoch([s[0][e] for s in scheds], [s[1][e] for s in scheds], [s[2][e] for s in scheds])
    torch.cuda.synchronize()
    for m, (_, st1, x1), (_, st2, x2) in zip(members, ref, runs):
        assert _rel(x2, x1) <= 1e-5, m.cfg["name"]
        assert st2.k == st1.k == E * m.cfg["n_subsets"]
    with pytest.raises(ValueError):
        b.epoch([s[0][0][:-1] for s in scheds], [s[1][0] for s in scheds], [s[2][0] for s in scheds])
    b.close()


def test_batch_member_matches_oracle(members):
    pm = members[0].pm
    E = 3
    runs = [m.runner() for m in members]
    b = pm.Batch(runs)
    scheds = [m.schedule(E) for m in members]
    b.epochs([[int(v) for e in range(E) for v in s[0][e]] for s in scheds],
             [[v for e in range(E) for v in s[1][e]] for s in scheds],
             [[v for e in range(E) for v in s[2][e]] for s in scheds])
    psf_member = next(i for i, m in enumerate(members) if m.cfg.get("psf_fwhm", 0.0) > 0)
    for idx in (0, psf_member):
        m = members[idx]
        n = m.cfg["n_subsets"]
        x_gpu = runs[idx][2].cpu().double().numpy()
        prob = recon.Problem(m.cfg, m.d["y"], m.d["r"], m.d["mult"], beta=m.beta, gamma=2.0, eps=m.eps, alpha=1.0,
                             delta=m.eps)
        orders, taus, _ = scheds[idx]
        x0 = m.x0.cpu().double().numpy().reshape(prob.shape)
        x_orc = recon.svrg(prob, x0, E, recon.order_rule(orders), lambda k: taus[k // n][k % n],
                           recon.pc_update_iters(n)).ravel()
        err = np.linalg.norm(x_gpu - x_orc) / np.linalg.norm(x_orc)
        _say(f"[batch] {m.cfg['name']} after {E} rounds vs oracle: relative L2 {err:.2e}")
        assert err <= 1e-4
    b.close()


@pytest.mark.parametrize("shape", [(64, 2, 1), (300, 3, 0)])
def test_batch_few_waves_matches_individual_runs(members, shape):
    # fewer waves per workgroup than TOF segments: every wave takes several
    # segments of a line in turn
    pm = members[0].pm
    E = 2
    ref = [m.runner() for m in members]
    for m, (g, st, x) in zip(members, ref):
        orders, taus, upd = m.schedule(E)
        for e in range(E):
            pm.pet_svrg_epoch(g, st, x, orders[e], taus[e], upd[e])
    runs = [m.runner() for m in members]
    b = pm.Batch(runs)
    b.set_launch(*shape)
    scheds = [m.schedule(E) for m in members]
    b.epochs([[int(v) for e in range(E) for v in s[0][e]] for s in scheds],
             [[v for e in range(E) for v in s[1][e]] for s in scheds],
             [[v for e in range(E) for v in s[2][e]] for s in scheds])
    torch.cuda.synchronize()
    for m, (_, _, x1), (_, _, x2) in zip(members, ref, runs):
        err = _rel(x2, x1)
        _say(f"[batch {shape}] {m.cfg['name']}: batched vs single relative L2 {err:.2e}")
        assert err <= 1e-5, m.cfg["name"]
    with pytest.raises(pm.PetError):
        b.set_launch(64, 17)
    b.close()


def test_batch_autotune_keeps_results(members):
    pm = members[0].pm
    E = 2
    ref = [m.runner() for m in members]
    for m, (g, st, x) in zip(members, ref):
        orders, taus, upd = m.schedule(E)
        for e in range(E):
            pm.pet_svrg_epoch(g, st, x, orders[e], taus[e], upd[e])
    runs = [m.runner() for m in members]
    b = pm.Batch(runs)
    (blocks, waves, order), ms = b.autotune()
    _say(f"[batch] autotune: {blocks} workgroups x {waves} waves, order {order}, step {ms:.3f} ms")
    assert blocks > 0 and waves in (8, 12, 16) and order in (0, 1) and ms > 0
    scheds = [m.schedule(E) for m in members]
    b.epochs([[int(v) for e in range(E) for v in s[0][e]] for s in scheds],
             [[v for e in range(E) for v in s[1][e]] for s in scheds],
             [[v for e in range(E) for v in s[2][e]] for s in scheds])
    for m, (_, _, x1), (_, _, x2) in zip(members, ref, runs):
        assert _rel(x2, x1) <= 1e-5, m.cfg["name"]
    b.close()


def test_batch_c4_sized_members_match_individual_runs():
    # members at the batched workload's real sizes: a 128x128x71 TOF member
    # (2204 planes x 13 TOF bins) beside a 96x96x32 non-TOF one
    big = configs.batch_size_config(2, True)
    big.update(counts=2e7, n_subsets=25, seed=2001)
    big["beta"] = configs.beta_value(big)
    small = configs.batch_size_config(0, False)
    small.update(counts=3e6, n_subsets=8, seed=2002)
    small["beta"] = configs.beta_value(small) * 2.0
    _say("\n[batch c4 sizes] building members")
    ms = [Member(big, 1.0), Member(small, 1.0)]
    pm = ms[0].pm
    E = 2
    ref = [m.runner() for m in ms]
    for m, (g, st, x) in zip(ms, ref):
        orders, taus, upd = m.schedule(E)
        for e in range(E):
            pm.pet_svrg_epoch(g, st, x, orders[e], taus[e], upd[e])
    runs = [m.runner() for m in ms]
    b = pm.Batch(runs)
    scheds = [m.schedule(E) for m in ms]
    b.epochs([[int(v) for e in range(E) for v in s[0][e]] for s in scheds],
             [[v for e in range(E) for v in s[1][e]] for s in scheds],
             [[v for e in range(E) for v in s[2][e]] for s in scheds])
    torch.cuda.synchronize()
    for m, (_, st1, x1), (_, st2, x2) in zip(ms, ref, runs):
        err = _rel(x2, x1)
        _say(f"[batch c4 sizes] {m.cfg['name']}: batched vs single relative L2 {err:.2e}")
        assert err <= 1e-5, m.cfg["name"]
        assert st2.k == st1.k == E * m.cfg["n_subsets"]
    b.close()
