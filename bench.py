#!/usr/bin/env python3
"""Benchmark: preconditioned-SVRG epochs/s on the 3D TOF brain-sized workload.

Workload (default): 128x128x71 image (2.086 x 2.086 x 2.03 mm), 504-crystal
ring of radius 328 mm, 344 radial x 252 views, 64 rings with ring difference
<= 20 (2204 planes), 13 TOF bins of 40 mm with a 60 mm FWHM Gaussian truncated
at 3 sigma (2.48e9 TOF bins), head phantom with 3e7 true counts, background
r = 20% of prompts, 25 subsets, RDP gamma = 2 with 26 neighbours, harmonic
preconditioner updated in epochs 1-3, stepsize 1 / (1 + 0.02 k / n).

A step is one SVRG epoch (n iterations of the subset gradient, the RDP
stencil, the preconditioner (first epochs) and the clipped update; every
second epoch starts with a full snapshot pass).  The headline runs the
zero-count-aware data term (only bins with counts are projected; the
sensitivity terms cancel in the estimator); the dense path is timed on the
same schedule beside it.  Inputs are synthetic and resident in HBM before
timing starts.  One JSON line is printed.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SVRG epochs/s (fwd+back+RDP), 3D TOF; HBM GB/s vs peak; time to NRMSE<1%"

PEAK_HBM_GBPS = 8000.0

# HBM bytes per subset gradient of the zero-count-aware kernel (the counters'
# sum over its launches divided by the subset gradients they computed), from
# calibrated FETCH_SIZE / WRITE_SIZE counter runs, and its VALU issue fraction
# (SQ counters), valid for the kernel source with this hash only (reported as
# null otherwise).
MEASURED_TRAFFIC = {"c2_tof": (207.5e6, "bd0a0f7305f90c85")}
MEASURED_VALU = {"c2_tof": (0.78, "bd0a0f7305f90c85")}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg, d, x0, beta, eps, view=0):
    """Time the FP64 oracle's subset-gradient arithmetic (forward projection,
    ratio, backprojection) on a strided sample of one view's LORs, built with
    gcc -O3 -march=native on this host, with 1 thread and with every core of
    the process's affinity set: median of 5 timed runs after one warm-up each.
    The per-LOR time is scaled to one SVRG epoch (data passes per epoch x all
    LORs) plus n RDP gradients of the image (numpy, timed the same way)."""
    import statistics
    import tempfile

    import numpy as np
    import oracle
    from oracle import projector, rdp

    cores = len(os.sched_getaffinity(0))
    tmp = tempfile.mkdtemp(prefix="pet_oracle_")
    oracle.use_library(oracle.build_native(tmp))
    T = cfg["n_tof"]
    p1, p2 = projector.view_lors(cfg, [view])
    a = d["mult"][view].reshape(-1, 1).astype(np.float64)
    r = d["r"][view].reshape(-1, T).astype(np.float64)
    y = d["y"][view].reshape(-1, T).astype(np.float64)
    x = np.asarray(x0, np.float64).reshape(cfg["nz"], cfg["ny"], cfg["nx"])
    n_lor = p1.shape[0]

    def timed(threads, stride, reps=5):
        projector._NTHREADS = threads
        sel = slice(0, None, stride)
        q1, q2, aa, rr, yy = p1[sel], p2[sel], a[sel], r[sel], y[sel]

        def once():
            t0 = time.perf_counter()
            yb = aa * projector.fwd(cfg, x, q1, q2) + rr
            projector.back(cfg, aa * (1.0 - yy / yb), q1, q2)
            return time.perf_counter() - t0

        once()
        return statistics.median(once() for _ in range(reps)) / q1.shape[0], q1.shape[0]

    # samples sized for a few seconds per run: 1/64 of the view on 1 thread,
    # 1/4 on all cores
    t1, n1 = timed(1, 64)
    tn, nn = timed(cores, 4)
    w = rdp.default_weights(cfg["vx"], cfg["vy"], cfg["vz"], cfg["nz"])
    rdp.grad(x, w, 2.0, eps)
    t_rdp = statistics.median(
        (lambda t0: (rdp.grad(x, w, 2.0, eps), time.perf_counter() - t0)[1])(time.perf_counter()) for _ in range(5))
    n = cfg["n_subsets"]
    passes = (3 * n - 1) / (2 * n)  # data passes per epoch with a snapshot every 2 epochs
    lors = cfg["n_views"] * n_lor

    def epochs_per_s(t_lor):
        return 1.0 / (passes * lors * t_lor + n * t_rdp)

    return {"value": epochs_per_s(tn), "unit": "epochs/s", "cores": cores, "kind": "oracle",
            "single_thread_value": epochs_per_s(t1),
            "sample": f"FP64 oracle (gcc -O3 -march=native) fused subset gradient (fwd, ratio, back) on every "
                      f"4th LOR of view {view} ({nn} LORs x {T} TOF bins, {cores} threads: {1e6 * tn:.2f} us/LOR) "
                      f"and every 64th ({n1} LORs, 1 thread: {1e6 * t1:.2f} us/LOR), median of 5 after a "
                      f"warm-up; numpy RDP gradient {t_rdp:.2f} s; scaled by {passes:.3f} data passes x "
                      f"{lors} LORs and {n} RDP gradients per epoch (extrapolated)"}


def map_reference(cfg, geom, pm, cnt, sens, beta, eps, delta, x0, max_iter, target, polish_iters=1500):
    """Converged MAP image x* by preconditioned L-BFGS-B (as the paper's own
    reference reconstructions): variables z with x = s z, s = sqrt(D) for the
    harmonic preconditioner D at the initial image, bounds z >= 0.  Each
    evaluation is one zero-count-aware pass over all views (gradient and FP64
    KL from the bins with counts) plus the RDP gradient and FP64 value.
    L-BFGS-B stops when its line search cannot make progress; it is restarted
    from its last point (fresh curvature pairs) until the KKT residual
    ||min(x, grad Phi)|| / ||grad Phi(x0)|| reaches `target`, max_iter
    iterations are spent, or a restart gains less than 1%; projected
    Barzilai-Borwein steps then polish the image toward the target.  The
    residual's floor from FP32 arithmetic is measured as the spread of two
    gradient evaluations at the same point (different atomic summation
    orders)."""
    import numpy as np
    import scipy.optimize as so
    import torch

    dev = x0.device
    w27 = pm.rdp_weights27(cfg["vx"], cfg["vy"], cfg["vz"])
    g = torch.empty(geom.n_vox, device=dev)
    gp = torch.empty(geom.n_vox, device=dev)
    kl = torch.zeros(1, dtype=torch.float64, device=dev)
    sv = torch.zeros(1, dtype=torch.float64, device=dev)

    def value_grad(img):
        pm.pet_subset_grad_counts(geom, cnt, -1, img, sens, g, kl)
        pm.pet_rdp_grad_hessdiag(geom, img, None, w27, beta, cfg["gamma"], eps, gp, None, sv)
        return float(kl.cpu()) + float(sv.cpu()), g.double() + gp.double()

    h = torch.empty(geom.n_vox, device=dev)
    pm.pet_rdp_grad_hessdiag(geom, x0, None, w27, beta, cfg["gamma"], eps, gp, h)
    D = torch.empty(geom.n_vox, device=dev)
    pm.pet_precond(geom, x0, sens, h, 1.0, delta, D)
    s = torch.sqrt(D.double())
    s_np = s.cpu().numpy()
    z = np.where(s_np > 0, x0.double().cpu().numpy() / np.where(s_np > 0, s_np, 1.0), 0.0)
    g0 = value_grad(x0)[1]
    g0n = float(g0.norm())
    floor = float((value_grad(x0)[1] - g0).norm()) / g0n

    def fun(zz):
        f, gr = value_grad((torch.from_numpy(zz).to(dev) * s).float())
        return f, (gr * s).cpu().numpy()

    def kkt_of(xx):
        phi, gg = value_grad(xx)
        return float(torch.minimum(xx.double(), gg).norm()) / g0n, phi

    runs, used, kkt = [], 0, None
    t_ref = time.perf_counter()

    def progress(_xk, _state={"it": 0}):
        _state["it"] += 1
        if _state["it"] % 100 == 0:
            log(f"[bench] L-BFGS-B: {used + _state['it']} iterations ({time.perf_counter() - t_ref:.0f} s)")

    while used < max_iter:
        res = so.minimize(fun, z, jac=True, method="L-BFGS-B", bounds=[(0.0, None)] * z.size, callback=progress,
                          options=dict(maxiter=max_iter - used, maxcor=10, ftol=0.0, gtol=0.0,
                                       maxfun=2 * (max_iter - used)))
        used += int(res.nit)
        z = res.x
        new_kkt, phi = kkt_of((torch.from_numpy(z).to(dev) * s).float())
        runs.append({"iterations": int(res.nit), "kkt_residual": new_kkt, "objective": phi})
        log(f"[bench] L-BFGS-B run {len(runs)}: {res.nit} iterations, KKT {new_kkt:.3e}, objective {phi:.10g}")
        gain = kkt is None or new_kkt < 0.99 * kkt
        kkt = new_kkt
        if kkt <= target or res.nit == 0 or not gain:
            break
    lbfgs_kkt = kkt
    # Polishing with projected Barzilai-Borwein steps in z, alternating the
    # long and short BB lengths: gradients only, since the line search above
    # stops once objective differences fall below the objective's FP32
    # rounding.  The best iterate (lowest KKT residual) is kept; a residual ten
    # times the best restarts from the best with half the step.  The loop
    # aims at 0.8 target: the residual is re-evaluated at the end, and two
    # evaluations at one point differ by the FP32 floor (about 0.6e-6 on C2).
    zt = torch.from_numpy(z).to(dev)
    polish = 0
    if kkt > target and polish_iters > 0:
        def grad_z(zz):
            xx = (zz * s).float()
            phi_, gr_ = value_grad(xx)
            return phi_, gr_ * s, float(torch.minimum(xx.double(), gr_).norm()) / g0n
        _, gz, kz = grad_z(zt)
        best = (kz, zt.clone())
        alpha = 1.0
        for it in range(polish_iters):
            zn = torch.clamp(zt - alpha * gz, min=0.0)
            _, gn, kn = grad_z(zn)
            dz, dg = zn - zt, gn - gz
            sy = float(torch.dot(dz, dg))
            if sy > 0:
                alpha = float(torch.dot(dz, dz)) / sy if it % 2 == 0 else sy / float(torch.dot(dg, dg))
            alpha = min(max(alpha, 1e-6), 1e6)
            zt, gz = zn, gn
            polish = it + 1
            if kn < best[0]:
                best = (kn, zt.clone())
            elif kn > 10 * best[0]:
                zt = best[1].clone()
                _, gz, _ = grad_z(zt)
                alpha *= 0.5
            if best[0] <= 0.8 * target:
                break
            if polish % 200 == 0:
                log(f"[bench] BB polishing: {polish} iterations, best KKT {best[0]:.3e}")
        zt = best[1]
        kkt, phi = kkt_of((zt * s).float())
        log(f"[bench] BB polishing: {polish} iterations, KKT {kkt:.3e}, objective {phi:.10g}")
        runs.append({"iterations": polish, "kkt_residual": kkt, "objective": phi, "method": "projected BB"})
    xstar = (zt * s).float()
    return xstar, {"method": "preconditioned L-BFGS-B with restarts, then projected BB steps",
                   "iterations": used, "polish_iterations": polish, "runs": len(runs),
                   "kkt_residual": kkt, "kkt_after_lbfgsb": lbfgs_kkt, "kkt_target": target,
                   "kkt_floor_fp32": floor, "objective": runs[-1]["objective"], "per_run": runs}


def time_to_nrmse(args, cfg, geom, pm, cnt, epochs, y, r, a, beta, eps, delta, x0_host, mask_np, level):
    """Wall time to NRMSE < 1% of the converged MAP image x*, for each run in
    `epochs` (name -> (geometry, epoch function, BB state needed, counts of
    that geometry or None, seconds their compaction took)); the first is the
    headline.

    Each reconstruction is fresh and timed from the first device call after the
    data upload (compaction of the counts, timed once per geometry; sensitivity,
    one OSEM epoch, epochs of the estimator); the NRMSE
    sqrt(mean_M (x - x*)^2) / c over the phantom's outer region M, with c the
    value of that region in the scaled phantom, is evaluated after every epoch
    with the clock stopped."""
    import torch

    dev = y.device
    x0 = torch.from_numpy(x0_host.ravel()).to(dev)
    sens0 = torch.empty(geom.n_vox, device=dev)
    pm.pet_back(geom, -1, None, a, sens0)
    log(f"[bench] reference image (L-BFGS-B, at most {args.ref_iters} iterations) ...")
    t0 = time.perf_counter()
    xstar, ref = map_reference(cfg, geom, pm, cnt, sens0, beta, eps, delta, x0, args.ref_iters, args.kkt_target)
    del sens0
    log(f"[bench] reference done in {time.perf_counter() - t0:.1f} s: {ref}")
    mask = torch.from_numpy(mask_np.ravel()).to(dev)
    nm = float(mask.sum())

    def nrmse_of(img):
        dlt = (img.double() - xstar.double()) * mask
        return float(torch.sqrt((dlt * dlt).sum() / nm)) / level

    out = {}
    for name, (geom_run, epoch, bb, cnt_run, setup_s) in epochs.items():
        n_run = geom_run.n_subsets
        x1 = torch.empty(geom.n_vox, device=dev)
        xmax = torch.zeros(1, device=dev)
        sens = torch.empty(geom.n_vox, device=dev)
        torch.cuda.synchronize()
        t_clock = 0.0
        t_epochs = 0.0
        t0 = time.perf_counter()
        x1.fill_(1.0)
        if cnt_run is not None:
            # (the OSEM epoch also sums its subset sensitivities into sens)
            pm.pet_osem_epoch_counts(geom_run, cnt_run, x1, a, list(range(n_run)), xmax, sens_out=sens)
        else:
            pm.pet_back(geom_run, -1, None, a, sens)
            pm.pet_osem_epoch(geom_run, x1, y, r, a, list(range(n_run)), xmax)
        st1 = pm.SvrgStateBuffers(geom_run, y, r, a, sens, beta=beta, gamma=cfg["gamma"], eps=eps, alpha=1.0,
                                  delta=delta, bb=bb, counts=cnt_run)
        torch.cuda.synchronize()
        # (plus the compaction of the counts on the zero-count-aware path,
        # timed once per geometry: a reconstruction from uploaded data pays it)
        t_clock += time.perf_counter() - t0 + setup_s
        trace = [nrmse_of(x1)]
        reached = None
        for e in range(args.nrmse_max_epochs):
            t0 = time.perf_counter()
            epoch(e, st=st1, x=x1)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            t_clock += dt
            t_epochs += dt
            trace.append(nrmse_of(x1))
            if trace[-1] < 0.01:
                reached = e + 1
                break
        log(f"[bench] {name}: NRMSE after OSEM and each epoch: {['%.4f' % v for v in trace]}")
        out[name] = {"seconds": t_clock if reached else None, "epochs": reached, "threshold": 0.01,
                     "epochs_per_s": (len(trace) - 1) / t_epochs, "subsets": n_run,
                     "path": "zero-count-aware" if cnt_run is not None else "dense",
                     "min_nrmse": min(trace), "final_nrmse": trace[-1]}
        del st1, x1, sens
    return out, {"reference": ref, "region_voxels": int(nm), "level": level,
                 "includes": "sensitivity, 1 OSEM epoch (on the run's data-term path; the zero-count-aware "
                             "epoch sums its subset sensitivities into the sensitivity), the estimator's epochs and, "
                             "on the zero-count-aware path, the compaction of the counts (NRMSE evaluation excluded)"}


def differentiable_leg(pm):
    """Unrolled reconstruction of the differentiable workload (96x96x32 image,
    120 views x 180 radial x 268 planes, 8 subsets, 10 epochs): plain SVRG
    epochs/s against forward + reverse (torch.autograd through the unrolled
    epochs with per-epoch checkpoints) epochs/s, same GPU, same schedule."""
    import numpy as np
    import torch
    from synth import configs, data

    cfg = configs.get("c3_diff")
    dev = torch.device("cuda:0")
    n, E = cfg["n_subsets"], cfg["epochs"]
    d = data.make_dataset(cfg)
    y = torch.from_numpy(d["y"].reshape(-1)).to(dev)
    r = torch.from_numpy(d["r"].reshape(-1)).to(dev)
    a = torch.from_numpy(d["mult"].reshape(-1)).to(dev)
    tgt = torch.from_numpy(d["x_true"].reshape(-1)).to(dev)
    geom = pm.Geometry(cfg)
    sens = torch.empty(geom.n_vox, device=dev)
    pm.pet_back(geom, -1, None, a, sens)
    x0 = torch.ones(geom.n_vox, device=dev)
    xmax = torch.zeros(1, device=dev)
    pm.pet_osem_epoch(geom, x0, y, r, a, list(range(n)), xmax)
    eps = delta = 1e-3 * float(xmax.cpu())
    beta = configs.beta_value(cfg)
    orders = data.subset_orders(cfg, E)
    taus = [[1.0 / (1.0 + 0.02 * (e * n + j) / n) for j in range(n)] for e in range(E)]
    upd = [[(e * n + j) in (0, n, 2 * n) for j in range(n)] for e in range(E)]
    prob = pm.UnrolledProblem(geom, y, r, a, sens, gamma=cfg["gamma"], eps=eps, alpha=1.0, delta=delta,
                              orders=orders, taus=taus, updates=upd)

    def plain():
        st = prob.state(beta)
        x = x0.clone()
        for e in range(E):
            pm.pet_svrg_epoch(geom, st, x, orders[e], taus[e], upd[e])
        return x

    def diff():
        xi = x0.clone().requires_grad_(True)
        lb = torch.tensor(math.log(beta), dtype=torch.float64, device=dev, requires_grad=True)
        xf = pm.unrolled_svrg(xi, lb, prob)
        ((xf - tgt) ** 2).sum().backward()
        return xi.grad

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best

    tp, td = timed(plain), timed(diff)
    geom.close()
    return {"workload": f"c3_diff: {cfg['nx']}x{cfg['ny']}x{cfg['nz']} image, {cfg['n_views']} views x "
                        f"{cfg['n_rad']} radial x {configs.n_planes(cfg)} planes, {n} subsets, {E} unrolled epochs",
            "plain_epochs_per_s": E / tp, "forward_reverse_epochs_per_s": E / td, "reverse_cost_ratio": td / tp}


def batched_leg(args):
    """Batched workload: 24 independent reconstructions of uneven sizes, TOF
    settings, counts, beta and subset counts.  Member-epochs/s of the plain
    path (each member's epochs with pet_svrg_epoch, one member after another)
    against the batched path (pet_batch_epochs: one persistent subset-gradient
    launch per step for all members, HIP-graph-captured rounds, autotuned
    launch shape), same members, same schedules, inputs resident in HBM."""
    import numpy as np
    import torch

    import paper_2506_04976_amd as pm
    from synth import configs, data

    cfg = configs.get("c4_batch")
    members = data.batch_members(cfg)
    E = args.batch_rounds
    dev = torch.device("cuda:0")
    t0 = time.time()
    M = []
    for m in members:
        d = data.make_dataset(m)
        y = torch.from_numpy(d["y"].reshape(-1)).to(dev)
        r = torch.from_numpy(d["r"].reshape(-1)).to(dev)
        a = torch.from_numpy(d["mult"].reshape(-1)).to(dev)
        del d
        g = pm.Geometry(m)
        sens = torch.empty(g.n_vox, device=dev)
        pm.pet_back(g, -1, None, a, sens)
        x0 = torch.ones(g.n_vox, device=dev)
        xmax = torch.zeros(1, device=dev)
        n = m["n_subsets"]
        pm.pet_osem_epoch(g, x0, y, r, a, list(range(n)), xmax)
        eps = 1e-3 * float(xmax.cpu())
        orders = data.subset_orders(m, E + 1)
        taus = [[1.0 / (1.0 + 0.02 * (e * n + j) / n) for j in range(n)] for e in range(E + 1)]
        upd = [[(e * n + j) in (0, n, 2 * n) for j in range(n)] for e in range(E + 1)]
        M.append(dict(cfg=m, y=y, r=r, a=a, g=g, sens=sens, x0=x0, eps=eps, orders=orders, taus=taus, upd=upd))
        log(f"[bench] member {m['name']}: {g.n_bins} bins, y {y.dtype}, {n} subsets ({time.time() - t0:.0f} s)")

    def state(mm):
        return pm.SvrgStateBuffers(mm["g"], mm["y"], mm["r"], mm["a"], mm["sens"], beta=mm["cfg"]["beta"],
                                   gamma=mm["cfg"]["gamma"], eps=mm["eps"], alpha=1.0, delta=mm["eps"])

    # plain path: epoch 0 untimed, epochs 1..E timed
    finals = []
    t_plain = 0.0
    for mm in M:
        st, x = state(mm), mm["x0"].clone()
        pm.pet_svrg_epoch(mm["g"], st, x, mm["orders"][0], mm["taus"][0], mm["upd"][0])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for e in range(1, E + 1):
            pm.pet_svrg_epoch(mm["g"], st, x, mm["orders"][e], mm["taus"][e], mm["upd"][e])
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t1
        finals.append(x)
        del st
    # batched path
    runs = [(mm["g"], state(mm), mm["x0"].clone()) for mm in M]
    b = pm.Batch(runs)
    (blocks, waves, order), step_ms = b.autotune()
    log(f"[bench] autotuned: {blocks} workgroups x {waves} waves, order {order} ({step_ms:.2f} ms per test step)")

    def rounds(lo, hi):
        b.epochs([[int(v) for e in range(lo, hi) for v in mm["orders"][e]] for mm in M],
                 [[v for e in range(lo, hi) for v in mm["taus"][e]] for mm in M],
                 [[v for e in range(lo, hi) for v in mm["upd"][e]] for mm in M], use_graph=True)

    rounds(0, 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rounds(1, E + 1)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t1
    diff = max(float(torch.linalg.norm(x2 - x1) / torch.linalg.norm(x1)) for (_, _, x2), x1 in zip(runs, finals))
    b.close()
    n_ep = len(M) * E
    return {
        "metric": "batched SVRG reconstructions: member-epochs/s",
        "value": n_ep / t_batch, "unit": "member-epochs/s", "n_gpus": 1, "steps": E, "warmup": 1,
        "ms_per_step": 1e3 * t_batch / E, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4_batch: 24 reconstructions, 4 per (size in {96x96x32, 128x128x48, 128x128x71}, "
                               "TOF 13 bins / non-TOF) cell, counts 1e6-1e8, beta 0.1-10x, 8-25 subsets",
                   "members": [{"name": mm["cfg"]["name"], "bins": mm["g"].n_bins, "subsets": mm["cfg"]["n_subsets"],
                                "counts": mm["cfg"]["counts"], "beta": mm["cfg"]["beta"]} for mm in M],
                   "parallelism": "single GPU"},
        "plain_value": n_ep / t_plain, "speedup_vs_plain": t_plain / t_batch,
        "autotuned": {"workgroups": blocks, "waves": waves, "order": ["longest lines first", "creation"][order]},
        "max_member_rel_diff_vs_plain": diff,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8, help="timed SVRG epochs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed SVRG epochs before timing")
    ap.add_argument("--config", default="c2_tof")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nrmse", action="store_true", help="skip the time-to-NRMSE measurement")
    ap.add_argument("--ref-iters", type=int, default=2000,
                    help="L-BFGS-B iterations (at most, over all restarts) of the reference image for the NRMSE")
    ap.add_argument("--kkt-target", type=float, default=1e-6)
    ap.add_argument("--nrmse-max-epochs", type=int, default=300)
    ap.add_argument("--no-estimators", action="store_true",
                    help="time to NRMSE for SVRG only (not SAGA, SGD, ALG1, ALG2, ALG3)")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiable (unrolled) leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg's summary")
    ap.add_argument("--batched", action="store_true",
                    help="measure only the batched workload (24 reconstructions; prints its own JSON line)")
    ap.add_argument("--batch-rounds", type=int, default=3)
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="also run a device-to-device copy of this many MiB (a known-size reference kernel "
                         "for calibrating hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the reconstruction would shard views across GPUs with one image all-reduce per iteration; "
              "that path is not built)", file=sys.stderr)
        sys.exit(2)

    if args.batched:
        print(json.dumps(batched_leg(args)), flush=True)
        return

    import numpy as np
    import torch

    import paper_2506_04976_amd as pm
    from paper_2506_04976_amd import schedules
    from synth import configs, data

    cfg = configs.get(args.config)
    dev = torch.device("cuda:0")
    n = cfg["n_subsets"]
    t0 = time.time()
    log(f"[bench] generating {cfg['name']} data ...")
    d = data.make_dataset(cfg)
    log(f"[bench] data ready in {time.time() - t0:.1f} s: y {d['y'].dtype} {d['y'].shape}")
    y = torch.from_numpy(d["y"].reshape(-1)).to(dev)
    r = torch.from_numpy(d["r"].reshape(-1)).to(dev)
    a = torch.from_numpy(d["mult"].reshape(-1)).to(dev)
    keep = {"y": d["y"][:1].copy(), "r": d["r"][:1].copy(), "mult": d["mult"][:1].copy()}
    nrmse_mask, nrmse_level = data.nrmse_region(cfg, d["scale"])
    del d
    geom = pm.Geometry(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cnt = pm.Counts(geom, y, r, a)
    torch.cuda.synchronize()
    t_counts = time.perf_counter() - t0
    n_items = cnt.info(-1)[0]
    log(f"[bench] uploaded; geometry ready ({geom.n_bins} bins, {geom.n_vox} voxels); {n_items} bins with "
        f"counts compacted in {t_counts:.2f} s")

    sens = torch.empty(geom.n_vox, device=dev)
    pm.pet_back(geom, -1, None, a, sens)
    x_osem = torch.ones(geom.n_vox, device=dev)
    xmax = torch.zeros(1, device=dev)
    pm.pet_osem_epoch(geom, x_osem, y, r, a, list(range(n)), xmax)
    mx = float(xmax.cpu())
    beta = configs.beta_value(cfg)
    eps = delta = 1e-3 * mx
    x0_host = x_osem.cpu().numpy()
    total = args.warmup + args.steps
    orders = data.subset_orders(cfg, max(total, args.nrmse_max_epochs))
    upd_iters = {0, n, 2 * n}

    def make_epoch(fn):
        # vanishing stepsize tau_k = 1 / (1 + 0.02 k / n) (Section 3) for every estimator
        def epoch(e, st, x):
            ks = [e * n + j for j in range(n)]
            fn(geom, st, x, orders[e], [1.0 / (1.0 + 0.02 * k / n) for k in ks], [k in upd_iters for k in ks])
        return epoch

    epoch = make_epoch(pm.pet_svrg_epoch)

    if args.copy_ref_mib > 0:
        src = torch.ones(args.copy_ref_mib * 262144, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def timed_epochs(counts, kern):
        """W warm-up and K timed SVRG epochs from the OSEM image; returns the
        elapsed time, the line kernel's total time and launches, the image."""
        x = x_osem.clone()
        st = pm.SvrgStateBuffers(geom, y, r, a, sens, beta=beta, gamma=cfg["gamma"], eps=eps, alpha=1.0,
                                 delta=delta, counts=counts)
        for e in range(args.warmup):
            epoch(e, st, x)
        torch.cuda.synchronize()
        pm.pet_profile_enable(geom, True)
        pm.pet_profile_read(geom, kern)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for e in range(args.warmup, total):
            epoch(e, st, x)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        kms, kl = pm.pet_profile_read(geom, kern)
        pm.pet_profile_enable(geom, False)
        return elapsed, kms, kl, x

    log(f"[bench] timing {args.steps} SVRG epochs (zero-count-aware path) ...")
    elapsed, grad_ms, grad_launches, x = timed_epochs(cnt, pm.PET_KERNEL_COUNTS)
    log(f"[bench] {args.steps} epochs in {elapsed:.3f} s; counts line kernel {grad_launches} launches, "
        f"{grad_ms:.1f} ms total")
    log("[bench] timing the dense path on the same schedule ...")
    elapsed_d, dense_ms, dense_launches, x_dense = timed_epochs(None, pm.PET_KERNEL_GRAD)
    log(f"[bench] dense: {args.steps} epochs in {elapsed_d:.3f} s; fused line kernel {dense_launches} launches, "
        f"{dense_ms:.1f} ms total")
    # The two paths give the same iterates up to FP32 rounding, and so do two
    # runs of one path (the order of the float atomics changes): compared over
    # all voxels and over the head region.  Outside the head the iterates carry
    # transient spikes of the method that are sensitive to rounding.
    _, _, _, x_rerun = timed_epochs(cnt, pm.PET_KERNEL_COUNTS)
    head = torch.from_numpy(nrmse_mask.ravel()).to(dev).double()

    def rel_diff(u, v, m=None):
        d = u.double() - v.double()
        w = v.double()
        if m is not None:
            d, w = d * m, w * m
        return float(d.norm() / w.norm())

    paths_rel_diff = {"all_voxels": rel_diff(x, x_dense), "head_region": rel_diff(x, x_dense, head)}
    rerun_rel_diff = {"all_voxels": rel_diff(x, x_rerun), "head_region": rel_diff(x, x_rerun, head)}
    x_max = float(x.max())
    del x_dense, x_rerun, head

    # algorithmic work of the subset gradients in the timed region.  The dense
    # path launches one per subset; the zero-count-aware path takes a snapshot
    # pass (all n subsets) in one launch, so its unit is the subset gradient.
    launched = []
    snapshots = 0
    for e in range(args.warmup, total):
        for j in range(n):
            k = e * n + j
            if k % (2 * n) == 0:
                launched += list(range(n))
                snapshots += 1
            else:
                launched += [int(orders[e][j])]
    units = len(launched)
    # (one launch per snapshot pass where the fused step serves the geometry,
    # one per subset otherwise, e.g. with a resolution model)
    assert units == dense_launches and grad_launches in (units, units - snapshots * (n - 1)), \
        (units, grad_launches, dense_launches, snapshots)
    # HBM bytes per unit (Section 8(d)'s dense data pass): per bin y (its storage
    # type) + r (FP32), per LOR mult (FP32); plus the image in and the gradient out
    hbm = 0.0
    items = 0
    for i in launched:
        nb, nl, _ = geom.info(i)
        hbm += nb * (y.element_size() + 4) + nl * 4 + 4 * geom.n_vox * 2
        items += cnt.info(i)[0]
    compulsory = 32.0 * items + 4 * geom.n_vox * 2 * len(launched)  # 32-byte records, image in, gradient out
    import hashlib
    src_hash = hashlib.sha256(open(os.path.join(ROOT, "paper_2506_04976_amd", "csrc", "counts.hip"),
                                   "rb").read()).hexdigest()[:16]
    traffic = None
    if cfg["name"] in MEASURED_TRAFFIC and MEASURED_TRAFFIC[cfg["name"]][1] == src_hash:
        traffic = MEASURED_TRAFFIC[cfg["name"]][0]
    valu = None
    if cfg["name"] in MEASURED_VALU and MEASURED_VALU[cfg["name"]][1] == src_hash:
        valu = MEASURED_VALU[cfg["name"]][0]
    grad_s = grad_ms / 1e3
    kernel_gbps = hbm / grad_s / 1e9

    w27 = pm.rdp_weights27(cfg["vx"], cfg["vy"], cfg["vz"])
    obj = torch.zeros(1, dtype=torch.float64, device=dev)
    pm.pet_objective_counts(geom, cnt, x, sens, None, w27, beta, cfg["gamma"], eps, obj)
    objective = float(obj.cpu())
    pm.pet_objective(geom, x, y, r, a, None, w27, beta, cfg["gamma"], eps, obj)
    objective_dense = float(obj.cpu())

    nrmse = None
    if not args.no_nrmse:
        algos = {"svrg": (geom, epoch, False, cnt, t_counts)}
        extra = []
        if not args.no_estimators:
            algos.update(svrg_dense=(geom, epoch, False, None, 0.0),
                         saga=(geom, make_epoch(pm.pet_saga_epoch), False, cnt, t_counts),
                         sgd=(geom, make_epoch(pm.pet_sgd_epoch), False, cnt, t_counts))
            # the submitted algorithms, each with its own subset count
            for alg, target in (("ALG1", 25.0), ("ALG2", 25.0), ("ALG3", 24.2)):
                n_alg = schedules.subsets_for(cfg["n_views"], target)
                g_alg = pm.Geometry(configs.get(cfg["name"], n_subsets=n_alg))
                torch.cuda.synchronize()
                t_alg = time.perf_counter()
                c_alg = pm.Counts(g_alg, y, r, a)
                torch.cuda.synchronize()
                t_alg = time.perf_counter() - t_alg
                extra.append((g_alg, c_alg))
                plan = schedules.algorithm_plan(alg, n_alg, args.nrmse_max_epochs,
                                                np.random.default_rng(data.seeds(cfg)[1]))

                def alg_epoch(e, st, x, g_alg=g_alg, plan=plan):
                    pe = plan[e]
                    pm.pet_svrg_epoch(g_alg, st, x, pe["subset_seq"], pe["tau"], pe["update_pc"],
                                      bb_update=pe["bb_update"])
                algos[alg.lower()] = (g_alg, alg_epoch, alg != "ALG1", c_alg, t_alg)
        runs, ref = time_to_nrmse(args, cfg, geom, pm, cnt, algos, y, r, a, beta, eps, delta, x0_host,
                                  nrmse_mask, nrmse_level)
        for g_alg, c_alg in extra:
            c_alg.close()
            g_alg.close()
        nrmse = {"threshold": 0.01, "reference": ref, "runs": runs}

    diff = None
    if not args.no_diff:
        log("[bench] differentiable leg (unrolled SVRG, forward + reverse) ...")
        diff = differentiable_leg(pm)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample of one view ...")
        cpu = cpu_baseline(cfg, keep, x0_host, beta, eps)

    cnt.close()
    geom.close()
    del y, r, a, sens, x, x_osem
    torch.cuda.empty_cache()
    batched = None
    if not args.no_batched:
        log("[bench] batched leg (24 reconstructions) ...")
        bl = batched_leg(args)
        batched = {k: bl[k] for k in ("value", "unit", "plain_value", "speedup_vs_plain",
                                      "max_member_rel_diff_vs_plain", "autotuned", "ms_per_step")}
        batched["rounds"] = bl["steps"]
        batched["workload"] = bl["config"]["workload"]

    value = args.steps / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "epochs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: {cfg['nx']}x{cfg['ny']}x{cfg['nz']} image, "
                               f"{cfg['n_views']} views x {cfg['n_rad']} radial x {geom.n_lors // (cfg['n_views'] * cfg['n_rad'])} planes"
                               f" x {cfg['n_tof']} TOF, {n} subsets, preconditioned SVRG (zero-count-aware data term)",
                   "bins": geom.n_bins, "bins_with_counts": n_items, "voxels": geom.n_vox,
                   "counts": cfg.get("counts"), "y_dtype": str(keep["y"].dtype), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": kernel_gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": kernel_gbps / PEAK_HBM_GBPS, "traffic": traffic,
                     "kernel": "k_line_counts<TOF, M_GRAD> (zero-count-aware subset gradient)",
                     # per subset gradient: a launch per iteration, one launch for
                     # all n subsets at a snapshot
                     "avg_ms_per_subset_gradient": grad_ms / units, "subset_gradients": units,
                     "launches": grad_launches,
                     "algorithmic_bytes_per_subset_gradient": hbm / units,
                     "compulsory_bytes_per_subset_gradient": compulsory / units,
                     # what the counters saw per subset gradient, as a rate against the same peak
                     "traffic_frac": (traffic / (grad_s / units) / 1e9 / PEAK_HBM_GBPS
                                      if traffic is not None else None),
                     "valu_issue": valu},
        "dense_path": {"value": args.steps / elapsed_d, "unit": "epochs/s",
                       "kernel": "k_line_tof<M_GRAD> (fused dense subset gradient)",
                       "avg_launch_ms": dense_ms / dense_launches,
                       "hbm_frac": hbm / (dense_ms / 1e3) / 1e9 / PEAK_HBM_GBPS,
                       "image_rel_diff_vs_counts_path": paths_rel_diff},
        "counts_path_rerun_rel_diff": rerun_rel_diff,
        "image_max_after_timed_epochs": x_max,
        "counts_setup_s": t_counts,
        "objective_final": objective,
        "objective_final_dense_formula": objective_dense,
        "time_to_nrmse": nrmse,
        "differentiable": diff,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
