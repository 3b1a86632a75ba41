"""GPU: the allocation-free subset gradient (pet_subset_grad_noalloc) through
the C ABI against pet_subset_grad, the entry point it mirrors, on calls in a
row whose inputs shrink (so each call finds the previous call's contents, in
another layout, in the shared static scratch), plus its size limit.

Both sides sum with floating-point atomics in different orders, so gradients
are compared to the cancellation-aware bar of the parity tests,
||g_a - g_b|| <= 1e-5 ||P_i^T a|| (a lower bound of the summand norm); the FP64
KL sums come from the same per-line partials and reductions and must agree to
rounding."""

import numpy as np
import pytest
import torch

from synth import configs, data

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import paper_2506_04976_amd as pm
    return pm


def _inputs(pm, name):
    cfg = configs.get(name)
    d = data.make_dataset(cfg)
    dev = torch.device("cuda:0")
    g = pm.Geometry(cfg)
    x = torch.from_numpy((d["x_true"] * 0.9 + 0.05 * d["x_true"].max()).astype(np.float32).ravel()).to(dev)
    y = torch.from_numpy(d["y"].ravel()).to(dev)
    r = torch.from_numpy(d["r"].ravel()).to(dev)
    a = torch.from_numpy(d["mult"].ravel()).to(dev)
    return cfg, g, x, y, r, a


def _compare(pm, name, subset):
    print(f"[noalloc {name} subset {subset}]", flush=True)
    cfg, g, x, y, r, a = _inputs(pm, name)
    dev = x.device
    ref = torch.empty(g.n_vox, device=dev)
    got = torch.full((g.n_vox,), float("nan"), device=dev)
    kl_ref = torch.zeros(1, dtype=torch.float64, device=dev)
    kl_got = torch.zeros(1, dtype=torch.float64, device=dev)
    pm.pet_subset_grad(g, subset, x, y, r, a, ref, kl_ref)
    pm.pet_subset_grad_noalloc(g, subset, x, y, r, a, got, kl_got)
    sens = torch.empty(g.n_vox, device=dev)
    pm.pet_back(g, subset, None, a, sens)
    torch.cuda.synchronize()
    err = float((got.double() - ref.double()).norm() / sens.double().norm())
    assert torch.isfinite(got).all()
    assert err <= 1e-5, (name, subset, err)
    assert float(kl_got) == pytest.approx(float(kl_ref), rel=1e-12)
    g.close()
    return err


def test_noalloc_matches_subset_grad_shrinking_inputs(pm):
    # 96x96x32 non-TOF (about 4.9 MB of sheets), then the 21x19x9 TOF geometry
    # with a resolution model (two extra image buffers), then a 23x17 2D one
    errs = [_compare(pm, "c3_diff", 2), _compare(pm, "mini_tof_psf", 1), _compare(pm, "mini_2d", -1)]
    print(f"noalloc vs pet_subset_grad: {errs}", flush=True)


def test_noalloc_repeat_call_same_geometry(pm):
    # a second call on the same input after a different geometry used the scratch
    _compare(pm, "mini_tof", 3)
    _compare(pm, "mini_nontof", 0)
    _compare(pm, "mini_tof", 3)


def test_noalloc_rejects_geometry_beyond_scratch(pm):
    # 128x128x100 non-TOF: its four sheets need 28 MB, more than the 24 MiB array
    cfg = configs.get("c1_3d", nz=100, n_subsets=25)
    g = pm.Geometry(cfg)
    dev = torch.device("cuda:0")
    x = torch.ones(g.n_vox, device=dev)
    y = torch.zeros(g.n_bins, dtype=torch.uint8, device=dev)
    out = torch.empty(g.n_vox, device=dev)
    with pytest.raises(pm.PetError, match="static scratch") as ei:
        pm.pet_subset_grad_noalloc(g, 0, x, y, None, None, out)
    assert ei.value.status == 1  # PET_E_ARG, before anything is enqueued
    torch.cuda.synchronize()
    g.close()
