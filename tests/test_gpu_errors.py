"""GPU: argument errors of the geometry description and of the extended epoch
entry points are reported as PET_E_ARG before any kernel runs (the geometry
handle needs a device, so these run where there is one)."""

import pytest
import torch

from synth import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import paper_2506_04976_amd as pm
    return pm


@pytest.mark.parametrize("bad", [dict(n_tof=33), dict(psf_fwhm=-1.0), dict(psf_fwhm=400.0),
                                 dict(n_subsets=0), dict(max_ring_diff=8)])
def test_geometry_description_errors(pm, bad):
    with pytest.raises(pm.PetError):
        pm.Geometry(configs.get("mini_tof", **bad))


def test_epoch_option_errors(pm):
    cfg = configs.get("mini_tof")
    g = pm.Geometry(cfg)
    dev = torch.device("cuda:0")
    y = torch.zeros(g.n_bins, dtype=torch.uint8, device=dev)
    r = torch.full((g.n_bins,), 0.1, device=dev)
    a = torch.ones(g.n_lors, device=dev)
    sens = torch.ones(g.n_vox, device=dev)
    x = torch.ones(g.n_vox, device=dev)
    n = g.n_subsets
    st = pm.SvrgStateBuffers(g, y, r, a, sens, beta=0.1, gamma=2.0, eps=1e-3)
    seq, tau, upd = list(range(n)), [1.0] * n, [True] + [False] * (n - 1)
    # BB update flags need the BB state and may sit on snapshot iterations only
    with pytest.raises(pm.PetError, match="bb"):
        pm.pet_svrg_epoch(g, st, x, seq, tau, upd, bb_update=[True] + [False] * (n - 1))
    stb = pm.SvrgStateBuffers(g, y, r, a, sens, beta=0.1, gamma=2.0, eps=1e-3, bb=True)
    with pytest.raises(pm.PetError, match="snapshot"):
        pm.pet_svrg_epoch(g, stb, x, seq, tau, upd, bb_update=[False, True] + [False] * (n - 2))
    # estimator weights must be positive and finite
    for w in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(pm.PetError, match="weights"):
            pm.pet_svrg_epoch(g, st, x, seq, tau, upd, weight=[w] * n)
    # subset indices
    with pytest.raises(pm.PetError, match="range"):
        pm.pet_saga_epoch(g, st, x, [n] + seq[1:], tau, upd)
    assert st.k == 0 and stb.k == 0, "a refused call must not advance the state"
    torch.cuda.synchronize()
    g.close()
