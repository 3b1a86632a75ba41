"""CPU-side checks of the C ABI: the library loads and exports every entry
point declared in include/pet.h; the binding refuses to run without a GPU."""

import ctypes
import os
import re

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pet.h")).read()
    return sorted(set(re.findall(r"\b(pet_[a-z_0-9]+)\s*\(", src)) - {"pet_geom"})


def test_header_declares_expected_entry_points():
    names = _declared()
    for n in ("pet_geom_create", "pet_geom_destroy", "pet_fwd", "pet_back", "pet_rdp_grad_hessdiag",
              "pet_svrg_epoch", "pet_subset_grad", "pet_osem_epoch", "pet_objective", "pet_precond",
              "pet_last_error", "pet_geom_info"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2506_04976_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpetmi.so not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    for n in _declared():
        assert hasattr(L, n), f"missing export {n}"
    assert sorted(_lib.EXPORTS) == _declared()


def test_argument_errors_without_gpu_work():
    from paper_2506_04976_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libpetmi.so not built")
    L = _lib.lib()
    # null handle / null descriptor are rejected synchronously with PET_E_ARG
    assert L.pet_fwd(None, 0, None, None, None, None, None) == 1
    assert b"null" in L.pet_last_error()
    assert L.pet_geom_create(None, None) == 1
    assert L.pet_geom_info(None, 0, None, None, None) == 1
    for fn in (L.pet_saga_epoch, L.pet_sgd_epoch):
        assert fn(None, None, None, None, None, None, None, None) == 1
    assert L.pet_svrg_epoch_ex(None, None, None, None, None, None, None, None, None) == 1
    assert L.pet_batch_set_launch(None, 64, 8, 0) == 1
    assert b"null" in L.pet_last_error()
    assert L.pet_batch_epoch(None, None, None, None, 1, None) == 1
    assert b"null" in L.pet_last_error()
    assert L.pet_subset_grad_noalloc(None, 0, None, None, 0, None, None, None, None, None) == 1
    assert b"null" in L.pet_last_error()
    assert L.pet_geom_set_flags(None, 1) == 1
    assert b"null" in L.pet_last_error()


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-GPU refusal")
def test_binding_refuses_without_gpu():
    import paper_2506_04976_amd as pm
    from synth import configs
    with pytest.raises(RuntimeError, match="no HIP GPU"):
        pm.Geometry(configs.get("mini_tof"))
