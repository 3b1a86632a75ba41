"""MI355X (gfx950) RDP-regularised PET reconstruction with prior-aware
preconditioned SVRG: HIP kernels behind the C ABI of include/pet.h, with a thin
ctypes binding that uses torch only for device memory and streams."""

from ._lib import (  # noqa: F401
    EXPORTS, LIB_PATH, PET_BACK_AUTO, PET_BACK_SCATTER, Geometry, PetError, SvrgStateBuffers, lib, pet_back,
    pet_fwd, pet_objective, pet_osem_epoch, pet_precond, pet_profile_enable, pet_profile_read, pet_rdp_grad_hessdiag,
    pet_subset_grad, pet_subset_grad_noalloc, pet_svrg_epoch, pet_saga_epoch, pet_sgd_epoch, pet_work_counts, PET_KERNEL_GRAD,
    PET_KERNEL_FWD, PET_KERNEL_BACK, rdp_weights27, y_dtype_code, pet_subset_hvp, pet_rdp_hvp, pet_precond_vjp, pet_svrg_epoch_vjp, VjpBuffers,
    PET_KERNEL_HVP, Batch, PET_CHECK, PET_SMALL_CHUNKS, PET_SIGNED_SHEETS, pet_geom_set_flags, Counts, pet_subset_grad_counts, pet_objective_counts,
    pet_osem_epoch_counts,
    PET_KERNEL_COUNTS, PET_KERNEL_GATHER, PET_BACK_GATHER,
)
from .unrolled import UnrolledProblem, UnrolledSVRG, unrolled_svrg  # noqa: F401
