"""MI355X (gfx950) ptychography loss + gradient library.

The forward model of Eq. 1 (wavelength-multiplexed, multi-mode ptychography),
its losses and its hand-written adjoint run as HIP kernels in libptycho.so
(C ABI in include/ptycho.h).  ``binding`` marshals torch tensors into that
ABI; ``autograd`` wraps it as torch.autograd.Function objects.
"""
from .binding import (  # noqa: F401
    Problem, PtychoError, ptycho_forward, ptycho_loss_grad, ptycho_step,
    ptycho_status, ptycho_supported, ptycho_workspace_bytes, ptycho_transpose_table,
    ptycho_release, resample_tables, workspace, LOSS_AMPLITUDE, LOSS_POISSON,
    LOSS_GAUSSIAN, LOSS_VJP,
)
