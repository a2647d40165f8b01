"""FP64 CPU oracle for the ptychography forward model, loss and gradient.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library: it is a plain, slow, NumPy complex128 implementation written
directly from the paper's statement of the model (Eq. 1 and its composite
form Eq. 2, Section "Universal Ptychography Algorithm based on Automatic
Differentiation"), the loss functions named there (MSE on the modulus,
Gaussian and Poisson maximum likelihood), and the Fourier shift theorem used
for differentiable scan positions (Section "Benchmarking with state-of-art
open-source ptychography algorithm").

Pins (tests/test_oracle_*.py) tie it to results fixed independently of its
own code: brute-force DFT double sums (also for the exact-ratio propagator,
which reduces to the zero-padded DFT at integer ratios and has closed forms
for discrete plane waves), closed-form shifts of single Fourier
modes, Parseval, the adjoint identity of every linear operator, zero loss and
gradient at the noiseless truth, invariance under unitary mode mixing, gauge
identities of the gradient and central finite differences.  The Adam step
(the paper's optimiser) is pinned by a hand-derived three-step table with
non-zero moments, the constant-gradient closed form and scale invariance.
"""

from .model import (
    split_positions, shift_patch, shift_patch_adjoint, propagate,
    propagate_adjoint, is_ratio, scaled_dft_matrix, propagate_dalpha, resample, resample_adjoint,
    forward, loss_grad, pointwise_loss, regulariser, adam_step, LOSS_AMPLITUDE, LOSS_POISSON, LOSS_GAUSSIAN,
    LOSS_VJP, LOSS_MIXED,
)

__all__ = [
    "split_positions", "shift_patch", "shift_patch_adjoint", "propagate",
    "propagate_adjoint", "is_ratio", "scaled_dft_matrix", "propagate_dalpha", "resample",
    "resample_adjoint", "forward", "loss_grad", "pointwise_loss", "LOSS_AMPLITUDE", "LOSS_POISSON",
    "LOSS_GAUSSIAN", "LOSS_VJP", "LOSS_MIXED", "regulariser", "adam_step",
]
