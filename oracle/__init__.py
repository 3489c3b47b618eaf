"""FP64 CPU oracle for the Gaussian-primitive slice acquisition model.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline leg use it to check the HIP path.  The product path never imports it.

* ``core``  -- ctypes wrapper of the C oracle (world frame, FP64, OpenMP).
* ``brute`` -- NumPy brute force over every (slice, pixel, Gaussian) triple.
* ``optim`` -- masked-MSE and L1 losses, the scale regulariser and AdamW.
* ``init``  -- content-adaptive sampling of the initial means (Eq. 6).
* ``topk``  -- the normalised Top-K model of Eqs. 2 and 5 (PyTorch FP64,
  gradients by autograd).
"""
from .core import (build, load, forward, forward_pixels, backward, backward_subset,
                   backward_band, forward_band, backward_subset_band, num_threads,
                   problem_arrays)
from .optim import masked_mse, masked_l1, scale_regularizer, adamw_step, StepLR
from .init import adaptive_means, sampling_weights, sampling_cdf, gradient_magnitude

__all__ = ["build", "load", "forward", "forward_pixels", "backward", "backward_subset",
           "backward_band", "forward_band", "backward_subset_band",
           "num_threads", "problem_arrays", "masked_mse", "masked_l1", "scale_regularizer", "adamw_step", "StepLR",
           "adaptive_means", "sampling_weights", "sampling_cdf", "gradient_magnitude"]
