"""ORACLE — test infrastructure only.

A plain, slow, FP64 CPU reference of the codebook-indexed differentiable
Gaussian-splatting render and its codebook gradient.  Only tests/, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path (the HIP library and its binding) never does, and shares no code with it.
"""
from .render import (AMBIGUITY_MARGIN, bin_tiles, codebook_grad_reduce, covariance3d,  # noqa: F401
                     decode_rows, exp_f32, keyspec, lib, loss_l1, project, quat_to_rot,
                     render_view, render_workload, sh_basis)
