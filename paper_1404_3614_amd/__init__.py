"""MI355X (gfx950) implementation of the FFT-based Galerkin method with
guaranteed upper-lower bounds on homogenized coefficients.

The compute path is the HIP library libhom.so (include/hom.h); this package
only marshals arguments and provides PyTorch-owned device memory and streams.
"""
from .api import (Problem, Batch, Group, coef_inclusions, coef_pixels, coef_from_cell, problem_from_cell, field_len,
                  workspace_bytes, HomError, set_tuning, cell_eig_range,
                  sample_cell, quad_grid, smooth_pixel_cell, probe_copy_gbs)

__all__ = ["Problem", "Batch", "Group", "coef_inclusions", "coef_pixels", "coef_from_cell", "problem_from_cell", "field_len",
           "workspace_bytes", "HomError", "set_tuning",
           "cell_eig_range", "sample_cell", "quad_grid", "smooth_pixel_cell", "probe_copy_gbs"]
