"""FP64 CPU oracle for local-ROI regularized tomography (TEST INFRASTRUCTURE ONLY).

This package is a plain, slow, obviously-correct NumPy/SciPy implementation of
what the library's hot path computes.  It exists to check the HIP path and is
never used by it: only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import it.  It shares no code with the HIP path; both sides
consume arrays from the seeded generator package `synth`, which holds no method
arithmetic.

Paper: D. M. Pelt, K. J. Batenburg, "A method for locally approximating
regularized iterative tomographic reconstruction methods" (arXiv 1604.02292).

Contents and the passages they follow:
  geometry   parallel-beam geometry, Section 2.1 (p: N_d N_theta values, x: N^2 pixels)
  projector  W, W^T, local operators W_L = W M_L, W_L^T = M_L W^T, Section 2.1 eq. (1)
             (ray-driven Joseph FP, pixel-driven hat BP, explicit sparse W_L)
  fbp        FBP(p, h) = W^T C_h p with the Ram-Lak filter, Section 2.2 eq. (fbp)
  tv         discrete gradient / divergence for g(x) = ||grad x||_1, Section 2.3
  solvers    Chambolle-Pock for eq. (priorsys) with D = {x >= 0} and g = TV; box-constrained
             SIRT, eq. (sirtit) + eq. (sirtbox), alpha = 1/(N_theta N_d) (Section 3.1);
             power iteration for the CP step size
  local      extended local part (Section 3.3), exterior subtraction via W = W_L + W_F
             (eq. locouter), the local solve, crop and stitch (Section 5.6)
  filters    SIRT-approximating FBP filters (Alg. 1, eq. filtcalc, eq. sirtapp), the
             per-angle detector convolution C_u, and the paper's local method
             (eq. localmethod, Alg. 2) with the box prior of eq. sirtbox
  fista      FGP total-variation denoiser and the paper's local FISTA-TV (Alg. 3)
  preprocess disc subtraction (Section 3.3) and constant padding of truncated data (Section 4)
  haar       Haar wavelet l1 prior (eq. sirtista) and its local FISTA

Every function is pinned by tests in tests/test_oracle_*.py against facts the paper
or mathematics fixes (adjoint identity between two independent projector codes,
dense brute force, closed-form disc chords, the Ram-Lak frequency response, an
independent ADMM minimiser, ...).  Parity unpinned: none of the numerical
functions; the phantom/noise generator (`synth`) is input data, not oracle.
"""

from .geometry import Geometry, make_geometry, roi_extend, band_exact
from .projector import (hat_weight, fp_ray, bp_pixel, sparse_local, dense_matrix_hat,
                        dense_matrix_ray)
from .fbp import ramlak_taps, ramp_filter, fbp_ramlak
from .tv import grad, div, tv_iso, tv_aniso
from .solvers import (cp_tv_nonneg, sirt_nonneg, power_norm_sq, cp_objective, cp_steps)
from .local import exterior_subtract, local_solve, crop, stitch
from .filters import (sirt_filters, filter_centres, filter_apply, fbp_filter, sirt_iterates,
                      local_method_box)
from .fista import fgp, local_fista_tv, prox_weight
from .preprocess import disc_image, disc_value, disc_subtract, disc_add, pad_truncated
from .haar import haar_forward, haar_inverse, haar_prox, local_fista_haar

__all__ = [
    "Geometry", "make_geometry", "roi_extend", "band_exact", "hat_weight", "fp_ray",
    "bp_pixel", "sparse_local", "dense_matrix_hat", "dense_matrix_ray", "ramlak_taps",
    "ramp_filter", "fbp_ramlak", "grad", "div", "tv_iso", "tv_aniso", "cp_tv_nonneg",
    "sirt_nonneg", "power_norm_sq", "cp_objective", "cp_steps", "exterior_subtract",
    "local_solve", "crop", "stitch", "sirt_filters", "filter_centres", "filter_apply",
    "fbp_filter", "sirt_iterates", "local_method_box", "fgp", "local_fista_tv", "prox_weight",
    "disc_image", "disc_value", "disc_subtract", "disc_add", "pad_truncated", "haar_forward",
    "haar_inverse", "haar_prox", "local_fista_haar",
]
