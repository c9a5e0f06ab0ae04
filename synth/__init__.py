"""Seeded synthetic inputs for the local-ROI tomography library.

This package only *generates data*: random-ellipse phantoms, their exact
(analytic) line integrals, measurement noise and random ROI/request lists.
It holds none of the reconstruction arithmetic (no projector, no filter, no
solver), so both the FP64 oracle and the HIP path can consume its arrays
without sharing any method code.

Shared conventions (parallel-beam geometry, pixel units):
  * image pixel (r, c) of an N x N grid has centre x = c - (N-1)/2, y = r - (N-1)/2;
  * detector bin i has centre s_i = (i - (N_d-1)/2) * spacing + offset;
  * angle k is theta_k = k * pi / N_theta (uniform in [0, pi));
  * a ray is the line {x cos(theta) + y sin(theta) = s}.
"""

from .phantom import (Ellipses, random_ellipses, texture_ellipses, concat_ellipses,
                      raster, analytic_sinogram, add_gaussian_noise, add_poisson_noise,
                      disc_sinogram, angles_uniform, bin_centres)
from .configs import WORKLOADS, workload, make_inputs, make_slices, roi_list, serving_requests

__all__ = [
    "Ellipses", "random_ellipses", "texture_ellipses", "concat_ellipses", "raster",
    "analytic_sinogram", "add_gaussian_noise", "add_poisson_noise", "disc_sinogram",
    "angles_uniform", "bin_centres", "WORKLOADS", "workload", "make_inputs", "roi_list",
    "serving_requests", "make_slices",
]
