"""FP64 CPU oracle of the object-centric 2DGS rasterizer hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP
implementation; its inputs are the same float32 arrays the GPU consumes,
promoted exactly to float64.

Modules
  geometry  projection of surfels, culling, conservative pixel rectangles,
            tile ranges, depth keys and the sorted (tile|depth, id) instance
            list (the bit-exact binning specification)
  sh        real spherical harmonics (view-dependent colour)
  render    differentiable per-pixel front-to-back compositing (torch float64)
  loss      background loss (Eq. 1) and the masked photometric L1 (Eq. 2)
  regularizers  the 2DGS depth distortion and normal consistency terms of
            the total loss (Eq. 3)
  ssim      masked SSIM / D-SSIM (the rest of Eq. 2's photometric loss) and
            masked PSNR
  prune     occlusion-aware pruning statistics (Section 4.3)
  prune_native  the same statistics from a plain-C per-pixel loop
            (prune_native.c, built with gcc on first use) for scenes of a
            million surfels over a hundred views
  densify   the screen-space gradient statistic of the density control
  gauss3d   the pruning statistics for 3D Gaussians (Appendix B): EWA
            projection, conservative rectangles, compositing decisions
  fd        central finite differences with decision-set filtering
"""
from .geometry import RasterParams, view_geometry64, bin64, tile_layout, rotation_columns64
from .sh import real_sh_basis, sh_basis_scipy, sh_coeff_count
from .render import render_pixels, render_view, Params64
from .loss import background_loss64, masked_l1_64
from .prune import prune_stats64
from .densify import screen_grad_stats64
from .gauss3d import view_geometry3d64, prune_pixels3d
from .regularizers import regularizer_loss64, depth_normal64, depth_points64, surface_depth64
from .ssim import dssim_loss64, masked_ssim64, masked_psnr64, ssim_map64, gaussian_1d64, window_2d64

__all__ = [
    "RasterParams", "view_geometry64", "bin64", "tile_layout", "rotation_columns64",
    "real_sh_basis", "sh_basis_scipy", "sh_coeff_count",
    "render_pixels", "render_view", "Params64",
    "background_loss64", "masked_l1_64", "prune_stats64", "screen_grad_stats64",
    "view_geometry3d64", "prune_pixels3d",
    "regularizer_loss64", "depth_normal64", "depth_points64", "surface_depth64",
    "dssim_loss64", "masked_ssim64", "masked_psnr64", "ssim_map64", "gaussian_1d64", "window_2d64",
]
