"""FP64 CPU oracle of the Gaussian-enhanced-surfel render (test infrastructure).

Only `tests/`, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP path and imports nothing from it.
"""
from .render import (Options, SURFEL_RADIUS, render, ambiguous, gradients, finite_difference,
                     gaussian_projection, surfel_frames, gaussian_candidates, surfel_candidates,
                     rect_pixels, Cam, quat_to_rot, scores, geometry, gaussian_normals, facing,
                     mip_filter3d)
from .sh import sh_basis, sh_colour
from .translucent import translucent_render, translucent_gradients, translucent_fd
from .gs2d import render_2dges, gauss2d_frames, gauss2d_pass, eps_2d
