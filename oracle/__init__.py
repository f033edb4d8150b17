"""Reference renderer for sparse local fields — TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct CPU implementation of what the
ray-casting renderer computes (Sec. 3.1 "Representation", Eq. 1-4, and the
octree ray casting paragraph of Sec. 3.2), and of the tile-based splatting of
the same voxels (Sec. 3.2 "Tile-based Splatting").  It exists to check the HIP renderer:
only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import it.  The renderer itself never imports, links or calls it, and it
shares no code with the renderer (only the seeded input generators in `synth`).

Layout:
  hitspec   FP32 ray/voxel interval rule, brute force over every voxel
  field     local field evaluation (corner-interpolated mode, the paper's Eq. 1-2 and Eq. 5-6)
  render    samples, compositing (Eq. 3-4) with early termination, per-ray outputs
  grad      analytic gradient of the composited outputs w.r.t. the raw field parameters
  refine    densification and pruning of the voxel set (Sec. 3.3)
  composite a static scene with dynamic actors placed by rigid poses (merged traversal)
  raster    tile-based splatting of the voxels onto a pinhole image (Sec. 3.2)
  sensors   pinhole, equidistant fisheye and spinning-LiDAR rays with rolling shutter
Everything downstream of the FP32 hit rule is float64.
"""
from .hitspec import PreparedScene, prepare, ray_frame, box_interval, hit_list, hit_lists
from .field import corner_weights, softplus, sigmoid, corner_field, paper_field, sdf_density, sdf_field, sh_basis
from .render import RenderOpts, render_rays, render_ray
from .grad import grad_rays
from .refine import refine, sigma_max, colour_grad_l1, field_at
from .composite import actor_ray, composite_rays
from .raster import raster, tile_lists, depth_key, footprints
from .sensors import sensor_rays, rodrigues

__all__ = [
    "actor_ray", "composite_rays", "raster", "tile_lists", "depth_key", "footprints",
    "refine", "sigma_max", "colour_grad_l1", "field_at",
    "PreparedScene", "prepare", "ray_frame", "box_interval", "hit_list", "hit_lists",
    "corner_weights", "softplus", "sigmoid", "corner_field", "paper_field", "sdf_density", "sdf_field", "sh_basis",
    "RenderOpts", "render_rays", "render_ray", "grad_rays", "sensor_rays", "rodrigues",
]
