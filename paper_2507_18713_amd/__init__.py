"""MI355X-native ray-casting renderer for sparse local fields (SaLF, arXiv 2507.18713).

The rendering path runs in hand-written HIP kernels behind the C ABI of `libsalf.so`
(include/salf.h); this package only marshals torch tensors and streams into those calls.
Importing it loads the library and fails loudly if it is not built.
"""
from ._lib import SalfError, lib as _load_lib, LIB_PATH
from .api import (Context, Scene, RenderFunction, Server, generate_rays, ray_count, render, render_backward,
                  render_composite, render_multi, render_raster, render_schedule, sensor_struct, trace_hits)

_load_lib()

__all__ = ["SalfError", "LIB_PATH", "Context", "Scene", "RenderFunction", "Server", "generate_rays", "ray_count",
           "render", "render_backward", "render_composite", "render_multi", "render_raster", "render_schedule", "sensor_struct",
           "trace_hits"]
