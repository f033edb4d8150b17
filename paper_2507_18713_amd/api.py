"""Python binding of the renderer: torch tensors supply device memory, torch streams supply the
HIP stream, and every call goes through the C ABI of libsalf.so (see include/salf.h).
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Dict, Iterable, Optional

import numpy as np
import torch

from . import _lib
from ._lib import call

OUTPUT_NAMES = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
FIELDS = {"corner": _lib.FIELD_CORNER, "paper": _lib.FIELD_PAPER, "sdf": _lib.FIELD_SDF}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_dev(t: torch.Tensor, dtype, device, name, shape=None):
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on {device}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Context:
    """A libsalf context bound to one HIP device (one per device per process)."""
    _cache: Dict[int, "Context"] = {}

    def __init__(self, device_index: int):
        h = C.c_void_p()
        call("salf_create", int(device_index), C.byref(h))
        self.handle = h
        self.device = torch.device("cuda", device_index)

    @classmethod
    def get(cls, device=None) -> "Context":
        idx = torch.device(device if device is not None else "cuda").index
        idx = torch.cuda.current_device() if idx is None else idx
        if idx not in cls._cache:
            cls._cache[idx] = Context(idx)
        return cls._cache[idx]

    def sync(self):
        """Synchronize the current stream; raises SalfError (TRUNCATED) if a ray of an earlier
        launch ran out of its traversal step budget."""
        call("salf_sync", self.handle, _stream(self.device))

    def set_step_budget(self, steps: int):
        """Walk steps a ray may take before it is cut short (default 2^22)."""
        call("salf_set_step_budget", self.handle, int(steps))


def sensor_struct(s: dict) -> _lib.Sensor:
    """salf_sensor from a sensor description dict (keys as in the C struct)."""
    st = _lib.Sensor()
    for k in ("model", "width", "height"):
        setattr(st, k, int(s[k]))
    for k in ("fx", "fy", "cx", "cy", "max_theta", "elev_min", "elev_max", "az0", "t0", "dt_line", "t_near"):
        setattr(st, k, float(s.get(k, 0.0)))
    st.t_far = float(s.get("t_far", math.inf))
    for k, n in (("R0", 9), ("p0", 3), ("v", 3), ("w", 3)):
        vals = np.asarray(s.get(k, np.eye(3).ravel() if k == "R0" else np.zeros(n)), np.float64).reshape(n)
        getattr(st, k)[:] = [float(x) for x in vals]
    return st


# Root cells whose finest voxel level is at most this get a dense leaf index by default (16 KiB
# per such cell at level 4).
DEFAULT_INDEX_LEVEL = 4


class Scene:
    """A scene registered with libsalf.  Holds the device tensors it borrows (parameters and the
    acceleration-structure workspace) for its lifetime."""

    def __init__(self, voxels: torch.Tensor, geo: torch.Tensor, rgb: Optional[torch.Tensor],
                 intensity: Optional[torch.Tensor], origin, root_size: float, root_dims, max_level: int,
                 field: str = "corner", preactivate: bool = False, index_level: int = DEFAULT_INDEX_LEVEL):
        """preactivate (corner field): store activated corner values at build time; forward
        renders read them (call refresh() after updating the parameters in place).
        index_level: root cells whose finest voxel level is at most this get a dense leaf index
        (0: octree walk only); see build_index()."""
        dev = geo.device
        self.ctx = Context.get(dev)
        n = int(voxels.shape[0])
        _check_dev(voxels, torch.int32, dev, "voxels", (n, 4))
        _check_dev(geo, torch.float32, dev, "geo", (n, 8))
        if rgb is not None:
            _check_dev(rgb, torch.float32, dev, "rgb", (n, 3, 8))
        if intensity is not None:
            _check_dev(intensity, torch.float32, dev, "intensity", (n, 8))
        d = _lib.SceneDesc()
        d.origin[:] = [float(x) for x in origin]
        d.root_size = float(root_size)
        d.root_dims[:] = [int(x) for x in root_dims]
        d.max_level = int(max_level)
        d.field = FIELDS[field]
        d.flags = _lib.SCENE_PREACTIVATE if preactivate else 0
        nbytes = C.c_size_t()
        call("salf_scene_workspace_size", C.byref(d), n, C.byref(nbytes))
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=dev)
        sid = C.c_int32()

        def chan(t):  # an empty tensor has no storage; any non-NULL pointer declares the channel
            if t is None:
                return None
            return _ptr(t) if t.numel() else _ptr(self.workspace)

        call("salf_scene_create", self.ctx.handle, C.byref(d), n, _ptr(voxels), _ptr(geo), chan(rgb), chan(intensity),
             _ptr(self.workspace), int(self.workspace.numel()), _stream(dev), C.byref(sid))
        self.id = int(sid.value)
        self.desc = d
        self.device = dev
        self.n = n
        self.field = field
        self.preactivate = preactivate
        self.geo, self.rgb, self.intensity = geo, rgb, intensity
        self._voxels = voxels
        self.index = None
        self.index_level = 0
        if index_level:
            self.build_index(index_level)

    def build_index(self, max_level: int):
        """(Re)build the dense leaf index for root cells whose finest level is <= max_level (0 drops
        it).  Blocks until built; call it when no render of this scene is in flight."""
        nbytes = C.c_size_t()
        call("salf_scene_index_size", self.ctx.handle, self.id, int(max_level), C.byref(nbytes))
        if max_level == 0:
            call("salf_scene_build_index", self.ctx.handle, self.id, 0, None, 0, _stream(self.device))
            self.index, self.index_level = None, 0
            return
        buf = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        call("salf_scene_build_index", self.ctx.handle, self.id, int(max_level), _ptr(buf), int(buf.numel()),
             _stream(self.device))
        self.index, self.index_level = buf, int(max_level)

    def refresh(self):
        """Re-derive the stored activated corner values from the parameters (pre-activated scenes)."""
        call("salf_scene_refresh", self.ctx.handle, self.id, _stream(self.device))

    @classmethod
    def from_data(cls, data, device="cuda", field: str = "corner", rgb: bool = True, intensity: bool = True,
                  requires_grad: bool = False, preactivate: bool = False,
                  index_level: int = None) -> "Scene":
        """Upload a scene given as numpy arrays (attributes origin, root_size, root_dims, max_level,
        voxels [N,4] int32, z_geo [N,8], z_rgb [N,3,8], z_int [N,8] or None)."""
        dev = torch.device(device)

        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt).contiguous()

        vox = up(data.voxels, torch.int32)
        geo = up(data.z_geo, torch.float32)
        col = up(data.z_rgb, torch.float32) if (rgb and data.z_rgb is not None) else None
        ity = up(data.z_int, torch.float32) if (intensity and data.z_int is not None) else None
        if requires_grad:
            for t in (geo, col, ity):
                if t is not None:
                    t.requires_grad_(True)
        return cls(vox, geo, col, ity, data.origin, data.root_size, data.root_dims, data.max_level, field,
                   preactivate, DEFAULT_INDEX_LEVEL if index_level is None else index_level)

    def refine(self, grad_rgb: Optional[torch.Tensor], grad_threshold: float, alpha_min: float = 1e-3) -> dict:
        """Densify and prune (Sec. 3.3; salf_refine): voxels whose edge opacity is below
        alpha_min are dropped, voxels whose colour-field gradient (L1) exceeds grad_threshold are
        split into 8 children carrying their field, the rest kept.  Returns the new scene's device
        arrays {voxels, geo, rgb, intensity} (build it with Scene(...))."""
        dev = self.device
        if grad_rgb is not None:
            _check_dev(grad_rgb, torch.float32, dev, "grad_rgb", (self.n, 3, 8))
        opts = _lib.RefineOpts(float(grad_threshold), float(alpha_min))
        wb = C.c_size_t()
        call("salf_refine_work_size", self.n, C.byref(wb))
        work = torch.empty(max(int(wb.value), 256), dtype=torch.uint8, device=dev)
        n_out = C.c_int64()
        g = _ptr(grad_rgb) if grad_rgb is not None else None
        st = _lib.lib().salf_refine(self.ctx.handle, self.id, _ptr(self._voxels), g, C.byref(opts), _ptr(work),
                                    int(work.numel()), None, None, None, None, 0, C.byref(n_out), _stream(dev))
        if st not in (0, _lib.ERR_OUT_OF_MEMORY):
            call("salf_refine", self.ctx.handle, self.id, _ptr(self._voxels), g, C.byref(opts), _ptr(work),
                 int(work.numel()), None, None, None, None, 0, C.byref(n_out), _stream(dev))
        m = int(n_out.value)
        out = {"voxels": torch.empty((m, 4), dtype=torch.int32, device=dev),
               "geo": torch.empty((m, 8), dtype=torch.float32, device=dev),
               "rgb": torch.empty((m, 3, 8), dtype=torch.float32, device=dev) if self.rgb is not None else None,
               "intensity": torch.empty((m, 8), dtype=torch.float32, device=dev) if self.intensity is not None else None}
        if m > 0:
            call("salf_refine", self.ctx.handle, self.id, _ptr(self._voxels), g, C.byref(opts), _ptr(work),
                 int(work.numel()), _ptr(out["voxels"]), _ptr(out["geo"]),
                 _ptr(out["rgb"]) if out["rgb"] is not None else None,
                 _ptr(out["intensity"]) if out["intensity"] is not None else None, m, C.byref(n_out), _stream(dev))
        return out

    def stats(self) -> dict:
        s = _lib.SceneStats()
        call("salf_scene_get_stats", self.ctx.handle, self.id, C.byref(s))
        return {k: int(getattr(s, k)) for k, _ in _lib.SceneStats._fields_}

    def destroy(self):
        if self.id >= 0:
            call("salf_scene_destroy", self.ctx.handle, self.id)
            self.id = -1

    def __del__(self):
        try:
            if getattr(self, "id", -1) >= 0 and _lib._lib is not None:
                _lib.lib().salf_scene_destroy(self.ctx.handle, self.id)
        except Exception:
            pass


def ray_count(sensor: dict) -> int:
    n = C.c_int64()
    call("salf_sensor_ray_count", C.byref(sensor_struct(sensor)), C.byref(n))
    return int(n.value)


def generate_rays(sensor: dict, device="cuda") -> Dict[str, torch.Tensor]:
    """Materialize a sensor's rays on the GPU: o [n,3], d [n,3], t [n] (float32), valid [n] (uint8)."""
    dev = torch.device(device)
    ctx = Context.get(dev)
    n = ray_count(sensor)
    o = torch.empty((n, 3), dtype=torch.float32, device=dev)
    d = torch.empty((n, 3), dtype=torch.float32, device=dev)
    t = torch.empty(n, dtype=torch.float32, device=dev)
    v = torch.empty(n, dtype=torch.uint8, device=dev)
    call("salf_generate_rays", ctx.handle, C.byref(sensor_struct(sensor)), _ptr(o), _ptr(d), _ptr(t), _ptr(v),
         _stream(dev))
    return {"o": o, "d": d, "t": t, "valid": v}


def _opts(samples, t_min, background, work: Optional[torch.Tensor] = None,
          mode: int = _lib.SCHEDULE_NONE, pieces: int = 1) -> _lib.RenderOpts:
    op = _lib.RenderOpts()
    op.samples_per_voxel = int(samples)
    op.t_min = float(t_min)
    op.background[:] = [float(x) for x in background]
    op.schedule = int(mode) if work is not None else _lib.SCHEDULE_NONE
    op.d_work = work.data_ptr() if work is not None else None
    op.work_bytes = work.numel() if work is not None else 0
    op.pieces = int(pieces)
    op.reserved = 0
    return op


def _schedule_work(sen, rays, dev) -> torch.Tensor:
    """An uninitialized schedule buffer for one launch layout (from torch's stream-ordered
    allocator, so launches on other streams never share it)."""
    n = C.c_size_t()
    call("salf_render_work_size", C.byref(sen) if sen is not None else None,
         C.byref(rays) if rays is not None else None, C.byref(n))
    return torch.empty(int(n.value), dtype=torch.uint8, device=dev)


def _schedule_args(schedule, sen, rays, dev):
    """(buffer, mode) for the schedule argument of render / render_backward: True builds a
    schedule in a fresh buffer during the call, a tensor from render_schedule is reused, False
    renders tiles in index order."""
    if isinstance(schedule, torch.Tensor):
        return schedule, _lib.SCHEDULE_REUSE
    if schedule:
        return _schedule_work(sen, rays, dev), _lib.SCHEDULE_BUILD
    return None, _lib.SCHEDULE_NONE


def render_schedule(scene: "Scene", sensor: Optional[dict] = None, o: Optional[torch.Tensor] = None,
                    d: Optional[torch.Tensor] = None, t_near: float = 0.0, t_far: float = math.inf,
                    image_width: int = 0) -> torch.Tensor:
    """Build the heaviest-tiles-first schedule of a render of `sensor` (or explicit rays) on
    `scene` and return its buffer; pass it as `schedule=` to render / render_backward to reuse it
    for renders with the same ray layout."""
    dev = scene.device
    sen = rays = None
    if sensor is not None:
        sen = sensor_struct(sensor)
    else:
        rays = _rays_struct(o, d, t_near, t_far, dev, image_width)
    work = _schedule_work(sen, rays, dev)
    call("salf_render_schedule", scene.ctx.handle, scene.id, C.byref(sen) if sen is not None else None,
         C.byref(rays) if rays is not None else None, C.byref(_opts(4, 1e-6, (0.0, 0.0, 0.0), work)), _stream(dev))
    return work


def _rays_struct(o, d, t_near, t_far, device, image_width=0):
    _check_dev(o, torch.float32, device, "o")
    _check_dev(d, torch.float32, device, "d")
    if o.shape != d.shape or o.dim() != 2 or o.shape[1] != 3:
        raise ValueError("o and d must both be [n, 3]")
    r = _lib.Rays()
    r.o = o.data_ptr()
    r.d = d.data_ptr()
    r.n = int(o.shape[0])
    r.t_near = float(t_near)
    r.t_far = float(t_far)
    r.image_width = int(image_width)
    r.reserved = 0
    return r


def render(scene: Scene, sensor: Optional[dict] = None, o: Optional[torch.Tensor] = None,
           d: Optional[torch.Tensor] = None, samples: int = 4, t_min: float = 1e-6, background=(0.0, 0.0, 0.0),
           outputs: Iterable[str] = ("rgb", "depth", "opacity"), t_near: float = 0.0, t_far: float = math.inf,
           out: Optional[Dict[str, torch.Tensor]] = None, image_width: int = 0,
           schedule=True, pieces: int = 1, hit_capacity: int = 0) -> Dict[str, torch.Tensor]:
    """Render a sensor (ray generation fused) or explicit rays (o, d float32 [n, 3]).
    image_width > 0 declares explicit rays to be a row-major image of that width (tiled launch).
    schedule: True builds a heaviest-tiles-first schedule in the call, a buffer from
    render_schedule reuses one, False keeps tile order, "static" builds it in the library's own
    per-device array (salf_render_static: no schedule memory is allocated; calls on one device
    must not overlap).  The outputs are the same bits in every case.
    pieces: lanes per ray (1; or 2, 4, 8: each ray's occupied root cells are shared out among that
    many lanes and their partial results folded front to back; the same hits, outputs equal to
    the one-lane render's up to FP32 rounding).
    hit_capacity > 0 also stores each ray's composited hits, at most that many per ray:
    "hit_voxel" int32 [hit_capacity, n] and "hit_t" float32 [hit_capacity, n, 2] (t_in, t_out),
    hit k of ray r at [k, r]; render_backward then reads them instead of walking the scene again.
    Returns a dict with the requested outputs (rgb [n,3]; depth, opacity, intensity, t_end [n];
    n_hits int32 [n])."""
    dev = scene.device
    outputs = tuple(outputs)
    for k in outputs:
        if k not in OUTPUT_NAMES:
            raise ValueError(f"unknown output {k}")
    sen = rays = None
    if sensor is not None:
        sen = sensor_struct(sensor)
        n = ray_count(sensor)
    else:
        rays = _rays_struct(o, d, t_near, t_far, dev, image_width)
        n = int(rays.n)
    res = {} if out is None else dict(out)
    for k in outputs:
        if k not in res:
            shape = (n, 3) if k == "rgb" else (n,)
            res[k] = torch.empty(shape, dtype=torch.int32 if k == "n_hits" else torch.float32, device=dev)
    ob = _lib.Outputs()
    for k in OUTPUT_NAMES:
        setattr(ob, k, res[k].data_ptr() if k in res else None)
    if hit_capacity > 0:
        cap = int(hit_capacity)
        res["hit_voxel"] = torch.empty((cap, n), dtype=torch.int32, device=dev)
        res["hit_t"] = torch.empty((cap, n, 2), dtype=torch.float32, device=dev)
        ob.hit_voxel, ob.hit_t, ob.hit_capacity = res["hit_voxel"].data_ptr(), res["hit_t"].data_ptr(), cap
    if isinstance(schedule, str):
        if schedule != "static":
            raise ValueError(f"unknown schedule {schedule!r}")
        call("salf_render_static", scene.ctx.handle, scene.id, C.byref(sen) if sen is not None else None,
             C.byref(rays) if rays is not None else None, C.byref(_opts(samples, t_min, background, pieces=pieces)),
             C.byref(ob), _stream(dev))
        return res
    work, mode = _schedule_args(schedule, sen, rays, dev)
    call("salf_render", scene.ctx.handle, scene.id, C.byref(sen) if sen is not None else None,
         C.byref(rays) if rays is not None else None, C.byref(_opts(samples, t_min, background, work, mode, pieces)),
         C.byref(ob), _stream(dev))
    return res


_MULTI_WORK: Dict[tuple, torch.Tensor] = {}


def render_multi(items, samples: int = 4, t_min: float = 1e-6, background=(0.0, 0.0, 0.0),
                 work: Optional[torch.Tensor] = None):
    """Render several sensors in one launch (salf_render_multi): items is a list of (scene, sensor,
    outputs) where outputs is a tuple of output names or a dict of preallocated tensors.  Returns a
    list of output dicts, each the same bits as render() of that item."""
    if not items:
        return []
    dev = items[0][0].device
    ctx = items[0][0].ctx
    arr = (_lib.RenderItem * len(items))()
    keep, results = [], []
    for i, (scene, sensor, outputs) in enumerate(items):
        n = ray_count(sensor)
        res = dict(outputs) if isinstance(outputs, dict) else {}
        for k in (outputs.keys() if isinstance(outputs, dict) else outputs):
            if k not in OUTPUT_NAMES:
                raise ValueError(f"unknown output {k}")
            if k not in res:
                shape = (n, 3) if k == "rgb" else (n,)
                res[k] = torch.empty(shape, dtype=torch.int32 if k == "n_hits" else torch.float32, device=dev)
        sen = sensor_struct(sensor)
        keep.append(sen)
        arr[i].scene_id = scene.id
        arr[i].reserved = 0
        arr[i].sensor = C.pointer(sen)
        arr[i].opts = _opts(samples, t_min, background)
        for k in OUTPUT_NAMES:
            setattr(arr[i].out, k, res[k].data_ptr() if k in res else None)
        results.append(res)
    if work is None:
        nb = C.c_size_t()
        call("salf_render_multi_work_size", len(items), C.byref(nb))
        key = (dev.index, len(items), torch.cuda.current_stream(dev).cuda_stream)
        work = _MULTI_WORK.get(key)
        if work is None or work.numel() < int(nb.value):
            work = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
            _MULTI_WORK[key] = work
    call("salf_render_multi", ctx.handle, len(items), arr, _ptr(work), int(work.numel()), _stream(dev))
    return results


def render_raster(scene: Scene, sensor: dict, samples: int = 4, t_min: float = 1e-6, background=(0.0, 0.0, 0.0),
                  outputs: Iterable[str] = ("rgb", "depth", "opacity"), out: Optional[Dict[str, torch.Tensor]] = None,
                  work: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
    """Render a global-shutter pinhole `sensor` by tile-based splatting (salf_render_raster): the
    same outputs, bit for bit, as render() of the sensor.  The call blocks once (it reads the
    frame's (voxel, tile) pair count back); the work area is kept on the scene and grown as frames
    need.  `work` overrides it."""
    dev = scene.device
    outputs = tuple(outputs)
    for k in outputs:
        if k not in OUTPUT_NAMES:
            raise ValueError(f"unknown output {k}")
    sen = sensor_struct(sensor)
    n = ray_count(sensor)
    res = {} if out is None else dict(out)
    for k in outputs:
        if k not in res:
            shape = (n, 3) if k == "rgb" else (n,)
            res[k] = torch.empty(shape, dtype=torch.int32 if k == "n_hits" else torch.float32, device=dev)
    ob = _lib.Outputs()
    for k in OUTPUT_NAMES:
        setattr(ob, k, res[k].data_ptr() if k in res else None)
    opts = _opts(samples, t_min, background)
    pairs = C.c_int64()
    for attempt in range(2):
        buf = work if work is not None else getattr(scene, "_raster_work", None)
        if buf is None:
            nb = C.c_size_t()
            call("salf_raster_work_size", scene.ctx.handle, scene.id, C.byref(sen),
                 max(4 * scene.n, 1 << 16) if attempt == 0 else int(pairs.value * 1.25) + 1024, C.byref(nb))
            buf = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
            if work is None:
                scene._raster_work = buf
        st = _lib.lib().salf_render_raster(scene.ctx.handle, scene.id, C.byref(sen), C.byref(opts), C.byref(ob),
                                           _ptr(buf), int(buf.numel()), C.byref(pairs), _stream(dev))
        if st == _lib.ERR_OUT_OF_MEMORY and work is None and attempt == 0:
            scene._raster_work = None
            continue
        if st != _lib.SALF_OK:
            msg = _lib.lib().salf_last_error()
            raise _lib.SalfError(st, "salf_render_raster", msg.decode() if msg else "")
        break
    scene.raster_pairs = int(pairs.value)
    return res


def render_composite(scene: Scene, actors, sensor: Optional[dict] = None, o: Optional[torch.Tensor] = None,
                     d: Optional[torch.Tensor] = None, samples: int = 4, t_min: float = 1e-6,
                     background=(0.0, 0.0, 0.0), outputs: Iterable[str] = ("rgb", "depth", "opacity"),
                     t_near: float = 0.0, t_far: float = math.inf, image_width: int = 0,
                     schedule=True) -> Dict[str, torch.Tensor]:
    """Render a static scene with dynamic actors (salf_render_composite): actors is a list of
    (Scene, R [3, 3], t [3]), a world point p being the actor point R^T (p - t).  Other arguments
    and the result as render()."""
    dev = scene.device
    outputs = tuple(outputs)
    for k in outputs:
        if k not in OUTPUT_NAMES:
            raise ValueError(f"unknown output {k}")
    sen = rays = None
    if sensor is not None:
        sen = sensor_struct(sensor)
        n = ray_count(sensor)
    else:
        rays = _rays_struct(o, d, t_near, t_far, dev, image_width)
        n = int(rays.n)
    res = {}
    for k in outputs:
        shape = (n, 3) if k == "rgb" else (n,)
        res[k] = torch.empty(shape, dtype=torch.int32 if k == "n_hits" else torch.float32, device=dev)
    ob = _lib.Outputs()
    for k in OUTPUT_NAMES:
        setattr(ob, k, res[k].data_ptr() if k in res else None)
    arr = (_lib.Actor * max(len(actors), 1))()
    for i, (sc, R, t) in enumerate(actors):
        arr[i].scene_id = sc.id
        arr[i].R[:] = [float(x) for x in np.asarray(R, np.float32).reshape(9)]
        arr[i].t[:] = [float(x) for x in np.asarray(t, np.float32).reshape(3)]
    work, mode = _schedule_args(schedule, sen, rays, dev)
    call("salf_render_composite", scene.ctx.handle, scene.id, len(actors), arr,
         C.byref(sen) if sen is not None else None, C.byref(rays) if rays is not None else None,
         C.byref(_opts(samples, t_min, background, work, mode)), C.byref(ob), _stream(dev))
    return res


def trace_hits(scene: Scene, o: torch.Tensor, d: torch.Tensor, max_hits: int, t_near: float = 0.0,
               t_far: float = math.inf, early_termination: bool = False, samples: int = 4, t_min: float = 1e-6):
    """Voxels hit by each ray, front to back: counts [n] and ids/t_in/t_out [n, max_hits]
    (entries past a ray's count are -1 / NaN).  early_termination: stop each ray after the voxel
    that leaves T < t_min with `samples` samples per voxel, as a render does (counts then equal the
    render's n_hits)."""
    dev = scene.device
    rays = _rays_struct(o, d, t_near, t_far, dev)
    n = int(rays.n)
    counts = torch.empty(n, dtype=torch.int32, device=dev)
    ids = torch.full((n, max_hits), -1, dtype=torch.int32, device=dev)
    ti = torch.full((n, max_hits), float("nan"), dtype=torch.float32, device=dev)
    to = torch.full((n, max_hits), float("nan"), dtype=torch.float32, device=dev)
    call("salf_trace_hits", scene.ctx.handle, scene.id, C.byref(rays), int(max_hits), int(bool(early_termination)),
         C.byref(_opts(samples, t_min, (0.0, 0.0, 0.0))), _ptr(counts), _ptr(ids), _ptr(ti), _ptr(to), _stream(dev))
    return counts, ids, ti, to


def render_backward(scene: Scene, saved: Dict[str, torch.Tensor], grads: Dict[str, Optional[torch.Tensor]],
                    sensor: Optional[dict] = None, o=None, d=None, samples: int = 4, t_min: float = 1e-6,
                    background=(0.0, 0.0, 0.0), t_near: float = 0.0, t_far: float = math.inf,
                    d_geo=None, d_rgb=None, d_int=None, image_width: int = 0, schedule=True):
    """Accumulate dL/d(params) of a render (corner or paper field) into d_geo/d_rgb/d_int (allocated
    zeroed if None and the scene has that parameter).  `saved` holds the forward's outputs, with
    its "hit_voxel" / "hit_t" if the forward stored hits (then those rays are not walked again).
    Returns (d_geo, d_rgb, d_int)."""
    dev = scene.device
    if d_geo is None:
        d_geo = torch.zeros_like(scene.geo, memory_format=torch.contiguous_format)
    if d_rgb is None and scene.rgb is not None and grads.get("rgb") is not None:
        d_rgb = torch.zeros_like(scene.rgb, memory_format=torch.contiguous_format)
    if d_int is None and scene.intensity is not None and grads.get("intensity") is not None:
        d_int = torch.zeros_like(scene.intensity, memory_format=torch.contiguous_format)
    sen = rays = None
    if sensor is not None:
        sen = sensor_struct(sensor)
    else:
        rays = _rays_struct(o, d, t_near, t_far, dev, image_width)
    sv = _lib.Outputs()
    for k in OUTPUT_NAMES:
        t = saved.get(k)
        setattr(sv, k, t.data_ptr() if t is not None else None)
    if saved.get("hit_voxel") is not None:
        hv, ht = saved["hit_voxel"], saved["hit_t"]
        if hv.dim() != 2 or tuple(ht.shape) != (hv.shape[0], hv.shape[1], 2):
            raise ValueError("hit_voxel [cap, n] and hit_t [cap, n, 2] expected")
        sv.hit_voxel, sv.hit_t, sv.hit_capacity = hv.data_ptr(), ht.data_ptr(), int(hv.shape[0])
    g = _lib.GradsIn()
    for k, f in (("rgb", "d_rgb"), ("depth", "d_depth"), ("opacity", "d_opacity"), ("intensity", "d_intensity")):
        t = grads.get(k)
        if t is not None:
            t = t.contiguous()
            grads[k] = t
        setattr(g, f, t.data_ptr() if t is not None else None)
    work, mode = _schedule_args(schedule, sen, rays, dev)
    call("salf_render_backward", scene.ctx.handle, scene.id, C.byref(sen) if sen is not None else None,
         C.byref(rays) if rays is not None else None, C.byref(_opts(samples, t_min, background, work, mode)),
         C.byref(sv),
         C.byref(g), _ptr(d_geo), _ptr(d_rgb), _ptr(d_int), _stream(dev))
    return d_geo, d_rgb, d_int


class RenderFunction(torch.autograd.Function):
    """Differentiable render (corner or paper field).  apply(geo, rgb, intensity, scene, sensor, o, d, opts) ->
    (rgb, depth, opacity, intensity); geo/rgb/intensity must be the scene's own parameter
    tensors (the render reads them in place).  rgb/intensity outputs are empty tensors when the
    scene lacks that parameter.  opts may hold hit_capacity > 0: the forward then stores up to that
    many hits per ray and the backward reads them instead of walking the scene again."""

    @staticmethod
    def forward(ctx, geo, rgb, intensity, scene: Scene, sensor, o, d, opts: dict):
        want = ["depth", "opacity", "t_end", "n_hits"]
        if rgb is not None:
            want.append("rgb")
        if intensity is not None:
            want.append("intensity")
        cap = int(opts.get("hit_capacity", 0))
        ropts = {k: v for k, v in opts.items() if k != "hit_capacity"}
        res = render(scene, sensor=sensor, o=o, d=d, outputs=want, hit_capacity=cap, **ropts)
        ctx.scene, ctx.sensor, ctx.o, ctx.d, ctx.opts = scene, sensor, o, d, ropts
        empty = torch.empty(0, device=geo.device)
        outs = (res.get("rgb", empty), res["depth"], res["opacity"], res.get("intensity", empty))
        hits = (res["hit_voxel"], res["hit_t"]) if cap > 0 else (empty, empty)
        # the backward reads the parameters in place and the forward's outputs (its suffix sums are
        # formed from them), so both go through autograd's saved-tensor version checks: an in-place
        # change of either before backward raises instead of corrupting the gradient
        ctx.save_for_backward(geo, rgb, intensity, *outs, res["t_end"], res["n_hits"], *hits)
        return outs

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_opacity, g_int):
        sc = ctx.scene
        _, _, _, o_rgb, o_depth, o_opacity, o_int, t_end, n_hits, hit_voxel, hit_t = ctx.saved_tensors
        saved = {"depth": o_depth, "opacity": o_opacity, "t_end": t_end, "n_hits": n_hits}
        if hit_voxel.numel():
            saved["hit_voxel"], saved["hit_t"] = hit_voxel, hit_t
        if o_rgb.numel():
            saved["rgb"] = o_rgb
        if o_int.numel():
            saved["intensity"] = o_int
        grads = {"rgb": g_rgb if sc.rgb is not None and g_rgb is not None and g_rgb.numel() else None,
                 "depth": g_depth, "opacity": g_opacity,
                 "intensity": g_int if sc.intensity is not None and g_int is not None and g_int.numel() else None}
        dg, dr, di = render_backward(sc, saved, grads, sensor=ctx.sensor, o=ctx.o, d=ctx.d, **ctx.opts)
        return dg, dr, di, None, None, None, None, None


_OUT_BITS = {"rgb": 1, "depth": 2, "opacity": 4, "intensity": 8}


class Server:
    """Continuous-batching render server (salf_server_*).  Outputs of admitted requests are carved
    from a device pool of `pool_bytes` (the HBM budget); results are views into that pool, valid
    until release().  max_launch_rays > 0 caps the rays of one launch (a request completes with
    its launch, so smaller launches complete small sensors sooner); 0 = no cap."""

    def __init__(self, pool_bytes: int, device="cuda", max_batch: int = 64, max_inflight: int = 2,
                 max_launch_rays: int = 0):
        dev = torch.device(device)
        self.ctx = Context.get(dev)
        self.device = dev
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=dev)
        op = _lib.ServerOpts()
        op.d_pool = self.pool.data_ptr()
        op.pool_bytes = int(pool_bytes)
        op.max_batch = int(max_batch)
        op.max_inflight = int(max_inflight)
        op.max_launch_rays = int(max_launch_rays)
        nbytes = C.c_size_t()
        call("salf_server_work_size", C.byref(op), C.byref(nbytes))
        self.work = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=dev)
        op.d_work = self.work.data_ptr()
        op.work_bytes = int(self.work.numel())
        torch.cuda.synchronize(dev)
        h = C.c_void_p()
        call("salf_server_create", self.ctx.handle, C.byref(op), C.byref(h))
        self.handle = h
        self._meta = {}

    @staticmethod
    def request_bytes(sensor: dict, outputs=("rgb", "depth", "opacity")) -> int:
        n = C.c_size_t()
        mask = sum(_OUT_BITS[k] for k in outputs)
        call("salf_server_request_bytes", C.byref(sensor_struct(sensor)), mask, C.byref(n))
        return int(n.value)

    def submit(self, scene: Scene, sensor: dict, outputs=("rgb", "depth", "opacity"), samples: int = 4,
               t_min: float = 1e-6, background=(0.0, 0.0, 0.0)) -> int:
        """Queue a render (on the server's own streams: synchronize the stream of any pending change
        to the scene first).  The scene's device buffers are held until release(), so dropping the
        Scene (or rebuilding its index) while the request is in flight cannot free memory the kernel
        reads."""
        t = C.c_uint64()
        mask = sum(_OUT_BITS[k] for k in outputs)
        call("salf_server_submit", self.handle, scene.id, C.byref(sensor_struct(sensor)),
             C.byref(_opts(samples, t_min, background)), mask, C.byref(t))
        held = (scene, scene.workspace, scene.index, scene.geo, scene.rgb, scene.intensity)
        self._meta[int(t.value)] = (tuple(outputs), int(sensor["width"]) * int(sensor["height"]), held)
        return int(t.value)

    def poll(self, ticket: int):
        """None while running; else (outputs dict of tensors viewing the pool, t_submit, t_done)."""
        done = C.c_int32()
        ob = _lib.Outputs()
        ts, td = C.c_double(), C.c_double()
        call("salf_server_poll", self.handle, C.c_uint64(ticket), C.byref(done), C.byref(ob), C.byref(ts),
             C.byref(td))
        if not done.value:
            return None
        outs, n, _ = self._meta[ticket]
        base = self.pool.data_ptr()
        res = {}
        for k in outs:
            off = getattr(ob, k) - base
            cnt = n * 3 if k == "rgb" else n
            v = self.pool.narrow(0, off, cnt * 4).view(torch.float32)
            res[k] = v.view(n, 3) if k == "rgb" else v
        return res, ts.value, td.value

    def wait(self, ticket: int, timeout: float = 60.0) -> bool:
        done = C.c_int32()
        call("salf_server_wait", self.handle, C.c_uint64(ticket), C.c_double(timeout), C.byref(done))
        return bool(done.value)

    def release(self, ticket: int):
        call("salf_server_release", self.handle, C.c_uint64(ticket))
        self._meta.pop(ticket, None)

    def stats(self) -> dict:
        s = _lib.ServerStats()
        call("salf_server_get_stats", self.handle, C.byref(s))
        return {k: int(getattr(s, k)) for k, _ in _lib.ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None:
            call("salf_server_destroy", self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
