"""Which voxels a ray crosses, and where: the FP32 interval rule, by brute force.

The paper casts each ray through the non-overlapping voxels it intersects
(Sec. 3.2, octree ray casting; voxels do not overlap, Sec. 3.4), and samples each
voxel on its ray segment (Sec. 3.1, text after Eq. 4).  The octree only skips
empty space, so testing every ray against every voxel and sorting the hits by
entry distance yields the same segments.  Segment end points are defined here in
FP32 so that a GPU traversal can reproduce them bit for bit:

  grid frame   og = (o - org) * gs,  dg = d * gs,  inv = 1 / dg   (FP32, each op rounded)
               org = float32(scene origin), gs = float32(2^K / s0) (finest cells per metre)
  per axis a   if dg_a == 0 or inv_a is infinite the axis is *parallel*: the voxel's
               slab is [-inf, +inf] when lo_a <= og_a < hi_a, else the ray misses;
               otherwise t = (P - og_a) * inv_a for the planes P = lo_a, hi_a, and the
               slab is [min, max] of the two.
  interval     t_in = max(t_near, slab starts), t_out = min(t_far, slab ends); a zero t_in
               is +0.  The ray hits the voxel iff t_in < t_out (strictly).
  invalid ray  any non-finite component of o or d, or all three axes parallel: no hits.

lo and hi are the voxel's integer bounds in finest-level cells (exact in FP32).
"""
from __future__ import annotations

import dataclasses

import numpy as np

F32 = np.float32


@dataclasses.dataclass
class PreparedScene:
    scene: object
    org32: np.ndarray      # float32 [3]
    gs32: np.float32       # finest cells per metre, FP32
    origin: np.ndarray     # float64 [3]
    gs: float              # finest cells per metre, float64
    lo_i: np.ndarray       # int64 [N, 3] finest-unit lower bounds
    n_i: np.ndarray        # int64 [N] finest-unit edge length
    lo32: np.ndarray       # float32 [3, N] (axis-major for fast per-axis passes)
    hi32: np.ndarray       # float32 [3, N]


def prepare(scene) -> PreparedScene:
    lo, hi = scene.finest_bounds()
    gs = float(1 << scene.max_level) / float(scene.root_size)
    return PreparedScene(scene=scene, org32=np.asarray(scene.origin, np.float64).astype(F32), gs32=F32(gs),
                         origin=np.asarray(scene.origin, np.float64), gs=gs, lo_i=lo,
                         n_i=(hi[:, 0] - lo[:, 0]), lo32=np.ascontiguousarray(lo.T.astype(F32)),
                         hi32=np.ascontiguousarray(hi.T.astype(F32)))


def ray_frame(o, d, org32, gs32):
    """One ray's grid-frame quantities (FP32): og, dg, inv [3] and the parallel flags."""
    o = np.asarray(o, F32)
    d = np.asarray(d, F32)
    og = (o - org32) * gs32
    dg = d * gs32
    with np.errstate(divide="ignore"):
        inv = F32(1.0) / dg
    par = (dg == F32(0.0)) | np.isinf(inv)
    valid = bool(np.all(np.isfinite(o)) and np.all(np.isfinite(d)) and not np.all(par))
    return og, dg, inv, par, valid


def box_interval(og, inv, par, lo, hi, t_near=0.0, t_far=np.inf):
    """FP32 interval of one ray against M boxes given as float32 [3, M] bounds.
    Returns (t_in, t_out, hit) arrays of length M."""
    m = lo.shape[1]
    t_in = np.full(m, F32(t_near), F32)
    t_out = np.full(m, F32(t_far), F32)
    ok = np.ones(m, bool)
    for a in range(3):
        if par[a]:
            ok &= (lo[a] <= og[a]) & (og[a] < hi[a])
        else:
            ta = (lo[a] - og[a]) * inv[a]
            tb = (hi[a] - og[a]) * inv[a]
            t_in = np.maximum(t_in, np.minimum(ta, tb))
            t_out = np.minimum(t_out, np.maximum(ta, tb))
    t_in = np.where(t_in == F32(0.0), F32(0.0), t_in)     # a zero entry is +0
    hit = ok & (t_in < t_out)
    return t_in, t_out, hit


def hit_list(ps: PreparedScene, o, d, t_near=0.0, t_far=np.inf):
    """Hits of one FP32 ray, front to back: (ids int64 [H], t_in float32 [H], t_out float32 [H])."""
    og, dg, inv, par, valid = ray_frame(o, d, ps.org32, ps.gs32)
    if not valid:
        e = np.zeros(0)
        return e.astype(np.int64), e.astype(F32), e.astype(F32)
    t_in, t_out, hit = box_interval(og, inv, par, ps.lo32, ps.hi32, t_near, t_far)
    ids = np.nonzero(hit)[0]
    order = np.argsort(t_in[ids], kind="stable")
    ids = ids[order]
    return ids, t_in[ids], t_out[ids]


def hit_lists(ps: PreparedScene, o, d, t_near=0.0, t_far=np.inf):
    """hit_list for every ray of float32 [n, 3] origins and directions."""
    return [hit_list(ps, o[r], d[r], t_near, t_far) for r in range(o.shape[0])]
