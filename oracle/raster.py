"""Tile-based splatting of the voxels onto a pinhole image ("SaLF-Raster", Sec. 3.2 "Tile-based
Splatting"), float64 — TEST INFRASTRUCTURE ONLY (see the package header).

The steps follow the paper's order for a global-shutter pinhole camera (one eye for every pixel):
  1. projection and view-frustum culling.  Each voxel's eight corners are mapped into the camera
     frame (x right, y down, z forward; X_cam = R0^T (X - p0)).  A voxel whose corners all lie at
     z <= 0 is behind the camera and culled.  A voxel whose corners all lie at z >= z_near projects
     to the bounding rectangle of its projected corners (pixel-centre coordinate x = cx + fx X/Z,
     pixel u has its centre at u + 1/2), widened by `margin` pixels so that it also covers the
     pixels whose float32 rays graze it; a voxel reaching closer than z_near covers the whole image.
     A rectangle that misses the image is culled.
  2. tiling.  The image is cut into 16 x 16-pixel tiles; a tile's list holds every voxel whose
     rectangle overlaps it.
  3. sorting.  Each tile sorts its list by a depth key (below).
  4. compositing.  Every pixel walks its tile's sorted list; where its ray meets a voxel under the
     FP32 interval rule of `hitspec`, the ray's travel distance t_out - t_in inside the voxel gives
     the opacity (Eq. 4) and the field is sampled on that segment (S midpoints; S = 1 is the paper's
     single sample at the intersection), composited front to back with Eq. 3, the pixel stopping
     after the voxel that leaves T < t_min: the per-hit arithmetic of `render.render_ray`.
Pixel rays are the oracle's own float64 pinhole model (`sensors`) rounded to float32.

Depth keys (the paper sorts each tile's voxels by depth without saying which depth):
  "octree"  the front-to-back order of the voxel grid seen from the eye.  Along a ray from the eye
            the root-cell index of each axis moves away from the eye's root cell, so the L1 distance
            in root cells between a voxel's root cell and the eye's (clamped to one cell outside the
            grid) never decreases along the ray; inside a node the ray crosses each mid-plane at most
            once, from the eye's side to the other, so the octant index relative to the eye's side
            (child bit XOR eye-side bit per axis) only gains bits.  The key is that L1 distance
            followed by those relative octant digits from the top level down: it strictly increases
            along the hits of every pixel's ray, so every pixel composites its hits in the order a
            ray cast does.  The eye's side of a plane is decided on the FP32 grid-frame eye og of the
            interval rule (og >= plane: upper side), as the rule decides where the ray starts.
  "centre"  the camera-frame depth of the voxel centre (as Gaussian splatting sorts its particles):
            neighbouring voxels of different sizes can then be composited out of ray order for some
            pixels (the approximation the paper attributes to rasterization).
"""
from __future__ import annotations

import numpy as np

from .hitspec import F32, PreparedScene, box_interval, ray_frame
from .render import RenderOpts, render_ray
from .sensors import sensor_rays

TILE = 16
Z_NEAR = 1e-2   # metres; a voxel reaching closer to the camera plane covers the whole image
MARGIN = 1.0    # pixels added around each projected rectangle


def _camera(sensor):
    R = np.asarray(sensor["R0"], np.float64).reshape(3, 3)
    p = np.asarray(sensor["p0"], np.float64)
    return R, p


def footprints(ps: PreparedScene, sensor, margin=MARGIN, z_near=Z_NEAR):
    """Step 1: per voxel, its inclusive tile rectangle (tx0, ty0, tx1, ty1) or None when culled."""
    W, H = sensor["width"], sensor["height"]
    R, p = _camera(sensor)
    fx, fy, cx, cy = sensor["fx"], sensor["fy"], sensor["cx"], sensor["cy"]
    ntx, nty = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    out = []
    for v in range(ps.lo_i.shape[0]):
        lo = ps.lo_i[v].astype(np.float64)
        n = float(ps.n_i[v])
        corners = np.array([[lo[0] + n * (c & 1), lo[1] + n * ((c >> 1) & 1), lo[2] + n * ((c >> 2) & 1)]
                            for c in range(8)])
        world = ps.origin + corners / ps.gs
        cam = (world - p) @ R            # rows: R^T (X - p)
        z = cam[:, 2]
        if np.all(z <= 0.0):
            out.append(None)
            continue
        if np.any(z < z_near):
            out.append((0, 0, ntx - 1, nty - 1))
            continue
        xs = cx + fx * cam[:, 0] / z
        ys = cy + fy * cam[:, 1] / z
        u0 = int(np.floor(xs.min() - 0.5 - margin))
        u1 = int(np.ceil(xs.max() - 0.5 + margin))
        r0 = int(np.floor(ys.min() - 0.5 - margin))
        r1 = int(np.ceil(ys.max() - 0.5 + margin))
        if u1 < 0 or r1 < 0 or u0 > W - 1 or r0 > H - 1:
            out.append(None)
            continue
        u0, u1 = max(u0, 0), min(u1, W - 1)
        r0, r1 = max(r0, 0), min(r1, H - 1)
        out.append((u0 // TILE, r0 // TILE, u1 // TILE, r1 // TILE))
    return out


def depth_key(ps: PreparedScene, sensor, v: int, kind: str = "octree"):
    """Step 3's sort key of voxel v (smaller = nearer)."""
    sc = ps.scene
    if kind == "centre":
        R, p = _camera(sensor)
        centre = ps.origin + (ps.lo_i[v] + 0.5 * ps.n_i[v]) / ps.gs
        return float((centre - p) @ R[:, 2])
    K = int(sc.max_level)
    dims = np.asarray(sc.root_dims, np.int64)
    og, _, _, _, _ = ray_frame(np.asarray(sensor["p0"], np.float64).astype(F32), np.ones(3, F32), ps.org32, ps.gs32)
    og = og.astype(np.float64)                                   # exact values of the FP32 og
    eye_root = np.clip(np.floor(og / float(1 << K)), -1, dims).astype(np.int64)
    lo = ps.lo_i[v].astype(np.int64)
    level = K - int(np.log2(int(ps.n_i[v])))
    root = lo >> K
    l1 = int(np.sum(np.abs(root - eye_root)))
    digits = 0
    for j in range(1, K + 1):
        digits <<= 3
        if j > level:
            continue
        half = 1 << (K - j)
        mid = (lo >> (K - j + 1) << (K - j + 1)) + half         # mid-plane of v's level-(j-1) ancestor
        bit = (lo >> (K - j)) & 1                                 # the child v lies in
        eye = (og >= mid).astype(np.int64)                        # the eye's side of the mid-plane
        rel = bit ^ eye
        digits |= int(rel[0] | (rel[1] << 1) | (rel[2] << 2))
    return (l1 << (3 * K)) | digits


def tile_lists(ps: PreparedScene, sensor, kind: str = "octree", margin=MARGIN):
    """Steps 2-3: {(tx, ty): voxel ids sorted by depth key} for every tile with a voxel."""
    fps = footprints(ps, sensor, margin)
    lists = {}
    for v, fp in enumerate(fps):
        if fp is None:
            continue
        tx0, ty0, tx1, ty1 = fp
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                lists.setdefault((tx, ty), []).append(v)
    keys = {}
    for t, ids in lists.items():
        for v in ids:
            if v not in keys:
                keys[v] = depth_key(ps, sensor, v, kind)
        lists[t] = np.array(sorted(ids, key=lambda v: (keys[v], v)), np.int64)
    return lists


def raster(ps: PreparedScene, sensor, opts: RenderOpts, kind: str = "octree", margin=MARGIN):
    """Step 4: outputs of every pixel (dict of arrays as render.render_rays, pixel index r W + u),
    plus the per-pixel lists of composited voxel ids."""
    if sensor["model"] != 0:
        raise ValueError("splatting renders pinhole cameras")
    W, H = sensor["width"], sensor["height"]
    o64, d64, _, _ = sensor_rays(sensor)
    o, d = o64.astype(F32), d64.astype(F32)
    lists = tile_lists(ps, sensor, kind, margin)
    n = W * H
    out = {"rgb": np.zeros((n, 3)), "depth": np.zeros(n), "opacity": np.zeros(n), "intensity": np.zeros(n),
           "t_end": np.ones(n), "n_hits": np.zeros(n, np.int64)}
    composited = [np.zeros(0, np.int64)] * n
    for r in range(n):
        u, row = r % W, r // W
        ids = lists.get((u // TILE, row // TILE), np.zeros(0, np.int64))
        og, _, inv, par, valid = ray_frame(o[r], d[r], ps.org32, ps.gs32)
        if valid and ids.size:
            t_in, t_out, hit = box_interval(og, inv, par, ps.lo32[:, ids], ps.hi32[:, ids], opts.t_near, opts.t_far)
            sel = np.nonzero(hit)[0]
            hits = (ids[sel], t_in[sel], t_out[sel])
        else:
            hits = (np.zeros(0, np.int64), np.zeros(0, F32), np.zeros(0, F32))
        res = render_ray(ps, o[r], d[r], opts, hits=hits)
        for k in out:
            out[k][r] = res[k]
        composited[r] = hits[0][:int(res["n_hits"])]
    return out, composited
