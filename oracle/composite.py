"""Rendering a static scene with dynamic actors (the simulator's merged traversal, Sec. 4.1),
float64 — test infrastructure.

Each actor is a scene in its own canonical frame, placed by a rigid pose (R, t): a world point p is
the actor point R^T (p - t).  A ray (o, d) meets an actor in the actor frame, where it is
(R^T (o - t), R^T d), formed in FP32 in a fixed order (o - t first; then, per component i,
(R[0][i] p[0] + R[1][i] p[1]) + R[2][i] p[2], every operation rounded, never fused); a rigid map
keeps the ray parameter t, so depths and intervals of every scene share it.  The actor's box is
its root grid, met over [a_in, a_out) by the FP32 interval rule.

Per ray the actors it meets are taken in order of a_in (ties by index).  The ray's range is cut at
their boxes: the static scene is walked over [cur, a_in] before each actor and the actor over
[a_in, a_out]; then cur = max(cur, a_out), and the static scene over [cur, t_far] ends the ray.
All hits, in that order, are composited as in a single scene (samples, Eq. 3-4, early termination
after the voxel that leaves T < t_min).  Actors must not overlap one another or static voxels
(the simulator removes actors from the background), so the pieces never reorder a hit.
"""
from __future__ import annotations

import numpy as np

from .field import corner_field
from .hitspec import PreparedScene, box_interval, hit_list, ray_frame
from .render import RenderOpts, _sample_points

F32 = np.float32


def actor_ray(R, t, o, d):
    """The ray in an actor's frame, FP32, in the order stated above."""
    R = np.asarray(R, F32).reshape(3, 3)
    t = np.asarray(t, F32)
    p = (np.asarray(o, F32) - t).astype(F32)
    d = np.asarray(d, F32)
    oa = np.empty(3, F32)
    da = np.empty(3, F32)
    for i in range(3):
        oa[i] = F32(F32(R[0, i] * p[0]) + F32(R[1, i] * p[1])) + F32(R[2, i] * p[2])
        da[i] = F32(F32(R[0, i] * d[0]) + F32(R[1, i] * d[1])) + F32(R[2, i] * d[2])
    return oa, da


def _grid_interval(ps: PreparedScene, o, d, t_near, t_far):
    og, dg, inv, par, valid = ray_frame(o, d, ps.org32, ps.gs32)
    if not valid:
        return None
    dims = np.asarray(ps.scene.root_dims, np.int64) << ps.scene.max_level
    lo = np.zeros((3, 1), F32)
    hi = dims.astype(F32).reshape(3, 1)
    t_in, t_out, hit = box_interval(og, inv, par, lo, hi, t_near, t_far)
    return (float(t_in[0]), float(t_out[0])) if hit[0] else None


def composite_ray(static: PreparedScene, actors, o, d, opts: RenderOpts):
    """Outputs of one FP32 ray; actors: list of (PreparedScene, R [3, 3], t [3])."""
    o32, d32 = np.asarray(o, F32), np.asarray(d, F32)
    met = []
    for a, (ps, R, t) in enumerate(actors):
        oa, da = actor_ray(R, t, o32, d32)
        iv = _grid_interval(ps, oa, da, opts.t_near, opts.t_far)
        if iv is not None:
            met.append((iv[0], a, iv[1], oa, da))
    met.sort(key=lambda m: (m[0], m[1]))
    pieces = []  # (scene, o, d, t_near, t_far)
    cur = float(F32(opts.t_near))
    for a_in, a, a_out, oa, da in met:
        if cur < a_in:
            pieces.append((static, o32, d32, cur, a_in))
        pieces.append((actors[a][0], oa, da, a_in, a_out))
        cur = max(cur, a_out)
    pieces.append((static, o32, d32, cur, float(opts.t_far)))
    T, C, D, I, nh = 1.0, np.zeros(3), 0.0, 0.0, 0
    for ps, po, pd, tn, tf in pieces:
        if not tn < tf:
            continue
        ids, t_ins, t_outs = hit_list(ps, po, pd, tn, tf)
        o64, d64 = po.astype(np.float64), pd.astype(np.float64)
        sc = ps.scene
        for v, ti, to in zip(ids, t_ins, t_outs):
            zi = sc.z_int[v] if sc.z_int is not None else None
            for tk, x, dk in _sample_points(ps, o64, d64, v, float(ti), float(to), opts.samples):
                sigma, rgb, inten = corner_field(sc.z_geo[v], sc.z_rgb[v], zi, x)
                tau = sigma * dk
                w = T * -np.expm1(-tau)
                C += w * rgb
                D += w * tk
                I += w * inten
                T *= np.exp(-tau)
            nh += 1
            if T < opts.t_min:
                C += T * np.asarray(opts.background, np.float64)
                return {"rgb": C, "depth": D, "opacity": 1.0 - T, "intensity": I, "t_end": T, "n_hits": nh}
    C += T * np.asarray(opts.background, np.float64)
    return {"rgb": C, "depth": D, "opacity": 1.0 - T, "intensity": I, "t_end": T, "n_hits": nh}


def composite_rays(static: PreparedScene, actors, o, d, opts: RenderOpts):
    n = o.shape[0]
    out = {"rgb": np.zeros((n, 3)), "depth": np.zeros(n), "opacity": np.zeros(n), "intensity": np.zeros(n),
           "t_end": np.ones(n), "n_hits": np.zeros(n, np.int64)}
    for r in range(n):
        res = composite_ray(static, actors, o[r], d[r], opts)
        for k in out:
            out[k][r] = res[k]
    return out
