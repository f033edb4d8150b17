"""Per-ray outputs: midpoint samples, field values and front-to-back compositing (float64).

For every voxel a ray hits, in entry order (hitspec), with segment [t_in, t_out] and
delta = t_out - t_in, the segment is cut into S equal pieces and each piece is sampled at
its midpoint (the paper samples one midpoint per segment, Sec. 3.1 after Eq. 4; S = 1 is
that rule exactly):
    t_k = t_in + (k + 1/2) delta / S,   p_k = o + t_k d
    x_k = 2 ((p_k - origin) gs - lo) / n - 1, clamped to [-1, 1]^3   (gs = 2^K / s0)
Each piece is one compositing step with length delta / S (Eq. 4 and Eq. 3):
    tau = sigma delta / S,  alpha = 1 - exp(-tau),  w = T alpha,
    C += w rgb,  D += w t_k,  I += w intensity,  T <- T exp(-tau)
After each voxel the ray stops if T < t_min (t_min = 0 never stops).  At the end
C += T bg and the opacity is O = 1 - T.  D is the expected range along the ray's unit
direction (metres), not normalized by O.  n_hits counts the voxels composited.
"""
from __future__ import annotations

import dataclasses
from typing import Sequence

import numpy as np

from .field import corner_field, paper_field, sdf_field
from .hitspec import PreparedScene, hit_list


@dataclasses.dataclass
class RenderOpts:
    samples: int = 4
    t_min: float = 1e-6
    background: Sequence[float] = (0.0, 0.0, 0.0)
    t_near: float = 0.0
    t_far: float = float("inf")
    field: str = "corner"            # "corner" | "paper" | "sdf"


def _sample_points(ps: PreparedScene, o64, d64, v, t_in, t_out, S):
    delta = t_out - t_in
    lo = ps.lo_i[v].astype(np.float64)
    n = float(ps.n_i[v])
    for k in range(S):
        tk = t_in + (k + 0.5) * delta / S
        p = o64 + tk * d64
        x = 2.0 * ((p - ps.origin) * ps.gs - lo) / n - 1.0
        yield tk, np.clip(x, -1.0, 1.0), delta / S


def render_ray(ps: PreparedScene, o, d, opts: RenderOpts, hits=None):
    """Outputs of one FP32 ray (o, d float32 [3]) as a dict of float64 values."""
    sc = ps.scene
    if hits is None:
        hits = hit_list(ps, o, d, opts.t_near, opts.t_far)
    ids, t_ins, t_outs = hits
    o64 = np.asarray(o, np.float32).astype(np.float64)
    d64 = np.asarray(d, np.float32).astype(np.float64)
    T = 1.0
    C = np.zeros(3)
    D = 0.0
    I = 0.0
    nh = 0
    for v, ti, to in zip(ids, t_ins, t_outs):
        zg = sc.z_geo[v]
        zr = sc.z_rgb[v]
        zi = sc.z_int[v] if sc.z_int is not None else None
        for tk, x, dk in _sample_points(ps, o64, d64, v, float(ti), float(to), opts.samples):
            if opts.field == "corner":
                sigma, rgb, inten = corner_field(zg, zr, zi, x)
            elif opts.field == "sdf":
                sigma, rgb, inten = sdf_field(zg, zr, zi, x, d64)
            else:
                sigma, rgb, inten = paper_field(zg, zr, zi, x, d64)
            tau = sigma * dk
            alpha = -np.expm1(-tau)
            w = T * alpha
            C += w * rgb
            D += w * tk
            I += w * inten
            T *= np.exp(-tau)
        nh += 1
        if T < opts.t_min:
            break
    C += T * np.asarray(opts.background, np.float64)
    return {"rgb": C, "depth": D, "opacity": 1.0 - T, "intensity": I, "t_end": T, "n_hits": nh}


def render_rays(ps: PreparedScene, o, d, opts: RenderOpts, valid=None):
    """Outputs for float32 [n, 3] rays.  Rays with valid == False render the background
    with zero opacity.  Returns a dict of arrays (rgb [n, 3], others [n])."""
    n = o.shape[0]
    out = {"rgb": np.zeros((n, 3)), "depth": np.zeros(n), "opacity": np.zeros(n), "intensity": np.zeros(n),
           "t_end": np.ones(n), "n_hits": np.zeros(n, np.int64)}
    bg = np.asarray(opts.background, np.float64)
    for r in range(n):
        if valid is not None and not valid[r]:
            out["rgb"][r] = bg
            continue
        res = render_ray(ps, o[r], d[r], opts)
        for k in out:
            out[k][r] = res[k]
    return out
