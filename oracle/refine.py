"""Densification and pruning of the sparse voxel set (Sec. 3.3), float64 — test infrastructure.

For each voxel v of level l (edge s0 / 2^l metres):
  prune     if its edge opacity alpha_e = 1 - exp(-sigma_max s0 / 2^l) is below alpha_min
            (Sec. 3.3 uses 0.001): the opacity of a path one edge long at the voxel's largest
            density (a reading: the paper does not say which opacity; the longest chord of the
            cube is sqrt(3) edges, so this is not the largest opacity a ray can see in the voxel).
            sigma_max is the largest density inside the voxel; in every
            field mode it is reached at a corner (a trilinear interpolation of non-negative corner
            values, exp of an affine form, or Eq. 6's density, monotone in an affine s), so it is the
            largest of the eight corner densities.
  split     else, if the L1 norm of the loss gradient w.r.t. its colour field parameters exceeds
            grad_threshold and l < K: replaced by its 8 octree-aligned children of level l + 1,
            child b = bx + 2 by + 4 bz at (2i + bx, 2j + by, 2k + bz).  The colour field parameters
            are the 24 colour corner logits (corner mode) or the colour matrix W_c, rgb[ch][0:3]
            (paper / sdf mode; the SH coefficients are not W_c).
  keep      otherwise.
Outputs keep the input order; a split voxel's children follow in the order of b.

Children carry the parent's field exactly.  With the child's local coordinate x_c in [-1, 1]^3,
the parent's is x_p = x_c / 2 + o_b with o_b = (2b - 1) / 2 per axis.
  corner mode   the parent's activated field is trilinear, so on the child it is the trilinear
                interpolation of its values at the child's corners (points of the parent's
                3 x 3 x 3 lattice); the child's logits are the inverse activations of those values
                (softplus^-1 y = log(expm1 y), sigmoid^-1 y = log(y / (1 - y))).
  paper / sdf   an affine form w . x_p + c equals (w / 2) . x_c + (c + w . o_b): slopes halve and the
                offset absorbs w . o_b.  The colour has no offset of its own besides the SH DC term
                (times the constant C0), which absorbs it: rgb[ch][3] += (W_c . o_b) / C0.  The SH
                higher coefficients, the SDF's log a, log b and unused slots are copied.
"""
from __future__ import annotations

import math

import numpy as np

from .field import SH_C0, corner_weights, paper_field, sdf_density, sigmoid, softplus


def _corner_points():
    """Parent coordinates of the 8 corners of each child b: [8 children][8 corners][3]."""
    pts = np.empty((8, 8, 3))
    for b in range(8):
        ob = np.array([((b >> a) & 1) - 0.5 for a in range(3)])
        for c in range(8):
            xc = np.array([2.0 * ((c >> a) & 1) - 1.0 for a in range(3)])
            pts[b, c] = xc / 2.0 + ob
    return pts


def sigma_max(z_geo_v, field: str) -> float:
    """Largest density of one voxel: the largest of its corner densities."""
    corners = np.array([[2.0 * ((c >> a) & 1) - 1.0 for a in range(3)] for c in range(8)])
    z = np.asarray(z_geo_v, np.float64)
    if field == "corner":
        return float(np.max(softplus(z)))
    if field == "sdf":
        return max(sdf_density(z, x)[0] for x in corners)
    return max(float(np.exp(z[:3] @ x + z[3])) for x in corners)


def colour_grad_l1(d_rgb_v, field: str) -> float:
    g = np.asarray(d_rgb_v, np.float64)
    return float(np.sum(np.abs(g if field == "corner" else g[:, 0:3])))


def _children_params(z_geo_v, z_rgb_v, z_int_v, field: str):
    """(geo [8, 8], rgb [8, 3, 8], int [8, 8] or None) of the 8 children of one voxel."""
    zg = np.asarray(z_geo_v, np.float64)
    zr = np.asarray(z_rgb_v, np.float64)
    zi = None if z_int_v is None else np.asarray(z_int_v, np.float64)
    cg, cr = np.zeros((8, 8)), np.zeros((8, 3, 8))
    ci = None if zi is None else np.zeros((8, 8))
    if field == "corner":
        pts = _corner_points()
        sg, sr = softplus(zg), sigmoid(zr)
        si = None if zi is None else sigmoid(zi)
        for b in range(8):
            for c in range(8):
                w = corner_weights(pts[b, c])
                y = float(w @ sg)
                cg[b, c] = math.log(math.expm1(y))
                for ch in range(3):
                    q = float(sr[ch] @ w)
                    cr[b, ch, c] = math.log(q / (1.0 - q))
                if si is not None:
                    q = float(si @ w)
                    ci[b, c] = math.log(q / (1.0 - q))
        return cg, cr, ci
    for b in range(8):
        ob = np.array([((b >> a) & 1) - 0.5 for a in range(3)])
        cg[b] = zg
        cg[b, :3] = zg[:3] / 2.0
        cg[b, 3] = zg[3] + zg[:3] @ ob
        cr[b] = zr
        for ch in range(3):
            cr[b, ch, :3] = zr[ch, :3] / 2.0
            cr[b, ch, 3] = zr[ch, 3] + (zr[ch, :3] @ ob) / SH_C0
        if zi is not None:
            ci[b] = zi
            ci[b, :3] = zi[:3] / 2.0
            ci[b, 3] = zi[3] + zi[:3] @ ob
    return cg, cr, ci


def refine(scene, d_rgb, grad_threshold: float, alpha_min: float = 1e-3, field: str = "corner"):
    """The refined scene (a copy of `scene` with new voxels and float64 parameters) and the
    per-voxel decisions (0 prune, 1 keep, 8 split)."""
    import dataclasses
    K = scene.max_level
    vox, gs, rs, its, dec = [], [], [], [], []
    for v in range(scene.n):
        lvl, i, j, k = (int(t) for t in scene.voxels[v])
        edge = float(scene.root_size) / (1 << lvl)
        zi = None if scene.z_int is None else scene.z_int[v]
        if 1.0 - math.exp(-sigma_max(scene.z_geo[v], field) * edge) < alpha_min:
            dec.append(0)
            continue
        if lvl < K and colour_grad_l1(d_rgb[v], field) > grad_threshold:
            dec.append(8)
            cg, cr, ci = _children_params(scene.z_geo[v], scene.z_rgb[v], zi, field)
            for b in range(8):
                vox.append((lvl + 1, 2 * i + (b & 1), 2 * j + ((b >> 1) & 1), 2 * k + ((b >> 2) & 1)))
                gs.append(cg[b])
                rs.append(cr[b])
                if ci is not None:
                    its.append(ci[b])
            continue
        dec.append(1)
        vox.append((lvl, i, j, k))
        gs.append(np.asarray(scene.z_geo[v], np.float64))
        rs.append(np.asarray(scene.z_rgb[v], np.float64))
        if zi is not None:
            its.append(np.asarray(zi, np.float64))
    out = dataclasses.replace(
        scene, voxels=np.array(vox, np.int32).reshape(-1, 4), z_geo=np.array(gs).reshape(-1, 8),
        z_rgb=np.array(rs).reshape(-1, 3, 8), z_int=None if scene.z_int is None else np.array(its).reshape(-1, 8))
    return out, np.array(dec, np.int32)


def field_at(scene, v, x, field: str, omega=(0.0, 0.0, 1.0)):
    """(sigma, rgb, intensity) of voxel v at its local coordinates x (no clamping needed inside)."""
    from .field import corner_field
    zi = None if scene.z_int is None else scene.z_int[v]
    if field == "corner":
        return corner_field(scene.z_geo[v], scene.z_rgb[v], zi, x)
    if field == "sdf":
        sigma = sdf_density(scene.z_geo[v], x)[0]
        _, rgb, inten = paper_field(scene.z_geo[v], scene.z_rgb[v], zi, x, np.asarray(omega, np.float64))
        return sigma, rgb, inten
    return paper_field(scene.z_geo[v], scene.z_rgb[v], zi, x, np.asarray(omega, np.float64))
