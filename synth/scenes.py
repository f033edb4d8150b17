"""Seeded synthetic sparse-voxel scenes.

A scene is a set of non-overlapping cubic voxels on an adaptive grid (Sec. 3.1
"Representation": a regular root grid of edge s0, each cell subdividable into 8
children up to K levels, only non-empty voxels stored).  A voxel is given by its
level l (0 = root size s0, l = K finest) and its integer coordinates (i, j, k)
in units of that level's edge s_l = s0 / 2^l.

Per-voxel raw parameters are drawn from N(0, 1) and stored as float32:
  z_geo [N, 8]     density corner logits
  z_rgb [N, 3, 8]  colour corner logits (channel-major)
  z_int [N, 8]     LiDAR intensity corner logits
The corner index is c = bx + 2*by + 4*bz (b = 0 on the low face of an axis).
How those numbers become density and colour is the renderer's business; this
module never evaluates a field.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class SceneData:
    origin: np.ndarray          # float64 [3], world metres of the grid's min corner
    root_size: float            # s0 in metres
    root_dims: np.ndarray       # int64 [3], root cells per axis
    max_level: int              # K
    voxels: np.ndarray          # int32 [N, 4] = (level, i, j, k)
    z_geo: np.ndarray           # float32 [N, 8]
    z_rgb: np.ndarray           # float32 [N, 3, 8]
    z_int: Optional[np.ndarray] = None  # float32 [N, 8]
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.voxels.shape[0])

    def finest_bounds(self):
        """Integer bounds (lo, hi) of every voxel in finest-level units, int64 [N, 3] each."""
        lvl = self.voxels[:, 0].astype(np.int64)
        n = np.left_shift(np.int64(1), self.max_level - lvl)
        lo = self.voxels[:, 1:4].astype(np.int64) * n[:, None]
        return lo, lo + n[:, None]

    def permuted(self, perm: np.ndarray) -> "SceneData":
        """Same scene with voxel ids renamed: new voxel q is old voxel perm[q]."""
        return dataclasses.replace(
            self, voxels=self.voxels[perm].copy(), z_geo=self.z_geo[perm].copy(),
            z_rgb=self.z_rgb[perm].copy(),
            z_int=None if self.z_int is None else self.z_int[perm].copy())

    def subset(self, mask: np.ndarray) -> "SceneData":
        idx = np.nonzero(mask)[0]
        return self.permuted(idx)

    def save_npz(self, path: str) -> None:
        extra = {} if self.z_int is None else {"z_int": self.z_int}
        np.savez(path, origin=self.origin, root_size=np.float64(self.root_size), root_dims=self.root_dims,
                 max_level=np.int64(self.max_level), voxels=self.voxels, z_geo=self.z_geo, z_rgb=self.z_rgb,
                 name=np.array(self.name), **extra)

    @staticmethod
    def load_npz(path: str) -> "SceneData":
        with np.load(path, allow_pickle=False) as f:
            return SceneData(origin=f["origin"].astype(np.float64), root_size=float(f["root_size"]),
                             root_dims=f["root_dims"].astype(np.int64), max_level=int(f["max_level"]),
                             voxels=f["voxels"].astype(np.int32), z_geo=f["z_geo"].astype(np.float32),
                             z_rgb=f["z_rgb"].astype(np.float32),
                             z_int=f["z_int"].astype(np.float32) if "z_int" in f else None,
                             name=str(f["name"]))


def _draw_params(rng: np.random.Generator, n: int, intensity: bool = True):
    z_geo = rng.standard_normal((n, 8)).astype(np.float32)
    z_rgb = rng.standard_normal((n, 3, 8)).astype(np.float32)
    z_int = rng.standard_normal((n, 8)).astype(np.float32) if intensity else None
    return z_geo, z_rgb, z_int


# ----------------------------------------------------------------------------------------------
# Tiny scene: 4,096 voxels drawn uniformly from a 32^3 grid over a 10 m cube.
# ----------------------------------------------------------------------------------------------
def config0_scene(seed: int = 0) -> SceneData:
    rng = np.random.default_rng(seed)
    lin = rng.choice(32 * 32 * 32, size=4096, replace=False)
    i, j, k = lin % 32, (lin // 32) % 32, lin // 1024
    vox = np.stack([np.zeros_like(i), i, j, k], axis=1).astype(np.int32)
    z_geo, z_rgb, z_int = _draw_params(rng, vox.shape[0])
    return SceneData(origin=np.array([-5.0, -5.0, -5.0]), root_size=10.0 / 32.0,
                     root_dims=np.array([32, 32, 32], np.int64), max_level=0, voxels=vox,
                     z_geo=z_geo, z_rgb=z_rgb, z_int=z_int, name="tiny-4096")


def random_scene(seed: int, root_dims=(6, 5, 4), max_level: int = 2, root_size: float = 1.0,
                 origin=(-3.0, -2.5, -2.0), fill: float = 0.6, split: float = 0.5) -> SceneData:
    """Small adaptive scene for parity tests: every root cell is kept with probability `fill`,
    and a kept cell is split into 8 children with probability `split` while above level K;
    each child is then kept with probability `fill`."""
    rng = np.random.default_rng(seed)
    out = []

    def visit(level, c):
        if level < max_level and rng.random() < split:
            for b in range(8):
                ch = (2 * c[0] + (b & 1), 2 * c[1] + ((b >> 1) & 1), 2 * c[2] + ((b >> 2) & 1))
                if rng.random() < fill:
                    visit(level + 1, ch)
        else:
            out.append((level, c[0], c[1], c[2]))

    for kz in range(root_dims[2]):
        for jy in range(root_dims[1]):
            for ix in range(root_dims[0]):
                if rng.random() < fill:
                    visit(0, (ix, jy, kz))
    vox = np.array(out, np.int32).reshape(-1, 4)
    perm = rng.permutation(vox.shape[0])
    vox = vox[perm]
    z_geo, z_rgb, z_int = _draw_params(rng, vox.shape[0])
    return SceneData(origin=np.array(origin, np.float64), root_size=float(root_size),
                     root_dims=np.array(root_dims, np.int64), max_level=max_level, voxels=vox,
                     z_geo=z_geo, z_rgb=z_rgb, z_int=z_int, name=f"random-{seed}")


def single_voxel_scene(z_geo, z_rgb, z_int=None, root_size=1.0, origin=(0.0, 0.0, 0.0), dims=(1, 1, 1),
                       cell=(0, 0, 0)) -> SceneData:
    """One level-0 voxel with the given raw corner parameters."""
    z_geo = np.asarray(z_geo, np.float32).reshape(1, 8)
    z_rgb = np.asarray(z_rgb, np.float32).reshape(1, 3, 8)
    z_int = None if z_int is None else np.asarray(z_int, np.float32).reshape(1, 8)
    return SceneData(origin=np.array(origin, np.float64), root_size=float(root_size),
                     root_dims=np.array(dims, np.int64), max_level=0,
                     voxels=np.array([[0, *cell]], np.int32), z_geo=z_geo, z_rgb=z_rgb, z_int=z_int,
                     name="single")


def slab_scene(nx: int, ny: int, root_size: float, z_geo_value: float, seed: int = 3,
               origin=(0.0, 0.0, 0.0), nz: int = 2) -> SceneData:
    """A one-voxel-thick ground layer (z index 0) of nx * ny level-0 voxels, all with the same
    density logit and random colour/intensity logits, inside a grid nz cells tall."""
    rng = np.random.default_rng(seed)
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    vox = np.stack([np.zeros(nx * ny, np.int64), ii.ravel(), jj.ravel(), np.zeros(nx * ny, np.int64)], 1)
    n = vox.shape[0]
    z_geo = np.full((n, 8), z_geo_value, np.float32)
    z_rgb = rng.standard_normal((n, 3, 8)).astype(np.float32)
    z_int = rng.standard_normal((n, 8)).astype(np.float32)
    return SceneData(origin=np.array(origin, np.float64), root_size=float(root_size),
                     root_dims=np.array([nx, ny, nz], np.int64), max_level=0, voxels=vox.astype(np.int32),
                     z_geo=z_geo, z_rgb=z_rgb, z_int=z_int, name="slab")


# ----------------------------------------------------------------------------------------------
# Driving-scale scene: ~2M adaptive voxels over a 200 x 200 x 20.8 m region, 5 levels
# (1.6 m root down to 0.1 m).  A ground slab z in [0, 0.1) m whose target voxel size grows
# with lateral distance |y| from the road centre line, plus 300 hollow boxes (vehicles and
# buildings) whose shells are resolved at 0.2 m (one in three) or 0.4 m.
# Generation is top-down: a cell becomes a voxel when it touches some material and its edge
# is no larger than the smallest target size among the materials it touches; otherwise it
# is split into 8.  Voxels are therefore non-overlapping by construction.
# All geometry is done in integer finest-level units (0.1 m).
# ----------------------------------------------------------------------------------------------
C1_ROOT = 1.6
C1_K = 4
C1_DIMS = (125, 125, 13)
C1_ORIGIN = (-100.0, -100.0, 0.0)
# ground bands: (|y| upper edge in finest units, target edge in finest units)
C1_BANDS = ((180, 1), (420, 2), (700, 4), (940, 8))
C1_NBOX = 300


def _morton3(x, y, z):
    def spread(v):
        v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v
    return spread(x) | (spread(y) << np.uint64(1)) | (spread(z) << np.uint64(2))


def _boxes(rng, nbox, dims_f, box_min=2.0, box_max=10.0, unit=0.1, snap=4):
    """Axis-aligned boxes in finest units, snapped to `snap` units, standing on z = 0."""
    e = rng.uniform(box_min, box_max, size=(nbox, 3))
    e = np.maximum(snap, np.round(e / unit / snap).astype(np.int64) * snap)
    x0 = rng.uniform(0.0, 1.0, size=nbox) * (dims_f[0] - e[:, 0])
    y0 = rng.uniform(0.0, 1.0, size=nbox) * (dims_f[1] - e[:, 1])
    x0 = (np.floor(x0 / snap).astype(np.int64)) * snap
    y0 = (np.floor(y0 / snap).astype(np.int64)) * snap
    lo = np.stack([x0, y0, np.zeros(nbox, np.int64)], 1)
    hi = lo + e
    fine = rng.random(nbox) < (1.0 / 3.0)
    target = np.where(fine, 2, 4).astype(np.int64)
    return lo, hi, target


def _ground_target(ylo, yhi, centre, bands):
    miny = np.where((ylo <= centre) & (centre < yhi), 0,
                    np.where(ylo > centre, ylo - centre, centre - yhi))
    t = np.full(ylo.shape, 16, np.int64)
    for edge, size in reversed(bands):
        t = np.where(miny < edge, size, t)
    return t


def _adaptive_scene(rng, dims, K, bands, box_lo, box_hi, box_t):
    dims = np.asarray(dims, np.int64)
    centre_y = dims[1] * (1 << K) // 2
    INF = np.int64(1 << 40)
    # level-0 candidate cells: the ground layer and every root cell overlapping a box
    gi, gj = np.meshgrid(np.arange(dims[0]), np.arange(dims[1]), indexing="ij")
    ground = np.stack([gi.ravel(), gj.ravel(), np.zeros(gi.size, np.int64)], 1)
    pc, pb = [], []
    n0 = 1 << K
    for b in range(box_lo.shape[0]):
        r0 = box_lo[b] // n0
        r1 = (box_hi[b] - 1) // n0
        xs, ys, zs = np.meshgrid(np.arange(r0[0], r1[0] + 1), np.arange(r0[1], r1[1] + 1),
                                 np.arange(r0[2], r1[2] + 1), indexing="ij")
        c = np.stack([xs.ravel(), ys.ravel(), zs.ravel()], 1)
        pc.append(c)
        pb.append(np.full(c.shape[0], b, np.int64))
    pcell = np.concatenate(pc, 0)
    pbox = np.concatenate(pb, 0)

    def lin(c, d):
        return c[:, 0] + d[0] * (c[:, 1] + d[1] * c[:, 2])

    def delin(l, d):
        return np.stack([l % d[0], (l // d[0]) % d[1], l // (d[0] * d[1])], 1)

    d_l = dims.copy()
    cells = np.unique(np.concatenate([lin(ground, d_l), lin(pcell, d_l)]))
    plin = lin(pcell, d_l)
    out = []
    for level in range(K + 1):
        n = np.int64(1 << (K - level))
        c = delin(cells, d_l)
        lo = c * n
        hi = lo + n
        gt = np.where(lo[:, 2] == 0, _ground_target(lo[:, 1], hi[:, 1], centre_y, bands), INF)
        # box shells: the layer of thickness t inside each box's faces
        cidx = np.searchsorted(cells, plin)
        cl, ch = lo[cidx], hi[cidx]
        bl, bh, bt = box_lo[pbox], box_hi[pbox], box_t[pbox]
        overlap = np.all((cl < bh) & (ch > bl), axis=1)
        inside = np.all((cl >= bl + bt[:, None]) & (ch <= bh - bt[:, None]), axis=1)
        keep = overlap & ~inside
        plin, pbox, cidx = plin[keep], pbox[keep], cidx[keep]
        btgt = np.full(cells.shape[0], INF, np.int64)
        np.minimum.at(btgt, cidx, box_t[pbox])
        tgt = np.minimum(gt, btgt)
        has = tgt < INF
        leaf = has & ((n <= tgt) | (level == K))
        lc = c[leaf]
        out.append(np.concatenate([np.full((lc.shape[0], 1), level, np.int64), lc], 1))
        sub = has & ~leaf
        if level == K or not np.any(sub):
            break
        # children of split cells, and the box pairs that follow them down
        d_next = d_l * 2
        sc = c[sub]
        kids = (2 * sc[:, None, :] + np.array([[b & 1, (b >> 1) & 1, (b >> 2) & 1] for b in range(8)])[None])
        kids = kids.reshape(-1, 3)
        is_sub = sub[cidx]
        pc_par = delin(plin[is_sub], d_l)
        pb_par = pbox[is_sub]
        pk = (2 * pc_par[:, None, :] + np.array([[b & 1, (b >> 1) & 1, (b >> 2) & 1] for b in range(8)])[None])
        plin = lin(pk.reshape(-1, 3), d_next)
        pbox = np.repeat(pb_par, 8)
        d_l = d_next
        cells = np.sort(lin(kids, d_l))
    vox = np.concatenate(out, 0)
    # spatially coherent storage order: Morton order of each voxel's finest-unit min corner
    nf = np.left_shift(np.int64(1), K - vox[:, 0])
    lo_f = vox[:, 1:4] * nf[:, None]
    order = np.argsort(_morton3(lo_f[:, 0], lo_f[:, 1], lo_f[:, 2]), kind="stable")
    return vox[order].astype(np.int32)


def config1_scene(seed: int = 1, nbox: int = C1_NBOX) -> SceneData:
    rng = np.random.default_rng(seed)
    dims_f = np.array(C1_DIMS, np.int64) * (1 << C1_K)
    blo, bhi, bt = _boxes(rng, nbox, dims_f)
    vox = _adaptive_scene(rng, C1_DIMS, C1_K, C1_BANDS, blo, bhi, bt)
    z_geo, z_rgb, z_int = _draw_params(rng, vox.shape[0])
    return SceneData(origin=np.array(C1_ORIGIN, np.float64), root_size=C1_ROOT,
                     root_dims=np.array(C1_DIMS, np.int64), max_level=C1_K, voxels=vox,
                     z_geo=z_geo, z_rgb=z_rgb, z_int=z_int, name=f"driving-{seed}")


def config1_variant(seed: int) -> SceneData:
    """Seeded variants of the driving-scale scene (other box layouts and parameters)."""
    return config1_scene(seed=seed)


def box_layout(seed: int = 1, nbox: int = C1_NBOX):
    """The boxes of the driving-scale scene in world metres: (lo [B,3], hi [B,3], target edge [B])."""
    rng = np.random.default_rng(seed)
    dims_f = np.array(C1_DIMS, np.int64) * (1 << C1_K)
    blo, bhi, bt = _boxes(rng, nbox, dims_f)
    unit = C1_ROOT / (1 << C1_K)
    org = np.array(C1_ORIGIN)
    return org + blo * unit, org + bhi * unit, bt * unit


def param_bytes(scene: SceneData) -> int:
    b = scene.z_geo.nbytes + scene.z_rgb.nbytes
    return b + (0 if scene.z_int is None else scene.z_int.nbytes)


def level_histogram(scene: SceneData):
    return {int(l): int(c) for l, c in zip(*np.unique(scene.voxels[:, 0], return_counts=True))}


def _deg(x):
    return math.radians(x)
