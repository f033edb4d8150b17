"""Pins of the CPU oracle against facts fixed by the paper and by mathematics (no GPU).

Each test checks the oracle against something other than itself: closed forms for
special scenes, invariants of front-to-back compositing, brute force with exact
rational arithmetic, quadrature convergence, and finite differences.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle.render import RenderOpts

F32 = np.float32


def _sp(z):            # softplus, scalar math
    return math.log1p(math.exp(z)) if z < 30 else z + math.log1p(math.exp(-z))


def _sig(z):
    return 1.0 / (1.0 + math.exp(-z))


def _inv_sp(s):        # inverse softplus
    return math.log(math.expm1(s))


def _slab(o, d, lo, hi):
    """Exact FP64 ray/box interval (world coordinates)."""
    t0, t1 = -math.inf, math.inf
    for a in range(3):
        if d[a] == 0:
            if not (lo[a] <= o[a] < hi[a]):
                return None
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    t0 = max(t0, 0.0)
    return (t0, t1) if t0 < t1 else None


def _rays_through_box(rng, n, lo, hi, dist=4.0):
    """FP32 rays from outside aimed at random interior points of the box [lo, hi]."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    tgt = lo + (hi - lo) * rng.uniform(0.15, 0.85, size=(n, 3))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = tgt - dist * d
    return o.astype(F32), d.astype(F32)


def _lerp_trilinear(vals, x):
    """Trilinear interpolation by successive lerps (x in [-1,1]^3, corner c = bx + 2by + 4bz)."""
    f = (np.asarray(x) + 1.0) / 2.0
    v = np.asarray(vals, float).reshape(2, 2, 2)       # [bz, by, bx]
    vx = v[:, :, 0] * (1 - f[0]) + v[:, :, 1] * f[0]
    vy = vx[:, 0] * (1 - f[1]) + vx[:, 1] * f[1]
    return vy[0] * (1 - f[2]) + vy[1] * f[2]


# ---------------------------------------------------------------- P1 empty scene / miss
def test_p1_empty_scene_and_miss():
    empty = synth.SceneData(origin=np.zeros(3), root_size=1.0, root_dims=np.array([4, 4, 4]), max_level=1,
                            voxels=np.zeros((0, 4), np.int32), z_geo=np.zeros((0, 8), F32),
                            z_rgb=np.zeros((0, 3, 8), F32), z_int=np.zeros((0, 8), F32))
    ps = oracle.prepare(empty)
    o, d = synth.random_rays(5, 50, (0, 0, 0), (4, 4, 4))
    bg = (0.25, 0.5, 0.75)
    out = oracle.render_rays(ps, o, d, RenderOpts(background=bg))
    assert np.all(out["rgb"] == np.array(bg)) and np.all(out["depth"] == 0)
    assert np.all(out["opacity"] == 0) and np.all(out["intensity"] == 0) and np.all(out["n_hits"] == 0)
    # rays pointing away from a non-empty scene miss everything
    sc = synth.random_scene(1)
    ps = oracle.prepare(sc)
    o = np.tile(np.array([[10.0, 10.0, 10.0]], F32), (20, 1))
    d = synth.random_rays(6, 20, (0, 0, 0), (1, 1, 1))[1]
    d = np.abs(d).astype(F32)                      # all components >= 0: away from the scene
    for r in range(20):
        ids, ti, to = oracle.hit_list(ps, o[r], d[r])
        assert ids.size == 0
    out = oracle.render_rays(ps, o, d, RenderOpts(background=bg))
    assert np.all(out["rgb"] == np.array(bg)) and np.all(out["opacity"] == 0)


# ---------------------------------------------------------------- P2 constant voxel
@pytest.mark.parametrize("S", [1, 4, 7])
def test_p2_constant_voxel_closed_form(S):
    rng = np.random.default_rng(20 + S)
    z_s, z_c = 0.75, np.array([0.25, -1.25, 2.0])     # exact in float32
    sc = synth.single_voxel_scene(np.full(8, z_s), np.repeat(z_c[:, None], 8, 1), np.full(8, -0.375),
                                  root_size=2.0, origin=(-1.0, -1.0, -1.0))
    ps = oracle.prepare(sc)
    sigma, c, ival = _sp(z_s), np.array([_sig(z) for z in z_c]), _sig(-0.375)
    o, d = _rays_through_box(rng, 40, (-1, -1, -1), (1, 1, 1))
    bg = np.array([0.1, 0.2, 0.9])
    for r in range(o.shape[0]):
        ids, ti, to = oracle.hit_list(ps, o[r], d[r])
        ex = _slab(o[r].astype(float), d[r].astype(float), (-1, -1, -1), (1, 1, 1))
        assert ids.tolist() == [0] and ex is not None
        assert abs(float(ti[0]) - ex[0]) < 1e-5 and abs(float(to[0]) - ex[1]) < 1e-5
        L = float(to[0]) - float(ti[0])
        out = oracle.render_ray(ps, o[r], d[r], RenderOpts(samples=S, background=bg))
        O = 1.0 - math.exp(-sigma * L)
        assert abs(out["opacity"] - O) < 1e-12
        assert np.allclose(out["rgb"], c * O + bg * (1 - O), atol=1e-12, rtol=0)
        assert abs(out["intensity"] - ival * O) < 1e-12
        tau = sigma * L / S
        D = sum(math.exp(-k * tau) * (1 - math.exp(-tau)) * (float(ti[0]) + (k + 0.5) * L / S) for k in range(S))
        assert abs(out["depth"] - D) < 1e-12


# ---------------------------------------------------------------- P3 density linear along x
def test_p3_linear_density_midpoint_exact():
    rng = np.random.default_rng(3)
    a, b = 1.3, 0.9                     # sigma(x) = a + b x_0, positive on [-1, 1]
    zg = [_inv_sp(a + b * (2 * (c & 1) - 1)) for c in range(8)]
    sc = synth.single_voxel_scene(zg, np.zeros((3, 8)), None, root_size=1.0, origin=(0.0, 0.0, 0.0))
    ps = oracle.prepare(sc)
    s_lo, s_hi = _sp(float(sc.z_geo[0, 0])), _sp(float(sc.z_geo[0, 1]))   # the float32-stored corners
    a, b = (s_lo + s_hi) / 2, (s_hi - s_lo) / 2
    o, d = _rays_through_box(rng, 30, (0, 0, 0), (1, 1, 1))
    for r in range(o.shape[0]):
        ids, ti, to = oracle.hit_list(ps, o[r], d[r])
        L = float(to[0]) - float(ti[0])
        mid = o[r].astype(float) + 0.5 * (float(ti[0]) + float(to[0])) * d[r].astype(float)
        sig_mid = a + b * (2.0 * mid[0] - 1.0)
        for S in (1, 2, 5, 16):
            out = oracle.render_ray(ps, o[r], d[r], RenderOpts(samples=S))
            assert abs(out["opacity"] - (1 - math.exp(-L * sig_mid))) < 1e-12


def test_p3_colour_corner_order_small_density_limit():
    # red varies along x, green along y, blue along z; with vanishing density C / O -> c(x_mid)
    rng = np.random.default_rng(4)
    zr = np.zeros((3, 8))
    vals = {0: (0.5, 0.3), 1: (0.5, -0.3), 2: (0.6, 0.2)}   # channel: (mean, slope)
    for ch, (m, s) in vals.items():
        for c in range(8):
            bit = (c >> ch) & 1
            v = m + s * (2 * bit - 1)
            zr[ch, c] = math.log(v / (1 - v))
    sc = synth.single_voxel_scene(np.full(8, _inv_sp(1e-7)), zr, None, root_size=1.0)
    ps = oracle.prepare(sc)
    o, d = _rays_through_box(rng, 20, (0, 0, 0), (1, 1, 1))
    for r in range(o.shape[0]):
        ids, ti, to = oracle.hit_list(ps, o[r], d[r])
        mid = o[r].astype(float) + 0.5 * (float(ti[0]) + float(to[0])) * d[r].astype(float)
        out = oracle.render_ray(ps, o[r], d[r], RenderOpts(samples=4))
        want = [vals[ch][0] + vals[ch][1] * (2 * mid[ch] - 1) for ch in range(3)]
        assert np.allclose(out["rgb"] / out["opacity"], want, atol=1e-6)


# ---------------------------------------------------------------- P4 opaque slab
@pytest.mark.parametrize("S", [1, 4])
def test_p4_opaque_slab_hit_depth(S):
    rng = np.random.default_rng(40 + S)
    sc = synth.slab_scene(8, 8, 1.0, 3000.0, nz=6)      # sigma = 3000 / m, slab z in [0, 1]
    ps = oracle.prepare(sc)
    checked = 0
    for _ in range(200):
        e = np.array([rng.uniform(1.1, 6.9), rng.uniform(1.1, 6.9), 1.0])
        d = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), -1.0])
        d /= np.linalg.norm(d)
        o = e - rng.uniform(2.0, 4.5) * d
        o32, d32 = o.astype(F32), d.astype(F32)
        o64, d64 = o32.astype(float), d32.astype(float)
        t_hit = (1.0 - o64[2]) / d64[2]
        p = o64 + t_hit * d64
        vx, vy = int(math.floor(p[0])), int(math.floor(p[1]))
        first = _slab(o64, d64, (vx, vy, 0), (vx + 1, vy + 1, 1))
        if first is None or 3000.0 * (first[1] - first[0]) / S < 30:
            continue
        out = oracle.render_ray(ps, o32, d32, RenderOpts(samples=S))
        d1 = first[1] - first[0]
        assert abs(out["depth"] - (t_hit + d1 / (2 * S))) < 1e-5
        assert 1.0 - out["opacity"] < 1e-12
        # colour = trilinear interpolation of the activated corners at the first sample
        t1 = t_hit + d1 / (2 * S)
        x = 2.0 * (o64 + t1 * d64 - np.array([vx, vy, 0.0])) - 1.0
        v = vx * 8 + vy
        want = [_lerp_trilinear([_sig(z) for z in sc.z_rgb[v, ch]], x) for ch in range(3)]
        assert np.allclose(out["rgb"], want, atol=1e-5)
        checked += 1
    assert checked > 100


# ---------------------------------------------------------------- P5 invariants
def test_p5_invariants_random_scenes():
    for seed in (7, 8):
        sc = synth.random_scene(seed)
        ps = oracle.prepare(sc)
        lo = sc.origin
        hi = sc.origin + sc.root_dims * sc.root_size
        o, d = synth.random_rays(seed, 150, lo, hi)
        bg = (0.3, 0.6, 0.1)
        out = oracle.render_rays(ps, o, d, RenderOpts(background=bg, t_min=0.0))
        assert all(np.all(np.isfinite(v)) for v in out.values())
        assert np.all(out["opacity"] >= 0) and np.all(out["opacity"] <= 1)
        assert np.allclose(out["opacity"], 1 - out["t_end"], atol=0, rtol=0)
        assert np.all(out["rgb"] >= -1e-15) and np.all(out["rgb"] <= 1 + 1e-15)
        assert np.all(out["intensity"] >= 0) and np.all(out["intensity"] <= out["opacity"] + 1e-15)
        for r in range(o.shape[0]):
            ids, ti, to = oracle.hit_list(ps, o[r], d[r])
            assert np.all(ti < to)
            assert np.all(to[:-1] <= ti[1:])                        # disjoint, ascending
            if ids.size:
                assert 0 <= out["depth"][r] <= out["opacity"][r] * float(to[-1]) + 1e-12
            else:
                assert out["depth"][r] == 0
        assert np.sum(out["n_hits"]) > 100


# ---------------------------------------------------------------- P6 over-operator split
def test_p6_front_back_split():
    sc = synth.random_scene(11, root_dims=(6, 4, 4), max_level=2)
    ps = oracle.prepare(sc)
    lo, hi = sc.finest_bounds()
    X = 3 * (1 << sc.max_level)                     # plane on a root-cell boundary
    front = sc.subset(hi[:, 0] <= X)
    back = sc.subset(lo[:, 0] >= X)
    assert front.n + back.n == sc.n and front.n > 10 and back.n > 10
    o, d = synth.random_rays(12, 150, sc.origin, sc.origin + sc.root_dims * sc.root_size)
    d = d.copy()
    d[:, 0] = np.abs(d[:, 0])                       # every ray crosses x = X at most once, forward
    bg = np.array([0.2, 0.4, 0.6])
    full = oracle.render_rays(ps, o, d, RenderOpts(background=bg, t_min=0.0))
    f = oracle.render_rays(oracle.prepare(front), o, d, RenderOpts(background=(0, 0, 0), t_min=0.0))
    b = oracle.render_rays(oracle.prepare(back), o, d, RenderOpts(background=bg, t_min=0.0))
    Tf = f["t_end"]
    assert np.allclose(full["rgb"], f["rgb"] + Tf[:, None] * b["rgb"], atol=1e-13, rtol=0)
    assert np.allclose(full["depth"], f["depth"] + Tf * b["depth"], atol=1e-12, rtol=0)
    assert np.allclose(full["intensity"], f["intensity"] + Tf * b["intensity"], atol=1e-13, rtol=0)
    assert np.allclose(full["t_end"], Tf * b["t_end"], atol=1e-14, rtol=0)
    assert np.sum((f["n_hits"] > 0) & (b["n_hits"] > 0)) > 20


# ---------------------------------------------------------------- P7 upload order
def test_p7_shuffle_only_renames():
    sc = synth.random_scene(13)
    perm = np.random.default_rng(0).permutation(sc.n)
    sp = sc.permuted(perm)
    o, d = synth.random_rays(14, 60, sc.origin, sc.origin + sc.root_dims * sc.root_size)
    a = oracle.render_rays(oracle.prepare(sc), o, d, RenderOpts())
    b = oracle.render_rays(oracle.prepare(sp), o, d, RenderOpts())
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    ps_a, ps_b = oracle.prepare(sc), oracle.prepare(sp)
    for r in range(o.shape[0]):
        ia, ta, ua = oracle.hit_list(ps_a, o[r], d[r])
        ib, tb, ub = oracle.hit_list(ps_b, o[r], d[r])
        assert np.array_equal(ia, perm[ib]) and np.array_equal(ta, tb) and np.array_equal(ua, ub)


# ---------------------------------------------------------------- P8 quadrature
def _gl_integrals(sigma_fn, rgb_fn, t0, t1, n=64):
    """Continuous volume rendering of one segment by composite Gauss-Legendre quadrature."""
    xg, wg = np.polynomial.legendre.leggauss(16)
    edges = np.linspace(t0, t1, n + 1)
    ts, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        ts.append((a + b) / 2 + (b - a) / 2 * xg)
        ws.append((b - a) / 2 * wg)
    ts, ws = np.concatenate(ts), np.concatenate(ws)
    sig = np.array([sigma_fn(t) for t in ts])
    # optical depth from t0 to each node, by the same quadrature on [t0, t]
    tau = np.array([_gl_tau(sigma_fn, t0, t) for t in ts])
    T = np.exp(-tau)
    C = np.sum(ws[:, None] * (T * sig)[:, None] * np.array([rgb_fn(t) for t in ts]), axis=0)
    return 1.0 - math.exp(-_gl_tau(sigma_fn, t0, t1)), C


def _gl_tau(sigma_fn, a, b):
    xg, wg = np.polynomial.legendre.leggauss(12)
    t = (a + b) / 2 + (b - a) / 2 * xg
    return float(np.sum((b - a) / 2 * wg * np.array([sigma_fn(x) for x in t])))


@pytest.mark.parametrize("field", ["corner", "paper"])
def test_p8_midpoint_rule_converges_quadratically(field):
    rng = np.random.default_rng(8)
    zg = rng.normal(0.5, 0.8, 8)
    zr = rng.normal(0, 1, (3, 8))
    if field == "paper":
        zg = np.array([0.6, -0.4, 0.3, 0.2, 0, 0, 0, 0])
    sc = synth.single_voxel_scene(zg, zr, None, root_size=2.0, origin=(0.0, 0.0, 0.0))
    ps = oracle.prepare(sc)
    o, d = _rays_through_box(rng, 1, (0, 0, 0), (2, 2, 2))
    o, d = o[0], d[0]
    ids, ti, to = oracle.hit_list(ps, o, d)
    t0, t1 = float(ti[0]), float(to[0])
    o64, d64 = o.astype(float), d.astype(float)

    def xl(t):
        return (o64 + t * d64) - 1.0            # local coords: (p - 0) * 2 / 2 - 1

    if field == "corner":
        sp = [_sp(z) for z in zg]
        sg = [[_sig(z) for z in zr[ch]] for ch in range(3)]
        sigma_fn = lambda t: _lerp_trilinear(sp, xl(t))
        rgb_fn = lambda t: np.array([_lerp_trilinear(sg[ch], xl(t)) for ch in range(3)])
    else:
        sigma_fn = lambda t: math.exp(float(np.dot(zg[:3], xl(t)) + zg[3]))
        C0, C1 = 0.28209479177387814, 0.4886025119029199
        gam = np.array([C0, C1 * d64[0], C1 * d64[1], C1 * d64[2]])
        rgb_fn = lambda t: np.array([_sig(float(np.dot(zr[ch, :3], xl(t)) + np.dot(zr[ch, 3:7], gam)))
                                     for ch in range(3)])
    O_ex, C_ex = _gl_integrals(sigma_fn, rgb_fn, t0, t1)
    errO, errC = [], []
    for S in (4, 8, 16, 32):
        out = oracle.render_ray(ps, o, d, RenderOpts(samples=S, t_min=0.0, field=field))
        errO.append(abs(out["opacity"] - O_ex))
        errC.append(np.max(np.abs(out["rgb"] - C_ex)))
    for e in (errO, errC):
        ratios = [e[i] / e[i + 1] for i in range(len(e) - 1)]
        assert all(3.3 < q < 4.7 for q in ratios), ratios


def test_p8_single_sample_is_the_paper_rule():
    """S = 1: alpha_i = 1 - exp(-sigma(mid_i) delta_i), C = sum_i prod_{j<i}(1 - alpha_j) alpha_i c(mid_i)."""
    sc = synth.random_scene(15)
    ps = oracle.prepare(sc)
    o, d = synth.random_rays(16, 40, sc.origin, sc.origin + sc.root_dims * sc.root_size)
    lo_i, hi_i = sc.finest_bounds()
    s_k = sc.root_size / (1 << sc.max_level)
    for r in range(o.shape[0]):
        ids, ti, to = oracle.hit_list(ps, o[r], d[r])
        alphas, cols = [], []
        for v, a, b in zip(ids, ti, to):
            a, b = float(a), float(b)
            mid = o[r].astype(float) + 0.5 * (a + b) * d[r].astype(float)
            lo_w = sc.origin + lo_i[v] * s_k
            hi_w = sc.origin + hi_i[v] * s_k
            x = np.clip(2 * (mid - lo_w) / (hi_w - lo_w) - 1, -1, 1)
            sig = _lerp_trilinear([_sp(z) for z in sc.z_geo[v]], x)
            alphas.append(1 - math.exp(-sig * (b - a)))
            cols.append([_lerp_trilinear([_sig(z) for z in sc.z_rgb[v, ch]], x) for ch in range(3)])
        C = np.zeros(3)
        for i in range(len(alphas)):
            C += np.prod([1 - alphas[j] for j in range(i)]) * alphas[i] * np.array(cols[i])
        out = oracle.render_ray(ps, o[r], d[r], RenderOpts(samples=1, t_min=0.0))
        assert np.allclose(out["rgb"], C, atol=1e-12)


# ---------------------------------------------------------------- P9 exact rational hits
def _exact_interval(o, d, org, gs, lo, hi):
    og = [(Fraction(float(o[a])) - Fraction(float(org[a]))) * gs for a in range(3)]
    dg = [Fraction(float(d[a])) * gs for a in range(3)]
    t0, t1 = Fraction(0), None
    for a in range(3):
        if dg[a] == 0:
            if not (lo[a] <= og[a] < hi[a]):
                return None, None
            continue
        ta, tb = (lo[a] - og[a]) / dg[a], (hi[a] - og[a]) / dg[a]
        t0 = max(t0, min(ta, tb))
        t1 = max(ta, tb) if t1 is None else min(t1, max(ta, tb))
    return t0, t1


def test_p9_fp32_hits_vs_exact_rationals():
    sc = synth.random_scene(17, root_dims=(4, 3, 3), max_level=2)
    ps = oracle.prepare(sc)
    gs = Fraction(1 << sc.max_level) / Fraction(sc.root_size)
    lo_i, hi_i = sc.finest_bounds()
    o, d = synth.random_rays(18, 60, sc.origin, sc.origin + sc.root_dims * sc.root_size)
    # a few axis-parallel rays exercise the parallel-axis rule
    d[:6] = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1]], F32)
    margin = Fraction(1, 10 ** 5) * gs                      # 1e-5 m in grid units
    n_deg = n_pairs = 0
    for r in range(o.shape[0]):
        ids, ti, to = oracle.hit_list(ps, o[r], d[r])
        got = {int(v): (float(a), float(b)) for v, a, b in zip(ids, ti, to)}
        dn = max(abs(Fraction(float(x))) for x in d[r]) * gs
        for v in range(sc.n):
            n_pairs += 1
            e0, e1 = _exact_interval(o[r], d[r], sc.origin.astype(F32), gs, lo_i[v], hi_i[v])
            if e0 is None:
                assert v not in got
                continue
            slack = (e1 - e0) * dn
            if slack > margin:
                assert v in got
                assert abs(got[v][0] - float(e0)) <= 1e-5 + 1e-6 * abs(float(e0))
                assert abs(got[v][1] - float(e1)) <= 1e-5 + 1e-6 * abs(float(e1))
            elif slack < -margin:
                assert v not in got
            else:
                n_deg += 1
    assert n_deg <= 0.01 * n_pairs


# ---------------------------------------------------------------- P10 sensor closed forms
def test_p10_pinhole_reprojects_to_its_pixel():
    R0 = synth.look_at((3, -4, 2), (0, 0, 0))
    s = synth.pinhole(33, 21, 70.0, R0, (3, -4, 2))
    o, d, t, valid = oracle.sensor_rays(s)
    assert np.all(valid) and np.allclose(np.linalg.norm(d, axis=1), 1, atol=1e-14)
    dc = d @ R0                                 # camera-frame directions (R0 orthonormal)
    u = s["fx"] * dc[:, 0] / dc[:, 2] + s["cx"] - 0.5
    v = s["fy"] * dc[:, 1] / dc[:, 2] + s["cy"] - 0.5
    uu, vv = np.meshgrid(np.arange(33), np.arange(21))
    assert np.allclose(u, uu.ravel(), atol=1e-9) and np.allclose(v, vv.ravel(), atol=1e-9)
    centre = 10 * 33 + 16                        # odd sizes: the principal point is a pixel centre
    assert np.allclose(d[centre], R0[:, 2], atol=1e-15)
    assert np.allclose(o, np.array([3, -4, 2.0]))


def test_p10_fisheye_equidistant():
    R0 = synth.yaw_pitch_camera(30.0, 10.0)
    s = synth.fisheye_equidistant(96, 72, 190.0, R0, (1, 2, 3))
    o, d, t, valid = oracle.sensor_rays(s)
    dc = d @ R0
    uu, vv = np.meshgrid(np.arange(96) + 0.5, np.arange(72) + 0.5)
    x, y = (uu.ravel() - s["cx"]), (vv.ravel() - s["cy"])
    r = np.hypot(x, y)
    theta = np.arccos(np.clip(dc[:, 2], -1, 1))
    assert np.all(valid == (r / s["fx"] <= s["max_theta"]))
    assert np.allclose(theta[valid], (r / s["fx"])[valid], atol=1e-12)
    assert np.allclose(np.arctan2(dc[valid, 1], dc[valid, 0]), np.arctan2(y, x)[valid], atol=1e-12)
    # the 90-degree circle has radius f pi / 2
    ring = valid & (np.abs(r - s["fx"] * math.pi / 2) < 0.5)
    assert np.any(ring) and np.all(np.abs(dc[ring, 2]) < 0.5 / s["fx"] + 1e-12)
    assert np.all(d[~valid] == 0)
    # 190 deg spans the width: f = (W / 2) / (95 deg)
    assert abs(s["fx"] - 48 / math.radians(95)) < 1e-12


def test_p10_lidar_angles_and_rolling_shutter():
    s = synth.lidar_spinning(16, 64, -25.0, 15.0, np.eye(3), (1, 2, 3), 0.1, v=(10, 0, 0), w=(0, 0, 0.5))
    o, d, t, valid = oracle.sensor_rays(s)
    B, J = 16, 64
    b, j = np.divmod(np.arange(B * J), J)
    elev = np.radians(-25 + 40 * b / (B - 1))
    tj = 0.1 * j / J
    az = 2 * math.pi * (j + 0.5) / J + 0.5 * tj         # spin about +z adds w t
    assert np.allclose(np.arcsin(np.clip(d[:, 2], -1, 1)), elev, atol=1e-12)
    dazi = np.angle(np.exp(1j * (np.arctan2(d[:, 1], d[:, 0]) - az)))
    assert np.allclose(dazi, 0, atol=1e-12)
    assert np.allclose(t, tj) and np.allclose(o, np.array([1, 2, 3]) + np.outer(tj, [10, 0, 0]))
    # no motion: rolling shutter equals the global shutter bit for bit
    s0 = synth.lidar_spinning(16, 64, -25.0, 15.0, np.eye(3), (1, 2, 3), 0.1)
    g = dict(s0, dt_line=0.0)
    a1, a2 = oracle.sensor_rays(s0), oracle.sensor_rays(g)
    assert np.array_equal(a1[0], a2[0]) and np.array_equal(a1[1], a2[1])


def test_p10_camera_rolling_shutter_rows():
    R0 = synth.yaw_pitch_camera(0, 0)
    s = synth.pinhole(8, 6, 60.0, R0, (0, 0, 1), t0=0.5, dt_line=30e-6, v=(10, 0, 0), w=(0, 0, 2.0))
    o, d, t, valid = oracle.sensor_rays(s)
    rows = np.arange(48) // 8
    assert np.allclose(t, 0.5 + rows * 30e-6)
    assert np.allclose(o, np.array([0, 0, 1.0]) + np.outer(rows * 30e-6, [10, 0, 0]))
    g = oracle.sensor_rays(dict(s, dt_line=0.0))
    # the yaw rate turns row r's rays by 2 * r * 30e-6 rad about +z relative to the global shutter
    ang = np.arctan2(d[:, 1], d[:, 0]) - np.arctan2(g[1][:, 1], g[1][:, 0])
    assert np.allclose(ang, 2.0 * rows * 30e-6, atol=1e-12)


def test_sh_basis_is_orthonormal():
    # Monte Carlo-free: exact spherical quadrature (Gauss-Legendre in cos theta x uniform phi)
    xg, wg = np.polynomial.legendre.leggauss(8)
    nphi = 16
    G = np.zeros((4, 4))
    for ct, w in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for k in range(nphi):
            ph = 2 * math.pi * k / nphi
            g = oracle.sh_basis([st * math.cos(ph), st * math.sin(ph), ct])
            G += w * (2 * math.pi / nphi) * np.outer(g, g)
    assert np.allclose(G, np.eye(4), atol=1e-12)


# ---------------------------------------------------------------- P11 gradient vs FD
def test_p11_oracle_gradient_matches_central_differences():
    sc = synth.random_scene(21, root_dims=(3, 3, 3), max_level=1, fill=0.7)
    o, d = synth.random_rays(22, 24, sc.origin, sc.origin + sc.root_dims * sc.root_size, inside_frac=0.0)
    rng = np.random.default_rng(23)
    n = o.shape[0]
    g_rgb, g_d, g_o, g_i = rng.normal(size=(n, 3)), rng.normal(size=n), rng.normal(size=n), rng.normal(size=n)
    opts = RenderOpts(samples=3, t_min=0.0, background=(0.1, 0.2, 0.3))
    # the FD runs in float64 end to end: parameters are perturbed as float64 copies
    sc64 = synth.SceneData(**{**sc.__dict__, "z_geo": sc.z_geo.astype(np.float64),
                              "z_rgb": sc.z_rgb.astype(np.float64), "z_int": sc.z_int.astype(np.float64)})

    def loss(s):
        out = oracle.render_rays(oracle.prepare(s), o, d, opts)
        return float(np.sum(g_rgb * out["rgb"]) + g_d @ out["depth"] + g_o @ out["opacity"] + g_i @ out["intensity"])

    dg, dr, di = oracle.grad_rays(oracle.prepare(sc64), o, d, opts, g_rgb, g_d, g_o, g_i)
    touched = np.nonzero(np.any(dg != 0, axis=1))[0]
    assert touched.size > 5
    eps = 1e-6
    for name, arr, grad in (("z_geo", sc64.z_geo, dg), ("z_rgb", sc64.z_rgb, dr), ("z_int", sc64.z_int, di)):
        for _ in range(8):
            v = int(rng.choice(touched))
            idx = (v,) + tuple(int(rng.integers(0, s)) for s in arr.shape[1:])
            old = arr[idx]
            arr[idx] = old + eps
            lp = loss(sc64)
            arr[idx] = old - eps
            lm = loss(sc64)
            arr[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grad[idx]) <= 1e-6 * abs(grad[idx]) + 1e-8, (name, idx, fd, grad[idx])


def test_p11_oracle_paper_field_gradient_matches_central_differences():
    """The same pin for the paper's field (Eq. 1-2): exponential-affine density, sigmoid colour
    with a degree-1 SH term, sigmoid-affine intensity."""
    sc = synth.random_scene(24, root_dims=(3, 3, 3), max_level=1, fill=0.7)
    rng = np.random.default_rng(25)
    n_v = sc.voxels.shape[0]
    geo = np.zeros((n_v, 8))
    geo[:, :3] = rng.normal(0, 0.5, (n_v, 3))
    geo[:, 3] = rng.normal(0, 1, n_v)
    rgb = np.zeros((n_v, 3, 8))
    rgb[:, :, :7] = rng.normal(0, 0.7, (n_v, 3, 7))
    ity = np.zeros((n_v, 8))
    ity[:, :4] = rng.normal(0, 0.7, (n_v, 4))
    sc64 = synth.SceneData(**{**sc.__dict__, "z_geo": geo, "z_rgb": rgb, "z_int": ity})
    o, d = synth.random_rays(26, 24, sc.origin, sc.origin + sc.root_dims * sc.root_size, inside_frac=0.0)
    n = o.shape[0]
    g_rgb, g_d, g_o, g_i = rng.normal(size=(n, 3)), rng.normal(size=n), rng.normal(size=n), rng.normal(size=n)
    opts = RenderOpts(samples=3, t_min=0.0, background=(0.1, 0.2, 0.3), field="paper")

    def loss(s):
        out = oracle.render_rays(oracle.prepare(s), o, d, opts)
        return float(np.sum(g_rgb * out["rgb"]) + g_d @ out["depth"] + g_o @ out["opacity"] + g_i @ out["intensity"])

    dg, dr, di = oracle.grad_rays(oracle.prepare(sc64), o, d, opts, g_rgb, g_d, g_o, g_i)
    touched = np.nonzero(np.any(dg != 0, axis=1))[0]
    assert touched.size > 5
    # the unused slots of each record get no gradient
    assert not dg[:, 4:].any() and not dr[:, :, 7].any() and not di[:, 4:].any()
    eps = 1e-6
    for name, arr, grad, width in (("z_geo", sc64.z_geo, dg, 4), ("z_rgb", sc64.z_rgb, dr, 7),
                                   ("z_int", sc64.z_int, di, 4)):
        for _ in range(8):
            v = int(rng.choice(touched))
            idx = (v,) + tuple(int(rng.integers(0, s)) for s in arr.shape[1:-1]) + (int(rng.integers(0, width)),)
            old = arr[idx]
            arr[idx] = old + eps
            lp = loss(sc64)
            arr[idx] = old - eps
            lm = loss(sc64)
            arr[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grad[idx]) <= 1e-6 * abs(grad[idx]) + 1e-8, (name, idx, fd, grad[idx])


def _sdf_scene(seed):
    sc = synth.random_scene(seed, root_dims=(3, 3, 3), max_level=1, fill=0.7)
    rng = np.random.default_rng(seed + 1)
    n_v = sc.voxels.shape[0]
    geo = np.zeros((n_v, 8))
    geo[:, :3] = rng.normal(0, 0.6, (n_v, 3))
    geo[:, 3] = rng.normal(0, 0.5, n_v)
    geo[:, 4] = rng.normal(0.5, 0.3, n_v)      # log a
    geo[:, 5] = rng.normal(-1.0, 0.3, n_v)     # log b
    rgb = np.zeros((n_v, 3, 8))
    rgb[:, :, :7] = rng.normal(0, 0.7, (n_v, 3, 7))
    ity = np.zeros((n_v, 8))
    ity[:, :4] = rng.normal(0, 0.7, (n_v, 4))
    return synth.SceneData(**{**sc.__dict__, "z_geo": geo, "z_rgb": rgb, "z_int": ity})


def test_sdf_density_is_a_scaled_laplace_cdf():
    """Eq. 6 is a times the CDF of a Laplace distribution of scale b at s (the VolSDF form):
    a/2 at s = 0, sigma(s) + sigma(-s) = a, a at s -> +inf, 0 at s -> -inf."""
    from scipy.stats import laplace
    rng = np.random.default_rng(31)
    for _ in range(200):
        z = np.zeros(8)
        z[:4] = rng.normal(0, 2.0, 4)
        z[4], z[5] = rng.normal(0, 1), rng.normal(-1, 1)
        x = rng.uniform(-1, 1, 3)
        sigma, s, a, b = oracle.sdf_density(z, x)
        assert abs(s - (z[:3] @ x + z[3])) < 1e-12
        assert abs(sigma - a * laplace.cdf(s, scale=b)) <= 1e-12 * a
        zm = z.copy()
        zm[:4] = -zm[:4]
        assert abs(sigma + oracle.sdf_density(zm, x)[0] - a) <= 1e-12 * a
    z = np.array([0.0, 0.0, 0.0, 0.0, math.log(3.0), math.log(0.1), 0.0, 0.0])
    assert abs(oracle.sdf_density(z, np.zeros(3))[0] - 1.5) < 1e-12
    z[3] = 50.0
    assert abs(oracle.sdf_density(z, np.zeros(3))[0] - 3.0) < 1e-12
    z[3] = -50.0
    assert oracle.sdf_density(z, np.zeros(3))[0] < 1e-12


def test_p11_oracle_sdf_gradient_matches_central_differences():
    """The central-difference pin for the SDF variant (Eq. 5-6), including a and b."""
    sc64 = _sdf_scene(27)
    rng = np.random.default_rng(29)
    o, d = synth.random_rays(28, 24, sc64.origin, sc64.origin + sc64.root_dims * sc64.root_size, inside_frac=0.0)
    n = o.shape[0]
    g_rgb, g_d, g_o, g_i = rng.normal(size=(n, 3)), rng.normal(size=n), rng.normal(size=n), rng.normal(size=n)
    opts = RenderOpts(samples=3, t_min=0.0, background=(0.1, 0.2, 0.3), field="sdf")

    def loss(s):
        out = oracle.render_rays(oracle.prepare(s), o, d, opts)
        return float(np.sum(g_rgb * out["rgb"]) + g_d @ out["depth"] + g_o @ out["opacity"] + g_i @ out["intensity"])

    dg, dr, di = oracle.grad_rays(oracle.prepare(sc64), o, d, opts, g_rgb, g_d, g_o, g_i)
    touched = np.nonzero(np.any(dg != 0, axis=1))[0]
    assert touched.size > 5
    assert not dg[:, 6:].any() and not dr[:, :, 7].any() and not di[:, 4:].any()
    eps = 1e-6
    for name, arr, grad, width in (("z_geo", sc64.z_geo, dg, 6), ("z_rgb", sc64.z_rgb, dr, 7),
                                   ("z_int", sc64.z_int, di, 4)):
        for k in range(10):
            v = int(rng.choice(touched))
            last = (k % width) if name == "z_geo" else int(rng.integers(0, width))
            idx = (v,) + tuple(int(rng.integers(0, s)) for s in arr.shape[1:-1]) + (last,)
            old = arr[idx]
            arr[idx] = old + eps
            lp = loss(sc64)
            arr[idx] = old - eps
            lm = loss(sc64)
            arr[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grad[idx]) <= 1e-6 * abs(grad[idx]) + 1e-8, (name, idx, fd, grad[idx])


# ---------------------------------------------------------------- densification and pruning
def _refine_scene(field, seed):
    sc = synth.random_scene(seed, root_dims=(3, 2, 2), max_level=2, fill=0.6)
    rng = np.random.default_rng(seed + 1)
    n_v = sc.voxels.shape[0]
    if field == "corner":
        return synth.SceneData(**{**sc.__dict__, "z_geo": sc.z_geo.astype(np.float64),
                                  "z_rgb": sc.z_rgb.astype(np.float64), "z_int": sc.z_int.astype(np.float64)})
    geo = np.zeros((n_v, 8))
    geo[:, :4] = rng.normal(0, 0.7, (n_v, 4))
    if field == "sdf":
        geo[:, 4], geo[:, 5] = rng.normal(0.5, 0.3, n_v), rng.normal(-1, 0.3, n_v)
    rgb = np.zeros((n_v, 3, 8))
    rgb[:, :, :7] = rng.normal(0, 0.7, (n_v, 3, 7))
    ity = np.zeros((n_v, 8))
    ity[:, :4] = rng.normal(0, 0.7, (n_v, 4))
    return synth.SceneData(**{**sc.__dict__, "z_geo": geo, "z_rgb": rgb, "z_int": ity})


@pytest.mark.parametrize("field", ["corner", "paper", "sdf"])
def test_refined_children_carry_the_parent_field(field):
    """Every child's field equals its parent's at the same world point (random points, float64),
    children tile their parent, and kept voxels are unchanged."""
    sc = _refine_scene(field, 41)
    rng = np.random.default_rng(42)
    d_rgb = rng.exponential(1.0, sc.z_rgb.shape)
    out, dec = oracle.refine(sc, d_rgb, grad_threshold=np.median([oracle.colour_grad_l1(g, field) for g in d_rgb]),
                             alpha_min=0.0, field=field)
    assert (dec == 8).sum() > 3 and (dec == 1).sum() > 3 and not (dec == 0).any()
    assert out.n == int(dec.sum())
    q = 0
    for v in range(sc.n):
        lvl, i, j, k = sc.voxels[v]
        if dec[v] == 1:
            assert tuple(out.voxels[q]) == (lvl, i, j, k)
            assert np.array_equal(out.z_geo[q], sc.z_geo[v]) and np.array_equal(out.z_rgb[q], sc.z_rgb[v])
            q += 1
            continue
        for b in range(8):
            bvec = np.array([(b >> a) & 1 for a in range(3)])
            assert tuple(out.voxels[q]) == (lvl + 1, 2 * i + bvec[0], 2 * j + bvec[1], 2 * k + bvec[2])
            for _ in range(4):
                xc = rng.uniform(-1, 1, 3)
                xp = xc / 2.0 + (bvec - 0.5)
                omega = rng.normal(size=3)
                omega /= np.linalg.norm(omega)
                sp, cp, ip = oracle.field_at(sc, v, xp, field, omega)
                sch, cch, ich = oracle.field_at(out, q, xc, field, omega)
                assert abs(sch - sp) <= 1e-9 * max(1.0, abs(sp))
                assert np.max(np.abs(cch - cp)) <= 1e-9 and abs(ich - ip) <= 1e-9
            q += 1
    assert q == out.n


@pytest.mark.parametrize("field", ["corner", "paper", "sdf"])
def test_pruning_uses_the_largest_opacity_in_the_voxel(field):
    """sigma_max is the largest density anywhere in the voxel (dense sampling never exceeds it and
    comes within 1%); pruning removes exactly the voxels whose alpha_max is below alpha_min."""
    sc = _refine_scene(field, 43)
    rng = np.random.default_rng(44)
    g = np.linspace(-1, 1, 9)
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    for v in range(sc.n):
        smax = oracle.sigma_max(sc.z_geo[v], field)
        dense = max(oracle.field_at(sc, v, x, field)[0] for x in pts)
        assert dense <= smax * (1 + 1e-12) and dense >= 0.99 * smax
    edge = sc.root_size / (1 << sc.voxels[:, 0].astype(np.int64))
    amax = np.array([1 - math.exp(-oracle.sigma_max(sc.z_geo[v], field) * edge[v]) for v in range(sc.n)])
    a_min = float(np.median(amax))
    out, dec = oracle.refine(sc, np.zeros(sc.z_rgb.shape), grad_threshold=1.0, alpha_min=a_min, field=field)
    assert np.array_equal(dec == 0, amax < a_min)
    assert out.n == int((amax >= a_min).sum())


# ---------------------------------------------------------------- dynamic actors
def test_composite_without_actors_is_the_plain_render():
    sc = synth.random_scene(71, root_dims=(3, 3, 2), max_level=2)
    ps = oracle.prepare(sc)
    o, d = synth.random_rays(72, 60, sc.origin, sc.origin + sc.root_dims * sc.root_size)
    opts = RenderOpts(background=(0.1, 0.2, 0.3))
    a, b = oracle.composite_rays(ps, [], o, d, opts), oracle.render_rays(ps, o, d, opts)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_composite_equals_the_merged_scene():
    """Moving the voxels of a slab of root cells into an actor (its own grid over that slab, placed
    with the identity pose) renders like the original scene: the actor's box splits the static walk
    exactly where the slab's voxels are (up to the rounding of the actor grid's own frame)."""
    sc = synth.random_scene(73, root_dims=(6, 3, 3), max_level=2, fill=0.7)
    lvl = sc.voxels[:, 0].astype(np.int64)
    cell_x = sc.voxels[:, 1].astype(np.int64) >> lvl      # root cell index along x
    inside = (cell_x >= 2) & (cell_x < 4)
    static = sc.subset(~inside)
    act = sc.subset(inside)
    act.voxels = act.voxels.copy()
    act.voxels[:, 1] -= (2 << act.voxels[:, 0]).astype(np.int32)
    act.origin = np.asarray(sc.origin, np.float64) + np.array([2 * sc.root_size, 0.0, 0.0])
    act.root_dims = np.array([2, sc.root_dims[1], sc.root_dims[2]])
    assert static.n > 20 and act.n > 20
    o, d = synth.random_rays(74, 300, sc.origin, sc.origin + sc.root_dims * sc.root_size)
    opts = RenderOpts(background=(0.1, 0.2, 0.3))
    got = oracle.composite_rays(oracle.prepare(static), [(oracle.prepare(act), np.eye(3), np.zeros(3))], o, d, opts)
    ref = oracle.render_rays(oracle.prepare(sc), o, d, opts)
    assert np.mean(got["n_hits"] != ref["n_hits"]) <= 0.01
    same = got["n_hits"] == ref["n_hits"]
    for k in ("rgb", "depth", "opacity", "intensity"):
        assert np.max(np.abs(got[k][same] - ref[k][same])) <= 1e-5, k
    assert int(ref["n_hits"].sum()) > 300


# ---------------------------------------------------------------- early termination
def test_early_termination_after_the_voxel_that_crosses_t_min():
    # two voxels in a row along x; the first is nearly opaque (optical depth ~ 30 along x)
    zg = np.array([[30.0] * 8, [0.5] * 8], F32)
    sc = synth.SceneData(origin=np.zeros(3), root_size=1.0, root_dims=np.array([2, 1, 1]), max_level=0,
                         voxels=np.array([[0, 0, 0, 0], [0, 1, 0, 0]], np.int32), z_geo=zg,
                         z_rgb=np.zeros((2, 3, 8), F32), z_int=np.zeros((2, 8), F32))
    ps = oracle.prepare(sc)
    o = np.array([-1.0, 0.5, 0.5], F32)
    d = np.array([1.0, 0.0, 0.0], F32)
    stop = oracle.render_ray(ps, o, d, RenderOpts(t_min=1e-6))
    full = oracle.render_ray(ps, o, d, RenderOpts(t_min=0.0))
    assert stop["n_hits"] == 1 and full["n_hits"] == 2
    assert stop["t_end"] < 1e-6 and full["t_end"] < stop["t_end"]
    # a threshold below the first voxel's transmittance lets the ray continue
    cont = oracle.render_ray(ps, o, d, RenderOpts(t_min=0.5 * stop["t_end"]))
    assert cont["n_hits"] == 2


# ---------------------------------------------------------------- rays lying on voxel faces
def test_axis_parallel_rays_on_faces_use_half_open_slabs():
    # a dense 4x4x4 block: a ray along +x lying exactly on a y (and z) face plane belongs to
    # the cells above the plane only, so its hits partition the block's x extent
    vox = np.array([[0, i, j, k] for k in range(4) for j in range(4) for i in range(4)], np.int32)
    n = vox.shape[0]
    sc = synth.SceneData(origin=np.zeros(3), root_size=1.0, root_dims=np.array([4, 4, 4]), max_level=0,
                         voxels=vox, z_geo=np.zeros((n, 8), F32), z_rgb=np.zeros((n, 3, 8), F32))
    ps = oracle.prepare(sc)
    for y, z in ((1.0, 2.0), (0.0, 0.5), (3.0, 3.0), (2.5, 1.0)):
        ids, ti, to = oracle.hit_list(ps, np.array([-2.0, y, z], F32), np.array([1.0, 0.0, 0.0], F32))
        assert ids.size == 4
        assert np.all(vox[ids, 1] == np.arange(4))
        assert np.all(vox[ids, 2] == int(y)) and np.all(vox[ids, 3] == int(z))
        assert np.array_equal(to[:-1], ti[1:])
    # on the grid's top face the ray is outside every cell
    ids, _, _ = oracle.hit_list(ps, np.array([-2.0, 4.0, 1.0], F32), np.array([1.0, 0.0, 0.0], F32))
    assert ids.size == 0


# ---------------------------------------------------------------- actors under rotated poses
_RZ90 = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.float64)    # +90 deg about z
_RX90 = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], np.float64)    # +90 deg about x


def _slab_as_actor(sc, cell_lo, cell_hi, R):
    """Cut the voxels of the root-cell box [cell_lo, cell_hi) out of `sc` into an actor scene in a
    canonical frame rotated by the signed permutation R (a world point p is the actor point
    R^T (p - t)).  The actor's grid has its min corner at its origin 0; t is the translation that
    puts it back over the box.  Voxel coordinates and the order of the 8 corner values are mapped
    by hand: actor axis j runs along world axis i where R[i, j] != 0, reversed when it is -1.
    Returns (static scene, actor scene, t)."""
    K, s0 = sc.max_level, float(sc.root_size)
    sK = s0 / (1 << K)
    lvl = sc.voxels[:, 0].astype(np.int64)
    cell = sc.voxels[:, 1:4].astype(np.int64) >> lvl[:, None]
    inside = np.all((cell >= cell_lo) & (cell < cell_hi), axis=1)
    static, act = sc.subset(~inside), sc.subset(inside)
    box_lo = np.asarray(sc.origin, float) + np.asarray(cell_lo, float) * s0
    box_hi = np.asarray(sc.origin, float) + np.asarray(cell_hi, float) * s0
    corners = np.array([[(box_lo, box_hi)[(c >> a) & 1][a] for a in range(3)] for c in range(8)])
    a_min = (corners @ R).min(axis=0)          # R^T p for each corner, row-wise
    t = R @ a_min
    dims = np.rint(np.abs(R.T) @ (np.asarray(cell_hi) - np.asarray(cell_lo))).astype(np.int64)
    # voxels: world finest-unit box -> actor metres -> actor finest units
    a_lvl = act.voxels[:, 0].astype(np.int64)
    n = np.left_shift(1, K - a_lvl)
    lo_w = np.asarray(sc.origin, float) + act.voxels[:, 1:4].astype(np.int64) * n[:, None] * sK
    hi_w = lo_w + n[:, None] * sK
    a_lo = np.minimum(lo_w @ R, hi_w @ R) - a_min
    lo_f = a_lo / sK
    assert np.allclose(lo_f, np.rint(lo_f), atol=1e-6)
    coords = np.rint(lo_f).astype(np.int64) // n[:, None]
    vox = np.concatenate([a_lvl[:, None], coords], 1).astype(np.int32)
    # corner c' of the actor voxel (bits b'_j) sits at world corner bits b_i = b'_j or 1 - b'_j
    perm = np.empty(8, np.int64)
    for cp in range(8):
        c = 0
        for i in range(3):
            j = int(np.nonzero(R[i])[0][0])
            bj = (cp >> j) & 1
            c |= (bj if R[i, j] > 0 else 1 - bj) << i
        perm[cp] = c
    actor = synth.SceneData(origin=np.zeros(3), root_size=s0, root_dims=dims, max_level=K, voxels=vox,
                            z_geo=act.z_geo[:, perm].copy(), z_rgb=act.z_rgb[:, :, perm].copy(),
                            z_int=None if act.z_int is None else act.z_int[:, perm].copy(), name="actor")
    return static, actor, t


@pytest.mark.parametrize("rot", ["z90", "x90", "z90x90"])
def test_composite_rotated_actor_equals_the_merged_scene(rot):
    """A slab of root cells moved into an actor whose canonical frame is rotated by an exact 90 deg
    turn (about z, about x, and both) and translated by whole cells renders like the original
    scene.  A transposed R, or t applied after the rotation, sends the actor's rays elsewhere."""
    R = {"z90": _RZ90, "x90": _RX90, "z90x90": _RZ90 @ _RX90}[rot]
    sc = synth.random_scene(75, root_dims=(6, 4, 3), max_level=2, fill=0.7, origin=(-3.0, -2.0, -1.5))
    static, actor, t = _slab_as_actor(sc, (2, 1, 0), (4, 4, 3), R)
    assert static.n > 20 and actor.n > 20
    o, d = synth.random_rays(76, 400, sc.origin, sc.origin + sc.root_dims * sc.root_size)
    opts = RenderOpts(background=(0.1, 0.2, 0.3))
    got = oracle.composite_rays(oracle.prepare(static), [(oracle.prepare(actor), R, t)], o, d, opts)
    ref = oracle.render_rays(oracle.prepare(sc), o, d, opts)
    # up to the rounding of the actor frame's own origin, the hit lists are the same
    assert np.mean(got["n_hits"] != ref["n_hits"]) <= 0.01
    same = got["n_hits"] == ref["n_hits"]
    for k in ("rgb", "depth", "opacity", "intensity"):
        assert np.max(np.abs(got[k][same] - ref[k][same])) <= 1e-5, k
    # the actor's voxels are really met: the rays that cross the slab see them
    assert int(ref["n_hits"].sum()) > 400
    # the transposed rotation is a different pose: it does not reproduce the scene
    bad = oracle.composite_rays(oracle.prepare(static), [(oracle.prepare(actor), R.T, t)], o, d, opts)
    assert np.mean(bad["n_hits"] != ref["n_hits"]) > 0.05


def _segments_closed_form(segs, S, bg):
    """Outputs of constant-field segments (sigma, rgb, intensity, t_in, t_out) composited front to
    back with S midpoint samples each (Eq. 3-4 written out for constant density)."""
    T, C, D, I = 1.0, np.zeros(3), 0.0, 0.0
    for sig, col, inten, t0, t1 in segs:
        L = t1 - t0
        tau = sig * L / S
        for k in range(S):
            w = T * math.exp(-k * tau) * (1.0 - math.exp(-tau))
            C += w * np.asarray(col)
            D += w * (t0 + (k + 0.5) * L / S)
            I += w * inten
        T *= math.exp(-sig * L)
    return C + T * np.asarray(bg), D, 1.0 - T, I


@pytest.mark.parametrize("S", [1, 3])
def test_composite_overlapping_boxes_hand_derived(S):
    """Two actors whose boxes overlap along a ray: each box is walked whole in order of entry, and
    the static scene resumes after the furthest exit, so a static voxel inside the boxes' span is
    skipped.  Static cells 0, 2, 4 of a 6 x 1 x 1 grid of 1 m cells; actor A is one 2 m voxel over
    x in [1, 3], actor B (turned 90 deg about x) one over x in [2, 4]; the ray runs along +x from
    x = -1.  Segments: static cell 0 on t in [1, 2], A on [2, 4], B on [3, 5], static cell 4 on
    [5, 6]."""
    zs = {0: -1.0, 2: 2.0, 4: 0.5}
    cols = {0: (0.25, -0.5, 1.0), 2: (1.5, 1.5, 1.5), 4: (-1.0, 0.75, 0.0)}
    ints = {0: 0.5, 2: -2.0, 4: 1.25}
    cells = sorted(zs)
    static = synth.SceneData(origin=np.zeros(3), root_size=1.0, root_dims=np.array([6, 1, 1]), max_level=0,
                             voxels=np.array([[0, c, 0, 0] for c in cells], np.int32),
                             z_geo=np.array([[zs[c]] * 8 for c in cells], F32),
                             z_rgb=np.array([np.repeat(np.array(cols[c])[:, None], 8, 1) for c in cells], F32),
                             z_int=np.array([[ints[c]] * 8 for c in cells], F32))
    a = synth.single_voxel_scene(np.full(8, 0.0), np.repeat(np.array([0.5, 0.0, -0.5])[:, None], 8, 1),
                                 np.full(8, -0.25), root_size=2.0)
    b = synth.single_voxel_scene(np.full(8, -0.5), np.repeat(np.array([-0.25, 1.0, 0.25])[:, None], 8, 1),
                                 np.full(8, 0.75), root_size=2.0)
    poses = [(np.eye(3), np.array([1.0, -0.5, -0.5])), (_RX90, np.array([2.0, 1.5, -0.5]))]
    o = np.array([[-1.0, 0.5, 0.5]], F32)
    d = np.array([[1.0, 0.0, 0.0]], F32)
    bg = (0.1, 0.2, 0.3)
    opts = RenderOpts(samples=S, t_min=0.0, background=bg)
    got = oracle.composite_rays(oracle.prepare(static), [(oracle.prepare(a), *poses[0]), (oracle.prepare(b), *poses[1])],
                                o, d, opts)
    seg = [(_sp(zs[0]), [_sig(x) for x in cols[0]], _sig(ints[0]), 1.0, 2.0),
           (_sp(0.0), [_sig(x) for x in (0.5, 0.0, -0.5)], _sig(-0.25), 2.0, 4.0),
           (_sp(-0.5), [_sig(x) for x in (-0.25, 1.0, 0.25)], _sig(0.75), 3.0, 5.0),
           (_sp(zs[4]), [_sig(x) for x in cols[4]], _sig(ints[4]), 5.0, 6.0)]
    C, D, O, I = _segments_closed_form(seg, S, bg)
    assert got["n_hits"][0] == 4
    assert np.allclose(got["rgb"][0], C, atol=1e-12, rtol=0)
    assert abs(got["depth"][0] - D) < 1e-12 and abs(got["opacity"][0] - O) < 1e-12
    assert abs(got["intensity"][0] - I) < 1e-12


# ---------------------------------------------------------------- paper-field intensity
def test_paper_field_intensity_closed_forms():
    """Eq. 1 density with zero slopes is constant, so O = 1 - exp(-sigma L); the intensity
    sigmoid(w_I . [x, 1]) with zero slopes is sigmoid(b) everywhere, so I = sigmoid(b) O.  With
    slopes along x and z only, a ray along +y at fixed local (x0, z0) sees the constant
    sigmoid(w_x x0 + w_z z0 + b): this pins the slot and the sign of each slope."""
    b_sig, b_int = -0.5, 0.75
    for w, (x0, z0) in (((0.0, 0.0, 0.0), (0.25, -0.5)), ((1.5, 0.0, -2.0), (0.25, -0.5)),
                        ((1.5, 0.0, -2.0), (-0.75, 0.5))):
        zg = np.zeros(8)
        zg[3] = b_sig
        zi = np.zeros(8)
        zi[:3], zi[3] = w, b_int
        sc = synth.single_voxel_scene(zg, np.zeros((3, 8)), zi, root_size=2.0, origin=(-1.0, -1.0, -1.0))
        ps = oracle.prepare(sc)
        o = np.array([x0, -3.0, z0], F32)
        d = np.array([0.0, 1.0, 0.0], F32)
        for S in (1, 4):
            out = oracle.render_ray(ps, o, d, RenderOpts(samples=S, field="paper", t_min=0.0))
            O = 1.0 - math.exp(-math.exp(b_sig) * 2.0)
            assert abs(out["opacity"] - O) < 1e-12
            assert abs(out["intensity"] - _sig(w[0] * x0 + w[2] * z0 + b_int) * O) < 1e-12


# ------------------------------------------------------------------ tile-based splatting (Sec. 3.2)
def _raster_cameras(data):
    """Pinholes around and inside an adaptive scene: outside looking in (ragged 40 x 30 image, 3 x 2
    tiles), looking straight down, inside the grid, and with the eye exactly on root and mid planes."""
    lo = np.asarray(data.origin, np.float64)
    ext = np.asarray(data.root_dims, np.float64) * data.root_size
    c = lo + ext / 2
    s0 = data.root_size
    eyes = [(c + np.array([1.3, -1.1, 0.7]) * ext.max(), c, 70.0),
            (c + np.array([0.05, 0.02, 1.5]) * ext.max(), c, 60.0),
            (lo + np.array([0.37, 0.41, 0.33]) * ext, c + np.array([0.2, 0.1, 0.05]) * ext, 100.0),
            (lo + np.array([2.0, 1.5, 1.0]) * s0, c + np.array([0.3, 0.2, -0.1]) * ext, 90.0),
            (lo + np.array([1.5, 2.25, 0.5]) * s0, lo + np.array([0.9, 0.2, 0.8]) * ext, 90.0)]
    return [synth.pinhole(40, 30, fov, synth.look_at(e, t), e) for e, t, fov in eyes]


@pytest.mark.parametrize("seed,K", [(301, 1), (302, 2), (303, 3)])
def test_raster_octree_order_equals_ray_casting(seed, K):
    """With the front-to-back octree key, splatting composites every pixel's hits in its ray's t_in
    order, so each pixel equals the ray cast of its ray exactly (every output, float64 ==), for
    cameras outside, above and inside the grid, eyes on grid planes, S = 1 and 4, with and without
    early termination; every composited list is the prefix of the pixel ray's hit list."""
    data = synth.random_scene(seed, root_dims=(5, 4, 3), max_level=K, fill=0.7)
    ps = oracle.prepare(data)
    for cam, (S, tmin, bg) in zip(_raster_cameras(data), [(4, 1e-6, (0.1, 0.2, 0.3)), (1, 0.0, (0, 0, 0)),
                                                           (4, 1e-2, (0.5, 0.5, 0.5)), (1, 1e-6, (0, 0, 0)),
                                                           (2, 1e-6, (0.2, 0.1, 0.0))]):
        opts = RenderOpts(samples=S, t_min=tmin, background=bg)
        out, comp = oracle.raster(ps, cam, opts)
        o, d, _, _ = oracle.sensor_rays(cam)
        o, d = o.astype(F32), d.astype(F32)
        ref = oracle.render_rays(ps, o, d, opts)
        for k in out:
            assert np.array_equal(out[k], ref[k]), k
        hit = 0
        for r in range(o.shape[0]):
            ids, _, _ = oracle.hit_list(ps, o[r], d[r])
            n = int(ref["n_hits"][r])
            assert np.array_equal(comp[r], ids[:n]), r
            hit += n
        assert hit > 200


def test_raster_keys_increase_along_every_ray_and_centre_depth_does_not():
    """The octree key strictly increases along the hit list of every pixel ray, whatever the eye's
    position; the centre-depth key (the 3D Gaussian splatting order) inverts some neighbouring
    hits, so splatting in that order differs from ray casting at some pixels."""
    bad_centre = 0
    for seed, K in ((311, 2), (312, 3)):
        data = synth.random_scene(seed, root_dims=(5, 4, 3), max_level=K, fill=0.8)
        ps = oracle.prepare(data)
        for cam in _raster_cameras(data):
            o, d, _, _ = oracle.sensor_rays(cam)
            o, d = o.astype(F32), d.astype(F32)
            kc = {}
            for r in range(0, o.shape[0], 3):
                ids, _, _ = oracle.hit_list(ps, o[r], d[r])
                ko = [oracle.depth_key(ps, cam, int(v)) for v in ids]
                assert all(a < b for a, b in zip(ko, ko[1:])), (seed, r)
                for v in ids:
                    if v not in kc:
                        kc[v] = oracle.depth_key(ps, cam, int(v), kind="centre")
                c = [kc[v] for v in ids]
                bad_centre += sum(a > b for a, b in zip(c, c[1:]))
    assert bad_centre > 0
    data = synth.random_scene(312, root_dims=(5, 4, 3), max_level=3, fill=0.8)
    ps = oracle.prepare(data)
    cam = _raster_cameras(data)[2]
    o, d, _, _ = oracle.sensor_rays(cam)
    ref = oracle.render_rays(ps, o.astype(F32), d.astype(F32), RenderOpts(t_min=0.0))
    out, _ = oracle.raster(ps, cam, RenderOpts(t_min=0.0), kind="centre")
    differ = np.sum(np.abs(out["depth"] - ref["depth"]) > 1e-9)
    assert differ > 0 and np.array_equal(out["t_end"] > 0, ref["t_end"] > 0)


def test_raster_culling_and_footprints():
    """Voxels wholly behind the camera are culled and no pixel ray hits them; a voxel reaching
    across the camera plane covers every tile; every voxel a pixel ray hits is in the list of that
    pixel's tile (and a one-voxel scene seen head-on covers exactly the tiles its image touches)."""
    data = synth.random_scene(321, root_dims=(6, 4, 3), max_level=2, fill=0.8)
    ps = oracle.prepare(data)
    lo = np.asarray(data.origin, np.float64)
    eye = lo + np.array([3.02, 2.01, 1.53]) * data.root_size       # inside the grid, looking +x
    cam = synth.pinhole(48, 32, 90.0, synth.look_at(eye, eye + np.array([1.0, 0.0, 0.0])), eye)
    fps = oracle.footprints(ps, cam)
    o, d, _, _ = oracle.sensor_rays(cam)
    o, d = o.astype(F32), d.astype(F32)
    gs = ps.gs
    xmax = ps.origin[0] + (ps.lo_i[:, 0] + ps.n_i) / gs
    xmin = ps.origin[0] + ps.lo_i[:, 0] / gs
    behind = xmax <= eye[0]
    straddle = (xmin < eye[0]) & (xmax > eye[0])
    assert behind.sum() > 10 and straddle.sum() > 0
    for v in np.nonzero(behind)[0]:
        assert fps[v] is None
    for v in np.nonzero(straddle)[0]:
        assert fps[v] == (0, 0, 2, 1)
    lists = oracle.tile_lists(ps, cam)
    for r in range(o.shape[0]):
        ids, _, _ = oracle.hit_list(ps, o[r], d[r])
        assert not np.any(behind[ids])
        tile = lists.get(((r % 48) // 16, (r // 48) // 16), np.zeros(0, np.int64))
        assert np.all(np.isin(ids, tile)), r
    # one voxel filling the middle of a 64 x 64 view: its image spans pixels 16..47 (2 x 2 tiles)
    one = synth.single_voxel_scene(np.zeros(8, F32), np.zeros((3, 8), F32), root_size=2.0, origin=(-1.0, -1.0, -1.0))
    ps1 = oracle.prepare(one)
    f = 32.0 / math.tan(math.radians(45.0))                         # 90 deg: fx = 32
    eye = np.array([0.0, 0.0, -5.0])                                 # the near face at z = -1 is 4 m away
    cam = synth.pinhole(64, 64, 90.0, synth.look_at(eye, (0.0, 0.0, 0.0), up=(0.0, -1.0, 0.0)), eye)
    assert abs(cam["fx"] - f) < 1e-9
    # near face corners project to 32 +- 32 * 1/4 = 24..40, far face (6 m) to 32 +- 32/6
    assert oracle.footprints(ps1, cam, margin=0.0) == [(1, 1, 2, 2)]
    assert oracle.footprints(ps1, cam, margin=9.0) == [(0, 0, 3, 3)]
