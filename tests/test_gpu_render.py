"""GPU parity of the HIP renderer against the CPU oracle (all calls go through the C ABI).

Bar: hit lists bit-exact (ids, t_in, t_out); colour, opacity and intensity within 1e-4 absolute;
depth within 1e-3 m; n_hits equal.  Rays fed to both sides come from the oracle's sensor models
(float64, rounded to float32) or from the seeded generators; nothing the GPU computes is used
as an oracle input.
"""
import math

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.render import RenderOpts

pytestmark = pytest.mark.gpu

TOL_C, TOL_D = 1e-4, 1e-3
F32 = np.float32


@pytest.fixture(scope="module")
def salf():
    import paper_2507_18713_amd as m
    return m


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def check_hits(salf, scene, ps, o, d, max_hits=256, t_near=0.0, t_far=math.inf, idx=None):
    """GPU trace_hits vs the oracle's brute force, bit for bit."""
    idx = np.arange(o.shape[0]) if idx is None else idx
    counts, ids, ti, to = salf.trace_hits(scene, to_dev(o[idx]), to_dev(d[idx]), max_hits, t_near, t_far)
    counts, ids, ti, to = (x.cpu().numpy() for x in (counts, ids, ti, to))
    total = 0
    for q, r in enumerate(idx):
        e_ids, e_ti, e_to = oracle.hit_list(ps, o[r], d[r], t_near, t_far)
        assert counts[q] == e_ids.size, (r, counts[q], e_ids.size)
        k = min(e_ids.size, max_hits)
        assert np.array_equal(ids[q, :k], e_ids[:k]), r
        assert np.array_equal(ti[q, :k].view(np.uint32), e_ti[:k].view(np.uint32)), r
        assert np.array_equal(to[q, :k].view(np.uint32), e_to[:k].view(np.uint32)), r
        total += e_ids.size
    return total


def check_outputs(got, ref, idx=None, keys=("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")):
    for k in keys:
        if k not in got:
            continue
        g = got[k].cpu().numpy()
        g = g if idx is None else g[idx]
        e = ref[k]
        if k == "n_hits":
            assert np.array_equal(g, e), k
            continue
        tol = TOL_D if k == "depth" else TOL_C
        err = np.max(np.abs(g.astype(np.float64) - e)) if g.size else 0.0
        assert err <= tol, (k, err)


def oracle_rays(sensor):
    o, d, t, valid = oracle.sensor_rays(sensor)
    return o.astype(F32), d.astype(F32), valid


# ------------------------------------------------------------------ tiny scene (config 0)
@pytest.mark.parametrize("S", [1, 4])
def test_tiny_scene_all_rays(salf, S):
    data = synth.config0_scene()
    ps = oracle.prepare(data)
    scene = salf.Scene.from_data(data, device=dev())
    o, d, _ = oracle_rays(synth.config0_camera())
    n_hit = check_hits(salf, scene, ps, o, d)
    assert n_hit > 5000
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
    got = salf.render(scene, o=to_dev(o), d=to_dev(d), samples=S, outputs=outs, image_width=64)
    ref = oracle.render_rays(ps, o, d, RenderOpts(samples=S))
    check_outputs(got, ref)
    # linear (untiled) launch gives the same bits
    lin = salf.render(scene, o=to_dev(o), d=to_dev(d), samples=S, outputs=outs)
    for k in outs:
        assert torch.equal(lin[k], got[k]), k


# index: the dense-leaf-index level of the scene (0: octree walk only; 2 with K = 3 mixes the two
# walks, since cells whose finest level is 3 keep the octree)
@pytest.mark.parametrize("seed,K,index", [(31, 1, 4), (32, 2, 4), (33, 3, 4), (32, 2, 0), (33, 3, 0), (33, 3, 2)])
def test_adaptive_scenes_random_rays(salf, seed, K, index):
    data = synth.random_scene(seed, root_dims=(5, 4, 3), max_level=K)
    ps = oracle.prepare(data)
    scene = salf.Scene.from_data(data, device=dev(), index_level=index)
    lo, hi = data.origin, data.origin + data.root_dims * data.root_size
    o, d = synth.random_rays(seed, 700, lo, hi)
    # axis-parallel rays, rays on faces and rays from inside a voxel exercise the rule's corners
    d[:6] = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1]], F32)
    o[6:12] = (data.origin + np.array([1.0, 1.0, 1.0]) * data.root_size).astype(F32)
    check_hits(salf, scene, ps, o, d)
    bg = (0.2, 0.3, 0.4)
    got = salf.render(scene, o=to_dev(o), d=to_dev(d), background=bg,
                      outputs=("rgb", "depth", "opacity", "intensity", "t_end", "n_hits"))
    check_outputs(got, oracle.render_rays(ps, o, d, RenderOpts(background=bg)))
    st = scene.stats()
    assert st["n_voxels"] == data.n and st["n_nodes"] > 0


def test_dense_index_changes_nothing(salf):
    """Renders, hit lists and gradients are the same bits with the dense leaf index at every level
    (cells above the level keep the octree walk) and without it."""
    data = synth.random_scene(35, root_dims=(4, 3, 3), max_level=4)
    scene = salf.Scene.from_data(data, device=dev(), index_level=0, requires_grad=True)
    lo, hi = data.origin, data.origin + data.root_dims * data.root_size
    o, d = synth.random_rays(36, 6000, lo, hi)
    d[:6] = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1]], F32)
    o[6:12] = (data.origin + np.array([1.0, 1.0, 1.0]) * data.root_size).astype(F32)
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")

    def run():
        r = salf.render(scene, o=to_dev(o), d=to_dev(d), outputs=outs, image_width=50)
        h = salf.trace_hits(scene, to_dev(o), to_dev(d), max_hits=512)
        grads = {"rgb": torch.ones_like(r["rgb"]), "depth": torch.full_like(r["depth"], 0.5),
                 "intensity": torch.ones_like(r["intensity"])}
        g = salf.render_backward(scene, r, grads, o=to_dev(o), d=to_dev(d), image_width=50)
        return r, h, g

    r0, h0, g0 = run()
    assert int(r0["n_hits"].sum()) > 12000 and g0[0].abs().sum() > 0
    for level in (1, 2, 3, 4, 6):
        scene.build_index(level)
        r, h, g = run()
        for k in outs:
            assert torch.equal(r[k], r0[k]), (level, k)
        for a, b in zip(h, h0):  # entries past a ray's count are NaN on both sides
            assert torch.equal(a, b) or bool(torch.all((a == b) | (torch.isnan(a) & torch.isnan(b)))), level
        for a, b in zip(g, g0):  # same hits; only the order of the gradient atomics may differ
            assert torch.allclose(a, b, rtol=1e-5, atol=1e-6), level
    scene.build_index(0)
    assert scene.index is None


def test_dense_index_errors(salf):
    from paper_2507_18713_amd._lib import MAX_INDEX_LEVEL, call
    data = synth.random_scene(37, root_dims=(3, 3, 2), max_level=3)
    scene = salf.Scene.from_data(data, device=dev(), index_level=0)
    nbytes = ctypes.c_size_t()
    for bad in (-1, MAX_INDEX_LEVEL + 1):
        with pytest.raises(salf.SalfError, match="index level"):
            call("salf_scene_index_size", scene.ctx.handle, scene.id, bad, ctypes.byref(nbytes))
    call("salf_scene_index_size", scene.ctx.handle, scene.id, 3, ctypes.byref(nbytes))
    need = int(nbytes.value)
    assert need >= 256
    buf = torch.empty(need + 256, dtype=torch.uint8, device=dev())
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(salf.SalfError, match="needs"):
        call("salf_scene_build_index", scene.ctx.handle, scene.id, 3, buf.data_ptr(), need - 4, stream)
    with pytest.raises(salf.SalfError, match="aligned"):
        call("salf_scene_build_index", scene.ctx.handle, scene.id, 3, buf.data_ptr() + 4, need, stream)
    with pytest.raises(salf.SalfError, match="no scene"):
        call("salf_scene_index_size", scene.ctx.handle, 999, 3, ctypes.byref(nbytes))
    # a failed build leaves the scene without an index; a good one renders as before
    o, d = synth.random_rays(38, 300, data.origin, data.origin + data.root_dims * data.root_size)
    ref = salf.render(scene, o=to_dev(o), d=to_dev(d), outputs=("rgb", "n_hits"))
    call("salf_scene_build_index", scene.ctx.handle, scene.id, 3, buf.data_ptr(), need, stream)
    got = salf.render(scene, o=to_dev(o), d=to_dev(d), outputs=("rgb", "n_hits"))
    assert torch.equal(got["rgb"], ref["rgb"]) and torch.equal(got["n_hits"], ref["n_hits"])


def test_paper_field_forward(salf):
    data = synth.random_scene(41, root_dims=(5, 4, 3), max_level=2)
    # Eq. 1-2 parameters: bias N(0,1), slopes N(0, 0.5^2), SH DC N(0,1), SH higher N(0, 0.25^2)
    rng = np.random.default_rng(42)
    n = data.n
    geo = np.zeros((n, 8), F32)
    geo[:, :3] = rng.normal(0, 0.5, (n, 3))
    geo[:, 3] = rng.normal(0, 1, n)
    rgb = np.zeros((n, 3, 8), F32)
    rgb[:, :, :3] = rng.normal(0, 0.5, (n, 3, 3))
    rgb[:, :, 3] = rng.normal(0, 1, (n, 3))
    rgb[:, :, 4:7] = rng.normal(0, 0.25, (n, 3, 3))
    ity = np.zeros((n, 8), F32)
    ity[:, :4] = rng.normal(0, 0.5, (n, 4))
    data.z_geo, data.z_rgb, data.z_int = geo, rgb, ity
    ps = oracle.prepare(data)
    scene = salf.Scene.from_data(data, device=dev(), field="paper")
    o, d = synth.random_rays(43, 600, data.origin, data.origin + data.root_dims * data.root_size)
    for S in (1, 4):
        got = salf.render(scene, o=to_dev(o), d=to_dev(d), samples=S,
                          outputs=("rgb", "depth", "opacity", "intensity", "n_hits"))
        check_outputs(got, oracle.render_rays(ps, o, d, RenderOpts(samples=S, field="paper")))


def test_sdf_field_forward(salf):
    """The SDF variant (Eq. 5-6): affine signed distance, density a/2 + a/2 sign(s) (1 - e^{-|s|/b})
    with a = exp(geo[4]), b = exp(geo[5]); colour and intensity as the paper field."""
    data = synth.random_scene(44, root_dims=(5, 4, 3), max_level=2)
    rng = np.random.default_rng(45)
    n = data.n
    geo = np.zeros((n, 8), F32)
    geo[:, :3] = rng.normal(0, 0.6, (n, 3))
    geo[:, 3] = rng.normal(0, 0.5, n)
    geo[:, 4] = rng.normal(0.5, 0.3, n)
    geo[:, 5] = rng.normal(-1.0, 0.3, n)
    rgb = np.zeros((n, 3, 8), F32)
    rgb[:, :, :7] = rng.normal(0, 0.5, (n, 3, 7))
    ity = np.zeros((n, 8), F32)
    ity[:, :4] = rng.normal(0, 0.5, (n, 4))
    data.z_geo, data.z_rgb, data.z_int = geo, rgb, ity
    ps = oracle.prepare(data)
    scene = salf.Scene.from_data(data, device=dev(), field="sdf")
    o, d = synth.random_rays(46, 600, data.origin, data.origin + data.root_dims * data.root_size)
    for S in (1, 4):
        got = salf.render(scene, o=to_dev(o), d=to_dev(d), samples=S,
                          outputs=("rgb", "depth", "opacity", "intensity", "n_hits"))
        check_outputs(got, oracle.render_rays(ps, o, d, RenderOpts(samples=S, field="sdf")))
    assert float(got["opacity"].max()) > 0.5


def test_tiny_scene_paper_field_camera(salf):
    data = synth.config0_scene()
    rng = np.random.default_rng(44)
    data.z_geo = np.concatenate([rng.normal(0, 0.5, (data.n, 3)), rng.normal(0, 1, (data.n, 1)),
                                 np.zeros((data.n, 4))], 1).astype(F32)
    ps = oracle.prepare(data)
    scene = salf.Scene.from_data(data, device=dev(), field="paper")
    o, d, _ = oracle_rays(synth.config0_camera())
    got = salf.render(scene, o=to_dev(o), d=to_dev(d), image_width=64, outputs=("rgb", "depth", "opacity"))
    check_outputs(got, oracle.render_rays(ps, o, d, RenderOpts(field="paper")))


# ------------------------------------------------------------------ edge cases
def test_empty_scene_and_misses(salf):
    empty = synth.SceneData(origin=np.zeros(3), root_size=1.0, root_dims=np.array([3, 3, 3]), max_level=2,
                            voxels=np.zeros((0, 4), np.int32), z_geo=np.zeros((0, 8), F32),
                            z_rgb=np.zeros((0, 3, 8), F32), z_int=np.zeros((0, 8), F32))
    scene = salf.Scene.from_data(empty, device=dev())
    o, d = synth.random_rays(1, 100, (0, 0, 0), (3, 3, 3))
    bg = (0.25, 0.5, 0.75)
    got = salf.render(scene, o=to_dev(o), d=to_dev(d), background=bg, outputs=("rgb", "depth", "opacity", "n_hits"))
    assert torch.all(got["rgb"].cpu() == torch.tensor(bg)) and torch.all(got["opacity"] == 0)
    assert torch.all(got["depth"] == 0) and torch.all(got["n_hits"] == 0)
    # zero rays
    z = torch.zeros((0, 3), device=dev())
    got = salf.render(scene, o=z, d=z, outputs=("rgb",))
    assert got["rgb"].shape == (0, 3)
    # refining an empty scene gives an empty scene
    out = scene.refine(None, 0.0)
    assert out["voxels"].shape == (0, 4) and out["geo"].shape == (0, 8)


def test_refine_and_index_edge_cases(salf):
    from paper_2507_18713_amd._lib import RefineOpts, call
    # a scene of level-0 voxels only (K = 0): no octree cells, so the index is empty, and no voxel
    # can split
    data = synth.random_scene(61, root_dims=(4, 3, 3), max_level=0, fill=0.5)
    scene = salf.Scene.from_data(data, device=dev(), index_level=0)
    o, d = synth.random_rays(62, 400, data.origin, data.origin + data.root_dims * data.root_size)
    ref = salf.render(scene, o=to_dev(o), d=to_dev(d), outputs=("rgb", "n_hits"))
    scene.build_index(4)
    got = salf.render(scene, o=to_dev(o), d=to_dev(d), outputs=("rgb", "n_hits"))
    assert torch.equal(got["rgb"], ref["rgb"]) and torch.equal(got["n_hits"], ref["n_hits"])
    big = torch.full((data.n, 3, 8), 1e3, device=dev())
    out = scene.refine(big, 0.0, 0.0)
    assert torch.equal(out["voxels"], to_dev(data.voxels, torch.int32))
    # argument errors
    nb = ctypes.c_size_t()
    call("salf_refine_work_size", scene.n, ctypes.byref(nb))
    work = torch.empty(int(nb.value), dtype=torch.uint8, device=dev())
    n_out = ctypes.c_int64()
    stream = torch.cuda.current_stream().cuda_stream
    for bad in (RefineOpts(-1.0, 0.0), RefineOpts(0.0, 2.0), RefineOpts(float("nan"), 0.0)):
        with pytest.raises(salf.SalfError, match="grad_threshold"):
            call("salf_refine", scene.ctx.handle, scene.id, scene._voxels.data_ptr(), None, ctypes.byref(bad),
                 work.data_ptr(), int(work.numel()), None, None, None, None, 0, ctypes.byref(n_out), stream)
    with pytest.raises(salf.SalfError, match="work area"):
        call("salf_refine", scene.ctx.handle, scene.id, scene._voxels.data_ptr(), None,
             ctypes.byref(RefineOpts(0.0, 0.0)), work.data_ptr(), 16, None, None, None, None, 0,
             ctypes.byref(n_out), stream)
    with pytest.raises(salf.SalfError, match="OUT_OF_MEMORY"):
        call("salf_refine", scene.ctx.handle, scene.id, scene._voxels.data_ptr(), None,
             ctypes.byref(RefineOpts(0.0, 0.0)), work.data_ptr(), int(work.numel()), None, None, None, None, 0,
             ctypes.byref(n_out), stream)
    assert n_out.value == data.n


def test_invalid_rays_render_background(salf):
    data = synth.random_scene(51)
    scene = salf.Scene.from_data(data, device=dev())
    o = np.zeros((4, 3), F32)
    d = np.array([[0, 0, 0], [np.nan, 0, 1], [1, 0, np.inf], [0.0, 0.0, 1e-45]], F32)
    got = salf.render(scene, o=to_dev(o), d=to_dev(d), background=(1, 0, 0), outputs=("rgb", "opacity", "n_hits"))
    assert torch.all(got["n_hits"] == 0) and torch.all(got["opacity"] == 0)
    assert torch.all(got["rgb"].cpu() == torch.tensor([1.0, 0.0, 0.0]))


def test_near_far_clipping(salf):
    data = synth.random_scene(52, root_dims=(6, 5, 4), max_level=2)
    ps = oracle.prepare(data)
    scene = salf.Scene.from_data(data, device=dev())
    o, d = synth.random_rays(53, 500, data.origin, data.origin + data.root_dims * data.root_size)
    check_hits(salf, scene, ps, o, d, t_near=1.5, t_far=4.0)
    got = salf.render(scene, o=to_dev(o), d=to_dev(d), t_near=1.5, t_far=4.0,
                      outputs=("rgb", "depth", "opacity", "n_hits"))
    check_outputs(got, oracle.render_rays(ps, o, d, RenderOpts(t_near=1.5, t_far=4.0)))


def test_early_termination_and_max_samples(salf):
    data = synth.random_scene(54, root_dims=(6, 5, 4), max_level=1, fill=0.9)
    data.z_geo = (data.z_geo + 3.0).astype(F32)          # dense: most rays stop early
    ps = oracle.prepare(data)
    scene = salf.Scene.from_data(data, device=dev())
    o, d = synth.random_rays(55, 500, data.origin, data.origin + data.root_dims * data.root_size)
    for S, tmin in ((4, 1e-6), (4, 1e-2), (32, 1e-6), (3, 0.0)):
        got = salf.render(scene, o=to_dev(o), d=to_dev(d), samples=S, t_min=tmin,
                          outputs=("rgb", "depth", "opacity", "t_end", "n_hits"))
        ref = oracle.render_rays(ps, o, d, RenderOpts(samples=S, t_min=tmin))
        check_outputs(got, ref)
        if tmin > 0:
            full = oracle.render_rays(ps, o, d, RenderOpts(samples=S, t_min=0.0))
            assert np.sum(ref["n_hits"] < full["n_hits"]) > 20


@pytest.mark.parametrize("field,preact", [("corner", False), ("corner", True), ("paper", False), ("sdf", False)])
def test_trace_with_early_termination_lists_what_the_render_shades(salf, field, preact):
    """salf_trace_hits with early termination: each ray's list is the prefix of its full list (the
    oracle's, bit for bit) that the render composites, its count equal to the render's n_hits."""
    data = synth.random_scene(56, root_dims=(6, 5, 4), max_level=2, fill=0.9)
    if field == "corner":
        data.z_geo = (data.z_geo + 3.0).astype(F32)      # dense: most rays stop early
    else:                                                # affine density / SDF parameters
        rng = np.random.default_rng(57)
        data.z_geo = np.zeros_like(data.z_geo)
        data.z_geo[:, :3] = rng.normal(0, 0.5, (data.n, 3))
        data.z_geo[:, 3] = rng.normal(2.5, 0.5, data.n) if field == "paper" else rng.normal(0.5, 0.3, data.n)
        if field == "sdf":
            data.z_geo[:, 4] = rng.normal(2.0, 0.2, data.n)
            data.z_geo[:, 5] = rng.normal(-1.0, 0.2, data.n)
        data.z_geo = data.z_geo.astype(F32)
    ps = oracle.prepare(data)
    scene = salf.Scene.from_data(data, device=dev(), field=field, preactivate=preact)
    o, d = synth.random_rays(58, 600, data.origin, data.origin + data.root_dims * data.root_size)
    for S, tmin in ((4, 1e-6), (1, 1e-2)):
        got = salf.render(scene, o=to_dev(o), d=to_dev(d), samples=S, t_min=tmin, outputs=("n_hits",))
        cnt, ids, ti, to = salf.trace_hits(scene, to_dev(o), to_dev(d), 256, early_termination=True, samples=S,
                                           t_min=tmin)
        full, fids, _, _ = salf.trace_hits(scene, to_dev(o), to_dev(d), 256)
        cnt, ids, full, fids = (x.cpu().numpy() for x in (cnt, ids, full, fids))
        assert np.array_equal(cnt, got["n_hits"].cpu().numpy())
        assert np.sum(cnt < full) > 50
        for r in range(o.shape[0]):
            e_ids, _, _ = oracle.hit_list(ps, o[r], d[r])
            assert np.array_equal(fids[r, :full[r]], e_ids) and np.array_equal(ids[r, :cnt[r]], e_ids[:cnt[r]]), r


def test_step_budget_cuts_rays_short_and_is_reported(salf):
    """A tiny traversal step budget, forced from the host, cuts walks short: the kernels end normally,
    the next sync reports how many rays were cut (once), and the default budget renders as before."""
    data = synth.random_scene(59, root_dims=(6, 5, 4), max_level=2, fill=0.9)
    scene = salf.Scene.from_data(data, device=dev())
    o, d = synth.random_rays(60, 400, data.origin, data.origin + data.root_dims * data.root_size)
    ref = salf.render(scene, o=to_dev(o), d=to_dev(d), outputs=("rgb", "n_hits"))
    scene.ctx.sync()
    try:
        scene.ctx.set_step_budget(6)
        cut = salf.render(scene, o=to_dev(o), d=to_dev(d), outputs=("rgb", "n_hits"))
        with pytest.raises(salf.SalfError, match="TRUNCATED") as err:
            scene.ctx.sync()
        n_cut = int(str(err.value).split(": ")[-1].split(" ")[0])
        shorter = int((cut["n_hits"] < ref["n_hits"]).sum())
        assert 0 < shorter <= n_cut <= o.shape[0]
        scene.ctx.sync()                                 # reported once
    finally:
        scene.ctx.set_step_budget(1 << 22)
    again = salf.render(scene, o=to_dev(o), d=to_dev(d), outputs=("rgb", "n_hits"))
    scene.ctx.sync()
    assert torch.equal(again["rgb"], ref["rgb"]) and torch.equal(again["n_hits"], ref["n_hits"])
    with pytest.raises(salf.SalfError, match="INVALID_ARG"):
        scene.ctx.set_step_budget(0)


def test_upload_order_only_renames(salf):
    data = synth.random_scene(56)
    perm = np.random.default_rng(57).permutation(data.n)
    a = salf.Scene.from_data(data, device=dev())
    b = salf.Scene.from_data(data.permuted(perm), device=dev())
    o, d = synth.random_rays(58, 400, data.origin, data.origin + data.root_dims * data.root_size)
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
    ra = salf.render(a, o=to_dev(o), d=to_dev(d), outputs=outs)
    rb = salf.render(b, o=to_dev(o), d=to_dev(d), outputs=outs)
    for k in outs:
        assert torch.equal(ra[k], rb[k]), k
    ca, ia, _, _ = salf.trace_hits(a, to_dev(o), to_dev(d), 128)
    cb, ib, _, _ = salf.trace_hits(b, to_dev(o), to_dev(d), 128)
    ib = ib.cpu().numpy()
    mapped = np.where(ib >= 0, perm[np.maximum(ib, 0)], -1)
    assert torch.equal(ca, cb) and np.array_equal(ia.cpu().numpy(), mapped)


def test_scene_validation_errors(salf):
    data = synth.random_scene(59, max_level=2)
    bad = data.permuted(np.arange(data.n))
    bad.voxels = np.concatenate([bad.voxels, bad.voxels[3:4]], 0)          # duplicate
    bad.z_geo = np.concatenate([bad.z_geo, bad.z_geo[:1]], 0)
    bad.z_rgb = np.concatenate([bad.z_rgb, bad.z_rgb[:1]], 0)
    bad.z_int = np.concatenate([bad.z_int, bad.z_int[:1]], 0)
    with pytest.raises(salf.SalfError, match="overlaps or repeats"):
        salf.Scene.from_data(bad, device=dev())
    # a voxel containing another
    lo_i, _ = data.finest_bounds()
    v = int(np.nonzero(data.voxels[:, 0] == 2)[0][0])
    par = data.voxels[v].copy()
    par[0] = 1
    par[1:] //= 2
    bad.voxels = np.concatenate([data.voxels, par[None]], 0)
    with pytest.raises(salf.SalfError, match="overlaps or repeats"):
        salf.Scene.from_data(bad, device=dev())
    # out of range
    bad.voxels = np.concatenate([data.voxels, np.array([[0, 99, 0, 0]], np.int32)], 0)
    with pytest.raises(salf.SalfError, match=f"voxel {data.n} "):
        salf.Scene.from_data(bad, device=dev())


# ------------------------------------------------------------------ sensors
def _ray_errors(gpu, o64, d64, valid):
    go, gd = gpu["o"].cpu().numpy().astype(np.float64), gpu["d"].cpu().numpy().astype(np.float64)
    gv = gpu["valid"].cpu().numpy().astype(bool)
    assert np.array_equal(gv, valid)
    ang = np.arccos(np.clip(np.sum(gd[valid] * d64[valid], 1) / np.linalg.norm(gd[valid], axis=1), -1, 1))
    return float(np.max(np.abs(go - o64))), float(np.max(ang)) if ang.size else 0.0


@pytest.mark.parametrize("name", ["pinhole", "pinhole_rs", "fisheye_rs", "lidar"])
def test_sensor_rays_match_float64_models(salf, name):
    if name == "pinhole":
        s = synth.config1_camera()
    elif name == "pinhole_rs":
        s = synth.pinhole(1920, 1080, 70.0, synth.yaw_pitch_camera(60, -3), (10, -1.75, 1.6), dt_line=30e-6,
                          v=(10, 0, 0), w=(0, 0, 0.3))
    elif name == "fisheye_rs":
        s = synth.fisheye_equidistant(1280, 960, 190.0, synth.yaw_pitch_camera(90, 0), (10, -1.75, 1.6),
                                      dt_line=30e-6, v=(10, 0, 0), w=(0, 0, 0.3))
    else:
        s = synth.config2_lidar()
    gpu = salf.generate_rays(s, device=dev())
    o, d, t, valid = oracle.sensor_rays(s)
    eo, ed = _ray_errors(gpu, o, d, valid)
    assert eo <= 1e-5 and ed <= 1e-6, (eo, ed)
    assert np.max(np.abs(gpu["t"].cpu().numpy() - t)) <= 1e-6
    if name == "fisheye_rs":
        assert int(valid.sum()) == 1101128


def test_fused_sensor_render_equals_explicit_rays(salf):
    data = synth.random_scene(61, root_dims=(6, 5, 4), max_level=2)
    scene = salf.Scene.from_data(data, device=dev())
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
    for s in (synth.pinhole(37, 29, 80.0, synth.look_at((8, -7, 5), (0, 0, 0)), (8, -7, 5), dt_line=1e-3,
                            v=(1, 2, 0), w=(0, 0.5, 0.2)),
              synth.fisheye_equidistant(40, 30, 190.0, synth.look_at((0.1, 0.2, 0.3), (1, 0, 0)), (0.1, 0.2, 0.3)),
              synth.lidar_spinning(16, 100, -25, 15, np.eye(3), (0.5, -0.4, 0.3), 0.1, v=(10, 0, 0))):
        fused = salf.render(scene, sensor=s, outputs=outs)
        r = salf.generate_rays(s, device=dev())
        expl = salf.render(scene, o=r["o"], d=r["d"], outputs=outs, image_width=s["width"])
        valid = r["valid"].bool()
        for k in outs:
            a, b = fused[k], expl[k]
            assert torch.equal(a[valid], b[valid]), k
        assert torch.all(fused["opacity"][~valid] == 0)


def test_preactivated_scene_matches_oracle_and_refreshes(salf):
    data = synth.random_scene(63, root_dims=(6, 5, 4), max_level=2)
    ps = oracle.prepare(data)
    raw = salf.Scene.from_data(data, device=dev())
    pre = salf.Scene.from_data(data, device=dev(), preactivate=True)
    o, d = synth.random_rays(64, 600, data.origin, data.origin + data.root_dims * data.root_size)
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
    a = salf.render(raw, o=to_dev(o), d=to_dev(d), outputs=outs)
    b = salf.render(pre, o=to_dev(o), d=to_dev(d), outputs=outs)
    check_outputs(b, oracle.render_rays(ps, o, d, RenderOpts()))
    for k in outs:
        assert torch.allclose(a[k].float(), b[k].float(), atol=1e-6, rtol=0), k
    # in-place parameter update: stale until refresh, then equal to a fresh raw render
    with torch.no_grad():
        pre.geo.add_(0.5)
        pre.rgb.mul_(-1.0)
    stale = salf.render(pre, o=to_dev(o), d=to_dev(d), outputs=outs)
    assert torch.equal(stale["rgb"], b["rgb"])
    pre.refresh()
    fresh = salf.render(pre, o=to_dev(o), d=to_dev(d), outputs=outs)
    data2 = data.permuted(np.arange(data.n))
    data2.z_geo = data.z_geo + np.float32(0.5)
    data2.z_rgb = -data.z_rgb
    check_outputs(fresh, oracle.render_rays(oracle.prepare(data2), o, d, RenderOpts()))
    with pytest.raises(salf.SalfError, match="corner field only"):
        salf.Scene.from_data(data, device=dev(), field="paper", preactivate=True)


@pytest.mark.parametrize("field", ["corner", "paper", "sdf"])
def test_refine_matches_oracle(salf, field):
    """Densification and pruning (Sec. 3.3) on the GPU against the oracle: the same decisions and
    voxel list bit for bit, child parameters within 1e-5 (FP32 outputs of FP64 arithmetic)."""
    data = synth.random_scene(51, root_dims=(5, 4, 3), max_level=3)
    rng = np.random.default_rng(52)
    n = data.n
    if field != "corner":
        geo = np.zeros((n, 8), F32)
        geo[:, :4] = rng.normal(0, 0.7, (n, 4))
        if field == "sdf":
            geo[:, 4], geo[:, 5] = rng.normal(0.5, 0.3, n), rng.normal(-1, 0.3, n)
        rgb = np.zeros((n, 3, 8), F32)
        rgb[:, :, :7] = rng.normal(0, 0.7, (n, 3, 7))
        ity = np.zeros((n, 8), F32)
        ity[:, :4] = rng.normal(0, 0.7, (n, 4))
        data.z_geo, data.z_rgb, data.z_int = geo, rgb, ity
    grad = rng.exponential(1.0, (n, 3, 8)).astype(F32)
    l1 = np.array([oracle.colour_grad_l1(g, field) for g in grad])
    edge = data.root_size / (1 << data.voxels[:, 0].astype(np.int64))
    amax = np.array([1 - np.exp(-oracle.sigma_max(data.z_geo[v], field) * edge[v]) for v in range(n)])
    thr, a_min = float(np.quantile(l1, 0.6)), float(np.quantile(amax, 0.2))
    scene = salf.Scene.from_data(data, device=dev(), field=field)
    got = scene.refine(to_dev(grad), thr, a_min)
    ref, dec = oracle.refine(data, grad, thr, a_min, field)
    assert (dec == 0).sum() > 10 and (dec == 8).sum() > 10 and (dec == 1).sum() > 10
    assert np.array_equal(got["voxels"].cpu().numpy(), ref.voxels)
    for k, r in (("geo", ref.z_geo), ("rgb", ref.z_rgb), ("intensity", ref.z_int)):
        g = got[k].cpu().numpy().astype(np.float64)
        assert np.max(np.abs(g - r) / (1.0 + np.abs(r))) <= 1e-5, k
    # the refined set is a valid scene: it builds, and its parameters render
    data2 = synth.SceneData(**{**data.__dict__, "voxels": ref.voxels, "z_geo": got["geo"].cpu().numpy(),
                               "z_rgb": got["rgb"].cpu().numpy(), "z_int": got["intensity"].cpu().numpy()})
    scene2 = salf.Scene.from_data(data2, device=dev(), field=field)
    assert scene2.stats()["n_voxels"] == ref.n
    # no gradient: nothing splits; alpha_min 0: nothing is pruned
    same = scene.refine(None, 0.0, 0.0)
    assert torch.equal(same["voxels"], to_dev(data.voxels, torch.int32)) and torch.equal(same["geo"], to_dev(data.z_geo))


def _rotation(seed):
    q = np.random.default_rng(seed).normal(size=4)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]], np.float32)


def test_composite_render_matches_oracle(salf):
    """A static scene with three rotated, translated actors (disjoint from it and from one another):
    hits counted exactly, outputs within the render tolerance, explicit rays and a camera."""
    static = synth.random_scene(81, root_dims=(6, 4, 2), max_level=2, root_size=1.0, origin=(-3.0, -2.0, -1.0))
    lvl = static.voxels[:, 0].astype(np.int64)
    cx = static.voxels[:, 1].astype(np.int64) >> lvl
    static = static.subset(cx < 3)          # the background keeps the half x < 0
    actors, poses = [], []
    for a in range(3):
        data = synth.random_scene(90 + a, root_dims=(2, 2, 2), max_level=2, root_size=0.4, origin=(0.0, 0.0, 0.0))
        R = _rotation(95 + a)
        # the actor's 0.8 m cube lies within 0.7 m of its centre: centres 1.56 m or more apart and
        # 1.2 m or more beyond the background's x < 0 keep the cubes apart and off the background
        centre = np.array([(1.2, -1.2, 0.0), (2.2, 0.0, 0.0), (1.2, 1.2, 0.0)][a])
        t = (centre - R.astype(np.float64) @ np.array([0.4, 0.4, 0.4])).astype(np.float32)
        actors.append(data)
        poses.append((R, t))
    opts = RenderOpts(background=(0.1, 0.2, 0.3))
    sc = salf.Scene.from_data(static, device=dev(), preactivate=True)
    acts = [salf.Scene.from_data(a, device=dev(), preactivate=True) for a in actors]
    ps = oracle.prepare(static)
    aps = [(oracle.prepare(a), R, t) for a, (R, t) in zip(actors, poses)]
    lo, hi = np.array([-4.0, -3.0, -2.0]), np.array([4.0, 3.0, 2.0])
    o, d = synth.random_rays(97, 1500, lo, hi, inside_frac=0.0)
    outs = ("rgb", "depth", "opacity", "intensity", "n_hits")
    got = salf.render_composite(sc, [(s, R, t) for s, (R, t) in zip(acts, poses)], o=to_dev(o), d=to_dev(d),
                                background=opts.background, outputs=outs)
    ref = oracle.composite_rays(ps, aps, o, d, opts)
    assert int((ref["n_hits"] > 0).sum()) > 300
    check_outputs(got, ref, keys=outs)
    # a camera looking at the actors: fused ray generation, the oracle on the GPU's own rays
    cam = synth.pinhole(48, 32, 70.0, synth.look_at((4.5, -3.5, 2.5), (1.2, 0.0, 0.0)), (4.5, -3.5, 2.5))
    rays = salf.generate_rays(cam, device=dev())
    got = salf.render_composite(sc, [(s, R, t) for s, (R, t) in zip(acts, poses)], sensor=cam,
                                background=opts.background, outputs=outs)
    ro, rd = rays["o"].cpu().numpy(), rays["d"].cpu().numpy()
    check_outputs(got, oracle.composite_rays(ps, aps, ro, rd, opts), keys=outs)
    # an actor no ray meets leaves the plain render, bit for bit (the actor kernel's static walk)
    plain = salf.render(sc, o=to_dev(o), d=to_dev(d), background=opts.background, outputs=outs)
    far = salf.render_composite(sc, [(acts[0], np.eye(3, dtype=np.float32), np.array([500.0, 500.0, 500.0]))],
                                o=to_dev(o), d=to_dev(d), background=opts.background, outputs=outs)
    for k in outs:
        assert torch.equal(plain[k], far[k]), k


def test_composite_edge_cases_match_oracle(salf):
    """The maximum of seven actors, two of them with overlapping boxes (both sides then walk each
    box whole, in order of entry), rays that start inside an actor box or run along an axis, and a
    spinning LiDAR among the actors: hits exactly, outputs within the render tolerance; the fused
    sensor path equals explicit rays bit for bit."""
    static = synth.random_scene(111, root_dims=(4, 4, 2), max_level=2, root_size=1.0, origin=(-2.0, -2.0, -1.0))
    lvl = static.voxels[:, 0].astype(np.int64)
    cx = static.voxels[:, 1].astype(np.int64) >> lvl
    static = static.subset(cx < 2)          # the background keeps x < 0
    centres = [(2.0, -3.0, 0.0), (3.5, -1.5, 0.0), (3.5, 1.5, 0.0), (2.0, 3.0, 0.0), (-2.0, 3.5, 0.0),
               (-2.0, -3.5, 0.0), (-1.7, -3.3, 0.2)]      # the last two boxes overlap
    actors, poses = [], []
    for a, c in enumerate(centres):
        data = synth.random_scene(120 + a, root_dims=(2, 2, 2), max_level=2, root_size=0.4, origin=(0.0, 0.0, 0.0))
        R = _rotation(130 + a)
        t = (np.array(c) - R.astype(np.float64) @ np.array([0.4, 0.4, 0.4])).astype(np.float32)
        actors.append(data)
        poses.append((R, t))
    assert len(actors) == 7                 # the most one call takes
    opts = RenderOpts(background=(0.3, 0.1, 0.2))
    sc = salf.Scene.from_data(static, device=dev(), preactivate=True)
    acts = [salf.Scene.from_data(a, device=dev(), preactivate=True) for a in actors]
    items = [(s, R, t) for s, (R, t) in zip(acts, poses)]
    ps = oracle.prepare(static)
    aps = [(oracle.prepare(a), R, t) for a, (R, t) in zip(actors, poses)]
    rng = np.random.default_rng(141)
    # rays from inside each box, rays along the axes through the actor ring, random rays
    o_in = np.repeat(np.array(centres, np.float32), 40, axis=0) + rng.uniform(-0.2, 0.2, (280, 3)).astype(F32)
    d_in = rng.normal(size=(280, 3)).astype(F32)
    o_ax = np.zeros((6, 3), F32)
    d_ax = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], F32)
    o_ax[:, 2] = 0.05
    o_r, d_r = synth.random_rays(142, 600, np.array([-5.0, -5.0, -2.0]), np.array([5.0, 5.0, 2.0]), inside_frac=0.3)
    o = np.concatenate([o_in, o_ax, o_r.astype(F32)])
    d = np.concatenate([d_in, d_ax, d_r.astype(F32)])
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
    got = salf.render_composite(sc, items, o=to_dev(o), d=to_dev(d), background=opts.background, outputs=outs)
    ref = oracle.composite_rays(ps, aps, o, d, opts)
    assert int((ref["n_hits"][:280] > 0).sum()) > 150
    check_outputs(got, ref, keys=outs)
    # a spinning LiDAR at the middle of the ring (with ego motion), fused against explicit rays
    lid = synth.lidar_spinning(16, 128, -20, 10, np.eye(3), (0.8, 0.1, 0.1), 0.1, v=(5, 0, 0))
    fused = salf.render_composite(sc, items, sensor=lid, background=opts.background, outputs=outs)
    r = salf.generate_rays(lid, device=dev())
    expl = salf.render_composite(sc, items, o=r["o"], d=r["d"], background=opts.background, outputs=outs,
                                 image_width=lid["width"])
    valid = r["valid"].bool()
    for k in outs:
        assert torch.equal(fused[k][valid], expl[k][valid]), k
    ro, rd = r["o"].cpu().numpy(), r["d"].cpu().numpy()
    vi = np.nonzero(valid.cpu().numpy())[0]
    ref = oracle.composite_rays(ps, aps, ro[vi], rd[vi], opts)
    assert int((ref["n_hits"] > 0).sum()) > 200
    check_outputs(fused, ref, idx=vi, keys=outs)
