"""GPU backward pass: against the oracle's analytic gradient on small scenes (corner field and the
paper's field of Eq. 1-2), and against central finite differences of the GPU forward on the
driving scene (corner field) and on a small paper-field scene.

Bars: GPU vs oracle |g - g_o| <= 1e-3 |g_o| + 1e-5 max|g_o|; GPU vs FD (eps = 1e-3, loss summed in
float64, t_min = 0) |g - g_fd| <= 2e-2 |g_fd| + 1e-3 max|g_fd|.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.render import RenderOpts

from test_gpu_render import dev, oracle_rays, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def salf():
    import paper_2507_18713_amd as m
    return m


def _close(g, ref, rel=1e-3, absr=1e-5):
    scale = np.max(np.abs(ref))
    assert scale > 0
    err = np.abs(g - ref) - (rel * np.abs(ref) + absr * scale)
    worst = np.argsort(-err.ravel())[:5]
    detail = [(int(i), float(g.ravel()[i]), float(ref.ravel()[i])) for i in worst]
    assert np.max(err) <= 0, detail


@pytest.mark.parametrize("which", ["tiny", "adaptive"])
def test_gradient_matches_oracle(salf, which):
    if which == "tiny":
        data = synth.config0_scene()
        o, d, _ = oracle_rays(synth.config0_camera())
        width = 64
    else:
        data = synth.random_scene(81, root_dims=(5, 4, 3), max_level=2)
        o, d = synth.random_rays(82, 600, data.origin, data.origin + data.root_dims * data.root_size)
        width = 0
    n = o.shape[0]
    rng = np.random.default_rng(83)
    g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
    g_d, g_o, g_i = (rng.normal(size=n).astype(np.float32) for _ in range(3))
    bg = (0.1, 0.2, 0.3)
    scene = salf.Scene.from_data(data, device=dev())
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
    saved = salf.render(scene, o=to_dev(o), d=to_dev(d), background=bg, outputs=outs, image_width=width)
    grads = {"rgb": to_dev(g_rgb), "depth": to_dev(g_d), "opacity": to_dev(g_o), "intensity": to_dev(g_i)}
    dg, dr, di = salf.render_backward(scene, saved, grads, o=to_dev(o), d=to_dev(d), background=bg,
                                      image_width=width)
    ps = oracle.prepare(data)
    eg, er, ei = oracle.grad_rays(ps, o, d, RenderOpts(background=bg), g_rgb, g_d, g_o, g_i)
    _close(dg.cpu().numpy(), eg)
    _close(dr.cpu().numpy(), er)
    _close(di.cpu().numpy(), ei)


def _paper_scene(seed):
    """A seeded scene with Eq. 1-2 parameters: density slopes N(0, 0.5^2) and offset N(0, 1); colour
    slopes and SH coefficients N(0, 0.5^2), offsets N(0, 1); intensity likewise (as the paper-field
    forward test)."""
    data = synth.random_scene(seed, root_dims=(5, 4, 3), max_level=2)
    rng = np.random.default_rng(seed + 1)
    n = data.n
    geo = np.zeros((n, 8), np.float32)
    geo[:, :3] = rng.normal(0, 0.5, (n, 3))
    geo[:, 3] = rng.normal(0, 1, n)
    rgb = np.zeros((n, 3, 8), np.float32)
    rgb[:, :, :3] = rng.normal(0, 0.5, (n, 3, 3))
    rgb[:, :, 3] = rng.normal(0, 1, (n, 3))
    rgb[:, :, 4:7] = rng.normal(0, 0.5, (n, 3, 3))
    ity = np.zeros((n, 8), np.float32)
    ity[:, :3] = rng.normal(0, 0.5, (n, 3))
    ity[:, 3] = rng.normal(0, 1, n)
    data.z_geo, data.z_rgb, data.z_int = geo, rgb, ity
    return data


def _sdf_scene(seed):
    """A seeded scene for the SDF variant (Eq. 5-6): signed-distance slopes N(0, 0.6^2) and offset
    N(0, 0.5^2), log a ~ N(0.5, 0.3^2), log b ~ N(-1, 0.3^2); colour and intensity as _paper_scene."""
    data = _paper_scene(seed)
    rng = np.random.default_rng(seed + 2)
    n = data.n
    geo = np.zeros((n, 8), np.float32)
    geo[:, :3] = rng.normal(0, 0.6, (n, 3))
    geo[:, 3] = rng.normal(0, 0.5, n)
    geo[:, 4] = rng.normal(0.5, 0.3, n)
    geo[:, 5] = rng.normal(-1.0, 0.3, n)
    data.z_geo = geo
    return data


@pytest.mark.parametrize("field,samples", [("paper", 1), ("paper", 4), ("sdf", 1), ("sdf", 4)])
def test_paper_field_gradient_matches_oracle(salf, field, samples):
    data = _paper_scene(85) if field == "paper" else _sdf_scene(85)
    o, d = synth.random_rays(87, 600, data.origin, data.origin + data.root_dims * data.root_size)
    n = o.shape[0]
    rng = np.random.default_rng(88)
    g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
    g_d, g_o, g_i = (rng.normal(size=n).astype(np.float32) for _ in range(3))
    bg = (0.1, 0.2, 0.3)
    scene = salf.Scene.from_data(data, device=dev(), field=field)
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
    saved = salf.render(scene, o=to_dev(o), d=to_dev(d), background=bg, samples=samples, outputs=outs)
    grads = {"rgb": to_dev(g_rgb), "depth": to_dev(g_d), "opacity": to_dev(g_o), "intensity": to_dev(g_i)}
    dg, dr, di = salf.render_backward(scene, saved, grads, o=to_dev(o), d=to_dev(d), background=bg,
                                      samples=samples)
    eg, er, ei = oracle.grad_rays(oracle.prepare(data), o, d, RenderOpts(background=bg, samples=samples,
                                                                          field=field),
                                  g_rgb, g_d, g_o, g_i)
    dg, dr, di = dg.cpu().numpy(), dr.cpu().numpy(), di.cpu().numpy()
    # the unused record slots receive nothing
    used = 6 if field == "sdf" else 4
    assert not dg[:, used:].any() and not dr[:, :, 7].any() and not di[:, 4:].any()
    _close(dg, eg)
    _close(dr, er)
    _close(di, ei)


@pytest.mark.parametrize("field", ["paper", "sdf"])
def test_paper_field_gradient_matches_finite_differences(salf, field):
    """Central differences (eps = 1e-3) of the GPU forward, summed in float64, on a paper-field
    (or SDF-variant) scene: the parameters are drawn from voxels that at least 8 of the rays hit."""
    data = _paper_scene(89) if field == "paper" else _sdf_scene(89)
    lo, hi = data.origin, data.origin + data.root_dims * data.root_size
    o, d = synth.random_rays(90, 4000, lo, hi)
    scene = salf.Scene.from_data(data, device=dev(), field=field)
    opts = dict(samples=4, t_min=0.0)
    O, D = to_dev(o), to_dev(d)
    n = o.shape[0]
    rng = np.random.default_rng(92)
    g_rgb = torch.from_numpy(rng.normal(size=(n, 3)).astype(np.float32)).to(dev())
    g_d = torch.from_numpy(rng.normal(size=n).astype(np.float32)).to(dev())

    def loss():
        r = salf.render(scene, o=O, d=D, outputs=("rgb", "depth"), **opts)
        return float((g_rgb.double() * r["rgb"].double()).sum() + (g_d.double() * r["depth"].double()).sum())

    saved = salf.render(scene, o=O, d=D, outputs=("rgb", "depth", "opacity", "t_end", "n_hits"), **opts)
    dg, dr, _ = salf.render_backward(scene, saved, {"rgb": g_rgb, "depth": g_d}, o=O, d=D, **opts)
    cnt, ids, _, _ = salf.trace_hits(scene, O, D, 256)
    ids = ids.cpu().numpy()
    hits = np.bincount(ids[ids >= 0], minlength=data.n)
    cand = np.nonzero(hits >= 8)[0]
    assert cand.size >= 10
    eps = 1e-3
    checks = []
    for arr, grad, width in ((scene.geo, dg, 6 if field == "sdf" else 4), (scene.rgb, dr, 7)):
        for _ in range(12):
            v = int(rng.choice(cand))
            idx = (v,) + ((int(rng.integers(0, 3)),) if arr.dim() == 3 else ()) + (int(rng.integers(0, width)),)
            old = float(arr[idx])
            arr[idx] = old + eps
            lp = loss()
            arr[idx] = old - eps
            lm = loss()
            arr[idx] = old
            checks.append(((lp - lm) / (2 * eps), float(grad[idx])))
    fd = np.array([c[0] for c in checks])
    g = np.array([c[1] for c in checks])
    scale = np.max(np.abs(fd))
    assert scale > 0
    assert np.all(np.abs(g - fd) <= 2e-2 * np.abs(fd) + 1e-3 * scale), list(zip(fd, g))


def test_gradient_matches_finite_differences_on_driving_scene(salf):
    """Central differences of the float32 forward carry noise of a few 1e-5 per ray that a
    perturbed parameter reaches (output rounding over 2 eps = 2e-3), so the 64 parameters are
    drawn from voxels that at least 16 camera rays (or 8 LiDAR rays) cross: their gradients
    then stand well above that floor.  Camera rays (80%) carry an L2 colour loss, LiDAR rays
    (20%) an L1 depth loss, as in the training batch."""
    data = synth.config1_scene()
    scene = salf.Scene.from_data(data, device=dev())
    # dense views: a narrow camera on the road ahead, and a LiDAR sweep over a 40 deg sector
    cam = synth.pinhole(192, 108, 30.0, synth.yaw_pitch_camera(0.0, -12.0), (-95.0, 0.0, 1.6))
    oc, dc, _ = oracle_rays(cam)
    # LiDAR-like rays: 64 beams in [-25, +15] deg x 48 azimuths over a 40 deg sector, one origin
    b, j = np.divmod(np.arange(64 * 48), 48)
    e = np.radians(-25.0 + 40.0 * b / 63)
    a = np.radians(-20.0 + 40.0 * (j + 0.5) / 48)
    dl = np.stack([np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)], 1).astype(np.float32)
    ol = np.tile(np.array([[-90.0, 0.37, 1.85]], np.float32), (dl.shape[0], 1))
    rng = np.random.default_rng(91)
    opts = dict(samples=4, t_min=0.0)
    Oc, Dc, Ol, Dl = to_dev(oc), to_dev(dc), to_dev(ol), to_dev(dl)
    # fixed targets; depth targets sit 2-5 m away from the current depth so that the L1 loss has
    # no kink within +-eps of any parameter
    tc = rng.uniform(0, 1, size=(oc.shape[0], 3))
    d_now = salf.render(scene, o=Ol, d=Dl, outputs=("depth",), **opts)["depth"].double().cpu().numpy()
    td = d_now + rng.choice([-1.0, 1.0], size=ol.shape[0]) * rng.uniform(2.0, 5.0, size=ol.shape[0])

    def loss():
        a_ = salf.render(scene, o=Oc, d=Dc, outputs=("rgb",), **opts)["rgb"].double().cpu().numpy()
        b_ = salf.render(scene, o=Ol, d=Dl, outputs=("depth",), **opts)["depth"].double().cpu().numpy()
        return float(np.sum((a_ - tc) ** 2) + np.sum(np.abs(b_ - td)))

    ca = salf.render(scene, o=Oc, d=Dc, outputs=("rgb", "depth", "opacity", "t_end", "n_hits"), **opts)
    la = salf.render(scene, o=Ol, d=Dl, outputs=("rgb", "depth", "opacity", "t_end", "n_hits"), **opts)
    g_c = (2.0 * (ca["rgb"].double().cpu().numpy() - tc)).astype(np.float32)
    g_l = np.sign(la["depth"].double().cpu().numpy() - td).astype(np.float32)
    dg, dr, _ = salf.render_backward(scene, ca, {"rgb": to_dev(g_c)}, o=Oc, d=Dc, **opts)
    dg2, _, _ = salf.render_backward(scene, la, {"depth": to_dev(g_l)}, o=Ol, d=Dl, **opts)
    dg = (dg + dg2).cpu().numpy()
    dr = dr.cpu().numpy()
    # voxels by the number of rays that cross them
    cnt_c, ids_c, _, _ = salf.trace_hits(scene, Oc, Dc, 512)
    cnt_l, ids_l, tin_l, _ = salf.trace_hits(scene, Ol, Dl, 512)
    hc = np.bincount(np.maximum(ids_c.cpu().numpy().ravel(), 0), minlength=data.n)
    # LiDAR voxels within 8 m: the float32 depth rounding (about 5e-7 m there) stays far below the
    # central difference of the loss
    il = ids_l.cpu().numpy().ravel()
    near = (il >= 0) & (tin_l.cpu().numpy().ravel() < 8.0)
    hl = np.bincount(il[near], minlength=data.n)
    hc[0] = hl[0] = 0
    dense_c = np.nonzero(hc >= 16)[0]
    dense_l = np.nonzero((hl >= 8) & (hc == 0))[0]
    assert dense_c.size >= 48 and dense_l.size >= 32, (dense_c.size, dense_l.size)
    # a depth moves by |g| eps / (rays) per ray; at 4-8 m one float32 ulp is 4.8e-7 m, so depth
    # differences resolve only parameters with a large per-ray effect: take the 16 LiDAR density
    # logits with the largest gradient among the densely hit near voxels
    gl = np.abs(dg[dense_l]).max(axis=1)
    lid_picks = dense_l[np.argsort(-gl)[:16]]
    eps = 1e-3
    fd, an = [], []
    picks = list(rng.choice(dense_c, 48, replace=False)) + list(lid_picks)
    for q, v in enumerate(picks):
        c = int(rng.integers(0, 8)) if q < 48 else int(np.argmax(np.abs(dg[v])))
        if q % 2 == 0 or q >= 48:       # LiDAR-only voxels: density logits (colour has no LiDAR loss)
            t, idx, g = scene.geo, (v, c), dg[v, c]
        else:
            ch = int(rng.integers(0, 3))
            t, idx, g = scene.rgb, (v, ch, c), dr[v, ch, c]
        with torch.no_grad():
            old = t[idx].item()
            t[idx] = old + eps
            lp = loss()
            t[idx] = old - eps
            lm = loss()
            t[idx] = old
        fd.append((lp - lm) / (2 * eps))
        an.append(g)
    fd, an = np.array(fd), np.array(an)
    _close(an, fd, rel=2e-2, absr=1e-3)


def test_gradient_matches_oracle_on_driving_scene(salf):
    """Sampled rays of the training-batch views on the 2M-voxel scene: GPU gradient vs the
    oracle's analytic gradient (brute force over every voxel), camera colour + depth and LiDAR
    depth + intensity losses, with and without early termination."""
    data = synth.config1_scene()
    scene = salf.Scene.from_data(data, device=dev())
    ps = oracle.prepare(data)
    rng = np.random.default_rng(97)
    cam = synth.pinhole(192, 108, 30.0, synth.yaw_pitch_camera(0.0, -12.0), (-95.0, 0.0, 1.6))
    oc, dc, _ = oracle_rays(cam)
    lid = synth.config2_lidar()
    ol, dl, _ = oracle_rays(lid)
    ic = rng.choice(oc.shape[0], 96, replace=False)
    il = rng.choice(ol.shape[0], 96, replace=False)
    o = np.concatenate([oc[ic], ol[il]])
    d = np.concatenate([dc[ic], dl[il]])
    n = o.shape[0]
    g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
    g_d, g_i = (rng.normal(size=n).astype(np.float32) for _ in range(2))
    g_rgb[96:] = 0.0
    g_i[:96] = 0.0
    for tmin in (1e-6, 0.0):
        opts = dict(samples=4, t_min=tmin)
        saved = salf.render(scene, o=to_dev(o), d=to_dev(d),
                            outputs=("rgb", "depth", "opacity", "intensity", "t_end", "n_hits"), **opts)
        grads = {"rgb": to_dev(g_rgb), "depth": to_dev(g_d), "intensity": to_dev(g_i)}
        dg, dr, di = salf.render_backward(scene, saved, grads, o=to_dev(o), d=to_dev(d), **opts)
        eg, er, ei = oracle.grad_rays(ps, o, d, RenderOpts(samples=4, t_min=tmin), g_rgb, g_d, np.zeros(n), g_i)
        touched = np.any(eg != 0, axis=1)
        assert touched.sum() > 500
        _close(dg.cpu().numpy()[touched], eg[touched])
        _close(dr.cpu().numpy()[touched], er[touched])
        _close(di.cpu().numpy()[touched], ei[touched])


def test_autograd_function(salf):
    data = synth.random_scene(95, root_dims=(4, 4, 3), max_level=1)
    scene = salf.Scene.from_data(data, device=dev(), requires_grad=True)
    o, d = synth.random_rays(96, 300, data.origin, data.origin + data.root_dims * data.root_size)
    opts = dict(samples=4, t_min=1e-6)
    rgb, depth, op, inten = salf.RenderFunction.apply(scene.geo, scene.rgb, scene.intensity, scene, None,
                                                      to_dev(o), to_dev(d), opts)
    loss = (rgb ** 2).sum() + depth.abs().sum() + inten.sum()
    loss.backward()
    assert scene.geo.grad is not None and torch.any(scene.geo.grad != 0)
    assert scene.rgb.grad is not None and scene.intensity.grad is not None
    # the same through the explicit backward call
    saved = salf.render(scene, o=to_dev(o), d=to_dev(d), outputs=("rgb", "depth", "opacity", "intensity", "t_end",
                                                                      "n_hits"), **opts)
    grads = {"rgb": 2 * saved["rgb"], "depth": torch.sign(saved["depth"]), "intensity": torch.ones_like(depth)}
    dg, dr, di = salf.render_backward(scene, saved, grads, o=to_dev(o), d=to_dev(d), **opts)
    assert torch.allclose(dg, scene.geo.grad, rtol=1e-4, atol=1e-6)
    assert torch.allclose(dr, scene.rgb.grad, rtol=1e-4, atol=1e-6)
    assert torch.allclose(di, scene.intensity.grad, rtol=1e-4, atol=1e-6)
    # with stored hits (2 per ray: most rays are walked for the rest) the same gradient
    g_walk = [t.grad.clone() for t in (scene.geo, scene.rgb, scene.intensity)]
    for t in (scene.geo, scene.rgb, scene.intensity):
        t.grad = None
    for cap in (2, 64):
        rgb, depth, op, inten = salf.RenderFunction.apply(scene.geo, scene.rgb, scene.intensity, scene, None,
                                                          to_dev(o), to_dev(d), dict(opts, hit_capacity=cap))
        ((rgb ** 2).sum() + depth.abs().sum() + inten.sum()).backward()
        for t, ref in zip((scene.geo, scene.rgb, scene.intensity), g_walk):
            assert torch.allclose(t.grad, ref, rtol=1e-4, atol=1e-6), cap
            t.grad = None
    # the backward reads the returned outputs: changing one in place before backward is an error,
    # not a silently wrong gradient
    rgb, depth, op, inten = salf.RenderFunction.apply(scene.geo, scene.rgb, scene.intensity, scene, None,
                                                      to_dev(o), to_dev(d), opts)
    rgb.clamp_(0.0, 0.5)
    with pytest.raises(RuntimeError, match="inplace"):
        (rgb.sum() + depth.sum()).backward()


def test_preactivated_scene_gives_the_same_gradient(salf):
    """A scene that keeps activated corner values renders and differentiates from them (softplus'
    taken as 1 - exp(-softplus)); gradients w.r.t. the raw logits match the raw-logit scene's, also
    after the logits change and the scene is refreshed."""
    data = synth.random_scene(97, root_dims=(5, 4, 3), max_level=2)
    raw = salf.Scene.from_data(data, device=dev())
    act = salf.Scene.from_data(data, device=dev(), preactivate=True)
    o, d = synth.random_rays(98, 512, data.origin, data.origin + data.root_dims * data.root_size)
    o, d = to_dev(o), to_dev(d)
    opts = dict(samples=4, t_min=1e-6)
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
    for step in range(2):
        if step == 1:  # change the logits of both scenes in place, refresh the stored activations
            for sc in (raw, act):
                sc.geo.mul_(1.1).add_(0.05)
                sc.rgb.mul_(0.9)
                sc.intensity.add_(0.1)
            act.refresh()
        sr = salf.render(raw, o=o, d=d, outputs=outs, **opts)
        sa = salf.render(act, o=o, d=d, outputs=outs, **opts)
        for k in ("rgb", "depth", "opacity", "intensity"):
            assert torch.allclose(sr[k], sa[k], rtol=1e-5, atol=1e-6), k
        grads = {"rgb": torch.cos(3 * sr["rgb"]), "depth": 0.1 * torch.sign(sr["depth"] - 1.0),
                 "opacity": torch.ones_like(sr["opacity"]), "intensity": 0.5 * torch.ones_like(sr["intensity"])}
        gr = salf.render_backward(raw, sr, dict(grads), o=o, d=d, **opts)
        ga = salf.render_backward(act, sa, dict(grads), o=o, d=d, **opts)
        for name, x, y in zip(("geo", "rgb", "intensity"), gr, ga):
            assert torch.any(x != 0), name
            _close(y.cpu().numpy(), x.cpu().numpy(), rel=1e-3, absr=1e-5)


@pytest.mark.parametrize("field,cap", [("corner", 64), ("corner", 2), ("corner-act", 64), ("paper", 64), ("sdf", 3)])
def test_stored_hits_give_the_oracle_gradient(salf, field, cap):
    """The forward stores each ray's composited hits (hit_capacity entries at most): they equal the
    traced hit list with the render's early termination bit for bit, the other outputs keep their
    bits, and the backward that reads them (walking only rays with more hits than were stored)
    gives the oracle's gradient.  cap 2 and 3 leave many rays to the walk."""
    if field in ("corner", "corner-act"):
        data = synth.random_scene(91, root_dims=(5, 4, 3), max_level=2)
    else:
        data = _paper_scene(92) if field == "paper" else _sdf_scene(92)
    o, d = synth.random_rays(93, 700, data.origin, data.origin + data.root_dims * data.root_size)
    n = o.shape[0]
    rng = np.random.default_rng(94)
    g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
    g_d, g_o, g_i = (rng.normal(size=n).astype(np.float32) for _ in range(3))
    bg = (0.1, 0.2, 0.3)
    kw = dict(field=field) if field in ("paper", "sdf") else dict(preactivate=field == "corner-act")
    scene = salf.Scene.from_data(data, device=dev(), **kw)
    outs = ("rgb", "depth", "opacity", "intensity", "t_end", "n_hits")
    plain = salf.render(scene, o=to_dev(o), d=to_dev(d), background=bg, outputs=outs)
    saved = salf.render(scene, o=to_dev(o), d=to_dev(d), background=bg, outputs=outs, hit_capacity=cap)
    for k in outs:
        assert torch.equal(saved[k], plain[k]), k
    nh = saved["n_hits"].cpu().numpy()
    if cap < 8:
        assert nh.max() > cap  # some rays are walked
    counts, ids, ti, to = salf.trace_hits(scene, to_dev(o), to_dev(d), int(nh.max()) + 1, early_termination=True)
    assert torch.equal(counts, saved["n_hits"])
    hv = saved["hit_voxel"].cpu().numpy()
    ht = saved["hit_t"].cpu().numpy()
    ids, ti, to = ids.cpu().numpy(), ti.cpu().numpy(), to.cpu().numpy()
    for r in range(n):
        k = min(int(nh[r]), cap)
        assert np.array_equal(hv[:k, r], ids[r, :k]), r
        assert np.array_equal(ht[:k, r, 0].view(np.uint32), ti[r, :k].view(np.uint32)), r
        assert np.array_equal(ht[:k, r, 1].view(np.uint32), to[r, :k].view(np.uint32)), r
    grads = {"rgb": to_dev(g_rgb), "depth": to_dev(g_d), "opacity": to_dev(g_o), "intensity": to_dev(g_i)}
    dg, dr, di = salf.render_backward(scene, saved, dict(grads), o=to_dev(o), d=to_dev(d), background=bg)
    wg, wr, wi = salf.render_backward(scene, plain, dict(grads), o=to_dev(o), d=to_dev(d), background=bg)
    eg, er, ei = oracle.grad_rays(oracle.prepare(data), o, d,
                                  RenderOpts(background=bg, field="corner" if field == "corner-act" else field),
                                  g_rgb, g_d, g_o, g_i)
    for got, walked, ref in ((dg, wg, eg), (dr, wr, er), (di, wi, ei)):
        got, walked = got.cpu().numpy(), walked.cpu().numpy()
        if field == "corner-act":  # the activated copies round once more: the bar of the pre-activated test
            _close(got, walked, rel=1e-4, absr=1e-6)
        else:
            _close(got, ref)
        _close(got, walked, rel=1e-4, absr=1e-6)


def test_backwards_on_two_streams_add_into_one_gradient(salf):
    """Two batches' backwards launched on two streams at once (one reading stored hits, one
    walking) add into the same gradient buffers with their atomics, as the training step's camera
    and LiDAR batches do: the sum is the oracle's gradient of both batches together."""
    data = synth.random_scene(95, root_dims=(5, 4, 3), max_level=2)
    o, d = synth.random_rays(96, 1400, data.origin, data.origin + data.root_dims * data.root_size)
    n, na = o.shape[0], 900
    rng = np.random.default_rng(97)
    g_rgb = rng.normal(size=(n, 3)).astype(np.float32)
    g_d = rng.normal(size=n).astype(np.float32)
    scene = salf.Scene.from_data(data, device=dev())
    outs = ("rgb", "depth", "opacity", "t_end", "n_hits")
    oa, da, ob, db = to_dev(o[:na]), to_dev(d[:na]), to_dev(o[na:]), to_dev(d[na:])
    sa = salf.render(scene, o=oa, d=da, outputs=outs, hit_capacity=64)
    sb = salf.render(scene, o=ob, d=db, outputs=outs)
    ga = {"rgb": to_dev(g_rgb[:na]), "depth": to_dev(g_d[:na])}
    gb = {"rgb": to_dev(g_rgb[na:]), "depth": to_dev(g_d[na:])}
    d_geo, d_rgb = torch.zeros_like(scene.geo), torch.zeros_like(scene.rgb)
    main = torch.cuda.current_stream(dev())
    side = torch.cuda.Stream(device=dev())  # default priority
    side.wait_stream(main)
    with torch.cuda.stream(side):
        salf.render_backward(scene, sb, dict(gb), o=ob, d=db, d_geo=d_geo, d_rgb=d_rgb)
    salf.render_backward(scene, sa, dict(ga), o=oa, d=da, d_geo=d_geo, d_rgb=d_rgb)
    main.wait_stream(side)
    torch.cuda.synchronize()
    zero = np.zeros(n, np.float32)
    eg, er, _ = oracle.grad_rays(oracle.prepare(data), o, d, RenderOpts(), g_rgb, g_d, zero, zero)
    _close(d_geo.cpu().numpy(), eg)
    _close(d_rgb.cpu().numpy(), er)
