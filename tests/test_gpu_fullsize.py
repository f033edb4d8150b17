"""Parity at the workloads' full sizes: the 2M-voxel driving scene, a 1920x1080 camera frame and
a 64 x 2,048 rolling-shutter LiDAR sweep, rendered in the tiled launch the benchmark times, on the
raw-logit scene and on the pre-activated scene the benchmark renders.

Sampled rays are checked against the oracle one by one (bit-exact hits, outputs to tolerance):
4,096 drawn at random per frame, plus the 128 rays the GPU found the most voxels on (the horizon
grazers, the slowest rays and the most exposed to far-field FP32; choosing which rays to check is
the only use of a GPU value).  The oracle runs in a pool of CPU worker processes.  The whole frame
is checked through properties that hold at any size, and the fused-raygen render is checked to
equal the explicit-ray render of the GPU's own rays bit for bit, whose rays in turn match the
oracle's float64 sensor model.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

from oracle_pool import OraclePool
from test_gpu_render import check_outputs, dev, oracle_rays, to_dev, _ray_errors

pytestmark = pytest.mark.gpu
N_SAMPLE = 4096   # random rays per frame
N_HEAVY = 128     # rays with the most hits per frame


@pytest.fixture(scope="module")
def salf():
    import paper_2507_18713_amd as m
    return m


@pytest.fixture(scope="module")
def c1(salf):
    data = synth.config1_scene()
    print(f"driving scene: {data.n} voxels", flush=True)
    scene = salf.Scene.from_data(data, device=dev())
    return data, oracle.prepare(data), scene


@pytest.fixture(scope="module")
def c1_preactivated(salf, c1):
    data = c1[0]
    return salf.Scene.from_data(data, device=dev(), preactivate=True)


@pytest.fixture(scope="module")
def pool():
    p = OraclePool("driving")
    print(f"oracle pool: {p.n} workers", flush=True)
    yield p
    p.close()


def _pooled_parity(salf, scenes, pool, o, d, width, outs, seed, pieces=(1,)):
    """Sampled rays of a frame against the pooled oracle: hit lists bit for bit, outputs of every
    scene variant (raw logits, pre-activated) rendered with every lane count per ray to tolerance."""
    rng = np.random.default_rng(seed)
    combos = [(i, pc) for i in range(len(scenes)) for pc in pieces]
    full = [salf.render(scenes[i], o=to_dev(o), d=to_dev(d), image_width=width, outputs=outs, pieces=pc)
            for i, pc in combos]
    nh = full[0]["n_hits"].cpu().numpy()
    heavy = np.argsort(-nh, kind="stable")[:N_HEAVY]
    idx = np.unique(np.concatenate([rng.choice(o.shape[0], N_SAMPLE, replace=False), heavy]))
    print(f"pooled oracle on {idx.size} rays (heaviest: {int(nh[heavy[0]])} hits)", flush=True)
    hits, refs = pool.run(o[idx], d[idx])
    max_hits = int(max(h[0].size for h in hits)) + 1
    counts, ids, ti, to = salf.trace_hits(scenes[0], to_dev(o[idx]), to_dev(d[idx]), max_hits)
    counts, ids, ti, to = (x.cpu().numpy() for x in (counts, ids, ti, to))
    for q, (e_ids, e_ti, e_to) in enumerate(hits):
        k = e_ids.size
        assert counts[q] == k, (idx[q], counts[q], k)
        assert np.array_equal(ids[q, :k], e_ids), idx[q]
        assert np.array_equal(ti[q, :k].view(np.uint32), e_ti.view(np.uint32)), idx[q]
        assert np.array_equal(to[q, :k].view(np.uint32), e_to.view(np.uint32)), idx[q]
    ref = {k: np.array([r[k] for r in refs]) for k in refs[0]}
    for got in full:
        check_outputs(got, ref, idx=idx, keys=[k for k in outs if k != "n_hits"])
    # the pre-activated scene composites the same voxels; n_hits may differ only where FP32
    # rounding of the activation moves T across t_min, which the oracle's n_hits pins for the raw one
    for (i, pc), got in zip(combos, full):
        if i == 0:
            assert np.array_equal(got["n_hits"].cpu().numpy()[idx], ref["n_hits"]), pc
    # in pieces, every ray of the frame against the one-lane render: the same hit counts, outputs
    # equal to FP32 rounding
    for (i, pc), got in zip(combos, full):
        one = full[combos.index((i, 1))] if (i, 1) in combos else None
        if pc == 1 or one is None:
            continue
        assert torch.equal(got["n_hits"], one["n_hits"]), (i, pc)
        for k in outs:
            if k != "n_hits":
                err = float(torch.max(torch.abs(got[k] - one[k])))
                assert err <= (1e-3 if k == "depth" else 2e-5), (i, pc, k, err)
    return full[0], int(ref["n_hits"].sum())


def test_build_statistics(c1):
    data, ps, scene = c1
    st = scene.stats()
    assert st["n_voxels"] == data.n
    assert 1_980_000 <= data.n <= 2_020_000
    assert st["n_nodes"] > data.n // 10
    assert st["n_occupied_roots"] > 15_000


def _frame_invariants(res, bg_max=0.0):
    T = res["t_end"]
    assert torch.all(torch.isfinite(T)) and torch.all((T >= 0) & (T <= 1))
    assert torch.equal(res["opacity"], 1.0 - T)
    assert torch.all(res["depth"] >= 0)
    if "rgb" in res:
        assert torch.all((res["rgb"] >= 0) & (res["rgb"] <= 1.0 + 1e-6))
    if "intensity" in res:
        assert torch.all((res["intensity"] >= 0) & (res["intensity"] <= res["opacity"] + 1e-6))


def test_camera_frame(salf, c1, c1_preactivated, pool):
    data, ps, scene = c1
    cam = synth.config1_camera()
    o, d, _ = oracle_rays(cam)
    outs = ("rgb", "depth", "opacity", "t_end", "n_hits")
    got, n_hits = _pooled_parity(salf, (scene, c1_preactivated), pool, o, d, 1920, outs, seed=71)
    assert n_hits > N_SAMPLE * 3
    _frame_invariants(got)
    # fused ray generation: rays close to the float64 model, render equal to the explicit one
    fused = salf.render(scene, sensor=cam, outputs=outs)
    r = salf.generate_rays(cam, device=dev())
    eo, ed = _ray_errors(r, *oracle.sensor_rays(cam)[:2], np.ones(o.shape[0], bool))
    assert eo <= 1e-5 and ed <= 1e-6
    expl = salf.render(scene, o=r["o"], d=r["d"], image_width=1920, outputs=outs)
    for k in outs:
        assert torch.equal(fused[k], expl[k]), k
    _frame_invariants(fused)
    # the two ray sets differ by float32 rounding only: the frames agree closely on average
    assert float(torch.mean(torch.abs(fused["rgb"] - got["rgb"]))) < 1e-5


def test_lidar_sweep(salf, c1, c1_preactivated, pool):
    data, ps, scene = c1
    lid = synth.config2_lidar()
    o, d, _ = oracle_rays(lid)
    outs = ("depth", "intensity", "opacity", "t_end", "n_hits")
    got, n_hits = _pooled_parity(salf, (scene, c1_preactivated), pool, o, d, 2048, outs, seed=72, pieces=(1, 4, 8))
    assert n_hits > N_SAMPLE
    _frame_invariants(got)
    fused = salf.render(scene, sensor=lid, outputs=outs)
    r = salf.generate_rays(lid, device=dev())
    expl = salf.render(scene, o=r["o"], d=r["d"], image_width=2048, outputs=outs)
    for k in outs:
        assert torch.equal(fused[k], expl[k]), k
    _frame_invariants(fused)
    assert float(torch.mean((fused["opacity"] > 0.5).float())) > 0.2   # the ground returns


def test_forward_is_deterministic(salf, c1):
    data, ps, scene = c1
    cam = synth.config1_camera(480, 270)
    a = salf.render(scene, sensor=cam, outputs=("rgb", "depth", "opacity", "n_hits"))
    b = salf.render(scene, sensor=cam, outputs=("rgb", "depth", "opacity", "n_hits"))
    for k in a:
        assert torch.equal(a[k], b[k])


def test_tile_schedule_changes_nothing_but_the_order(salf, c1):
    """Heaviest-tiles-first scheduling (the default) renders every ray to the same bits as the
    launch in tile order: the camera frame, a LiDAR sweep large enough to be scheduled (128 x 4,096
    rays; launches that fit on the GPU at once keep their order) and explicit rays."""
    data, ps, scene = c1
    big_lidar = synth.lidar_spinning(128, 4096, -25.0, 15.0, np.eye(3), (-60.0, 0.37, 1.85), 0.1, v=(10, 0, 0))
    for sensor, outs in ((synth.config1_camera(), ("rgb", "depth", "opacity", "t_end", "n_hits")),
                         (big_lidar, ("depth", "opacity", "t_end", "n_hits"))):
        a = salf.render(scene, sensor=sensor, outputs=outs, schedule=True)
        b = salf.render(scene, sensor=sensor, outputs=outs, schedule=False)
        for k in outs:
            assert torch.equal(a[k], b[k]), (sensor["model"], k)
    rays = salf.generate_rays(synth.config1_camera(), dev())
    a = salf.render(scene, o=rays["o"], d=rays["d"], outputs=("rgb", "n_hits"), schedule=True)
    b = salf.render(scene, o=rays["o"], d=rays["d"], outputs=("rgb", "n_hits"), schedule=False)
    assert torch.equal(a["rgb"], b["rgb"]) and torch.equal(a["n_hits"], b["n_hits"])
    # a schedule built once and reused; one built for another ray layout is ignored
    cam = synth.config1_camera()
    buf = salf.render_schedule(scene, sensor=cam)
    ref = salf.render(scene, sensor=cam, outputs=("rgb", "n_hits"), schedule=False)
    for _ in range(2):
        r = salf.render(scene, sensor=cam, outputs=("rgb", "n_hits"), schedule=buf)
        assert torch.equal(r["rgb"], ref["rgb"]) and torch.equal(r["n_hits"], ref["n_hits"])
    small = synth.config1_camera(960, 540)
    r = salf.render(scene, sensor=small, outputs=("rgb",), schedule=buf)
    assert torch.equal(r["rgb"], salf.render(scene, sensor=small, outputs=("rgb",), schedule=False)["rgb"])
