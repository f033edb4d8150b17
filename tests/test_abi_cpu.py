"""The C ABI library without a GPU: it loads, exports every declared entry point, its structs
have the layout the Python binding assumes, and its host-only calls validate arguments."""
import ctypes as C
import math
import os
import re
import subprocess
import sys
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "salf.h")


@pytest.fixture(scope="module")
def L():
    from paper_2507_18713_amd import _lib
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(salf_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function(L):
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, f"{name} has no Python signature"
    assert lib.salf_abi_version() == 1


def test_struct_layout_matches_the_header(L):
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "salf.h"
int main(void) {
  printf("SceneDesc %zu %zu %zu\n", sizeof(salf_scene_desc), offsetof(salf_scene_desc, root_dims), offsetof(salf_scene_desc, flags));
  printf("SceneStats %zu %zu\n", sizeof(salf_scene_stats), offsetof(salf_scene_stats, workspace_bytes));
  printf("Sensor %zu %zu %zu\n", sizeof(salf_sensor), offsetof(salf_sensor, R0), offsetof(salf_sensor, t_far));
  printf("Rays %zu %zu\n", sizeof(salf_rays), offsetof(salf_rays, t_far));
  printf("RenderOpts %zu %zu %zu %zu\n", sizeof(salf_render_opts), offsetof(salf_render_opts, schedule), offsetof(salf_render_opts, work_bytes), offsetof(salf_render_opts, pieces));
  printf("Outputs %zu %zu %zu %zu\n", sizeof(salf_outputs), offsetof(salf_outputs, n_hits), offsetof(salf_outputs, hit_t), offsetof(salf_outputs, hit_capacity));
  printf("GradsIn %zu %zu\n", sizeof(salf_grads_in), offsetof(salf_grads_in, d_intensity));
  printf("ServerOpts %zu %zu %zu\n", sizeof(salf_server_opts), offsetof(salf_server_opts, max_inflight), offsetof(salf_server_opts, max_launch_rays));
  printf("ServerStats %zu %zu\n", sizeof(salf_server_stats), offsetof(salf_server_stats, inflight));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "l.c")
        exe = os.path.join(td, "l")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {ln.split()[0]: [int(x) for x in ln.split()[1:]] for ln in out if ln.strip()}
    S = L
    want = {
        "SceneDesc": [C.sizeof(S.SceneDesc), S.SceneDesc.root_dims.offset, S.SceneDesc.flags.offset],
        "SceneStats": [C.sizeof(S.SceneStats), S.SceneStats.workspace_bytes.offset],
        "Sensor": [C.sizeof(S.Sensor), S.Sensor.R0.offset, S.Sensor.t_far.offset],
        "Rays": [C.sizeof(S.Rays), S.Rays.t_far.offset],
        "RenderOpts": [C.sizeof(S.RenderOpts), S.RenderOpts.schedule.offset, S.RenderOpts.work_bytes.offset,
                       S.RenderOpts.pieces.offset],
        "Outputs": [C.sizeof(S.Outputs), S.Outputs.n_hits.offset, S.Outputs.hit_t.offset, S.Outputs.hit_capacity.offset],
        "GradsIn": [C.sizeof(S.GradsIn), S.GradsIn.d_intensity.offset],
        "ServerOpts": [C.sizeof(S.ServerOpts), S.ServerOpts.max_inflight.offset, S.ServerOpts.max_launch_rays.offset],
        "ServerStats": [C.sizeof(S.ServerStats), S.ServerStats.inflight.offset],
    }
    assert got == want


def _desc(L, dims=(4, 4, 4), K=2, s0=1.0, field=0):
    d = L.SceneDesc()
    d.origin[:] = [0.0, 0.0, 0.0]
    d.root_size = s0
    d.root_dims[:] = list(dims)
    d.max_level = K
    d.field = field
    d.flags = 0
    return d


def test_workspace_size_host_logic(L):
    lib = L.lib()
    n = C.c_size_t()
    assert lib.salf_scene_workspace_size(C.byref(_desc(L)), 100, C.byref(n)) == 0
    small = n.value
    assert lib.salf_scene_workspace_size(C.byref(_desc(L)), 10000, C.byref(n)) == 0
    assert n.value > small
    # a K = 0 scene needs no nodes: the root grid and the finest-level grid (4 B per cell each),
    # the root-bounds grid (8 B per cell), the skip-distance grid and its two build-time
    # temporaries (1 B per cell each), the traversal's packed cell records (16 B per cell), each
    # voxel's box (16 B per voxel), a minimal hash table and the counters
    assert lib.salf_scene_workspace_size(C.byref(_desc(L, dims=(32, 32, 32), K=0)), 4096, C.byref(n)) == 0
    assert 32 ** 3 * 35 + 4096 * 16 <= n.value < 32 ** 3 * 35 + 4096 * 16 + 64 * 1024
    # invalid descriptions
    for bad in (_desc(L, K=9), _desc(L, s0=0.0), _desc(L, s0=math.nan), _desc(L, dims=(0, 4, 4)),
                _desc(L, dims=(1 << 17, 4, 4), K=4), _desc(L, field=7)):
        assert lib.salf_scene_workspace_size(C.byref(bad), 10, C.byref(n)) == -1
        assert len(lib.salf_last_error()) > 0
    assert lib.salf_scene_workspace_size(C.byref(_desc(L)), -1, C.byref(n)) == -1


def test_sensor_ray_count_host_logic(L):
    from paper_2507_18713_amd.api import sensor_struct
    import synth
    lib = L.lib()
    n = C.c_int64()
    assert lib.salf_sensor_ray_count(C.byref(sensor_struct(synth.config1_camera())), C.byref(n)) == 0
    assert n.value == 1920 * 1080
    assert lib.salf_sensor_ray_count(C.byref(sensor_struct(synth.config2_lidar())), C.byref(n)) == 0
    assert n.value == 131072
    bad = synth.config1_camera()
    bad["width"] = 0
    assert lib.salf_sensor_ray_count(C.byref(sensor_struct(bad)), C.byref(n)) == -1
    bad = dict(synth.config1_camera(), model=5)
    assert lib.salf_sensor_ray_count(C.byref(sensor_struct(bad)), C.byref(n)) == -1
    bad = dict(synth.config1_camera(), t_near=2.0, t_far=1.0)
    assert lib.salf_sensor_ray_count(C.byref(sensor_struct(bad)), C.byref(n)) == -1


def test_render_work_size_host_logic(L):
    from paper_2507_18713_amd.api import sensor_struct
    import synth
    lib = L.lib()
    n = C.c_size_t()
    up = lambda x: (x + 255) // 256 * 256
    # camera: 8x8 tiles; LiDAR: 32 columns x 2 beams; explicit rays: groups of 64 (or 8x8 tiles of
    # an image layout); a 256-byte header, per tile a cost key and an order entry, plus two
    # 256-entry histograms
    for s, tiles in ((synth.config1_camera(), 240 * 135), (synth.config2_lidar(), 64 * 32)):
        assert lib.salf_render_work_size(C.byref(sensor_struct(s)), None, C.byref(n)) == 0
        assert n.value == 256 + 2 * up(tiles * 4) + 2048
    r = L.Rays()
    r.o, r.d = 256, 512  # never dereferenced by a size query
    r.n, r.t_near, r.t_far, r.image_width = 1000, 0.0, math.inf, 0
    assert lib.salf_render_work_size(None, C.byref(r), C.byref(n)) == 0 and n.value == 256 + 2 * up(16 * 4) + 2048
    r.image_width = 50  # 50 x 20 image: 7 x 3 tiles
    assert lib.salf_render_work_size(None, C.byref(r), C.byref(n)) == 0 and n.value == 256 + 2 * up(21 * 4) + 2048
    assert lib.salf_render_work_size(None, None, C.byref(n)) == -1
    assert lib.salf_render_work_size(C.byref(sensor_struct(synth.config1_camera())), C.byref(r), C.byref(n)) == -1


def test_server_sizes_host_logic(L):
    from paper_2507_18713_amd.api import sensor_struct
    import synth
    lib = L.lib()
    n = C.c_size_t()
    op = L.ServerOpts()
    op.max_batch, op.max_inflight = 64, 2
    assert lib.salf_server_work_size(C.byref(op), C.byref(n)) == 0
    two = n.value
    op.max_batch = 128
    assert lib.salf_server_work_size(C.byref(op), C.byref(n)) == 0 and n.value > two > 2 * 64 * 256
    for mb, mi in ((0, 2), (257, 2), (64, 0), (64, 5)):
        op.max_batch, op.max_inflight = mb, mi
        assert lib.salf_server_work_size(C.byref(op), C.byref(n)) == -1
    op.max_batch, op.max_inflight, op.max_launch_rays = 64, 2, -1
    assert lib.salf_server_work_size(C.byref(op), C.byref(n)) == -1
    op.max_launch_rays = 1 << 21
    assert lib.salf_server_work_size(C.byref(op), C.byref(n)) == 0 and n.value == two
    cam = sensor_struct(synth.config1_camera())
    assert lib.salf_server_request_bytes(C.byref(cam), 1 | 2 | 4, C.byref(n)) == 0
    px = 1920 * 1080
    assert n.value == sum((b + 255) // 256 * 256 for b in (px * 12, px * 4, px * 4))
    assert lib.salf_server_request_bytes(C.byref(cam), 0, C.byref(n)) == -1
    assert lib.salf_server_request_bytes(C.byref(cam), 16, C.byref(n)) == -1
    assert lib.salf_server_create(None, None, None) == -1
    assert lib.salf_server_destroy(None) == -1


def test_null_arguments_are_rejected(L):
    lib = L.lib()
    assert lib.salf_create(0, None) == -1
    assert lib.salf_destroy(None) == -1
    assert lib.salf_sync(None, None) == -1
    assert lib.salf_render(None, 0, None, None, None, None, None) == -1
    assert lib.salf_scene_get_stats(None, 0, None) == -1


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2, r.stderr
    assert "one GPU" in r.stderr
