"""Several sensors rendered in one launch (salf_render_multi): every item equals salf_render of it
bit for bit (the same device function renders a tile) and the CPU oracle on its own rays to
tolerance, in a launch of few tiles (cost-ordered across items) and one of more than 2^17 tiles
(item order)."""
import numpy as np
import pytest
import torch

import synth

from test_gpu_render import dev
from test_gpu_serve import OUTS, _oracle_check, _sensors, prepared, salf, scenes  # noqa: F401 (fixtures)

pytestmark = pytest.mark.gpu


def test_multi_sensor_launch_equals_single_renders_and_the_oracle(salf, scenes, prepared):
    """salf_render_multi: every sensor of the uneven mix, over raw and pre-activated scenes, in one
    launch (few tiles: cost-ordered across items) equals salf_render of that sensor bit for bit and
    the oracle to tolerance; the same for a launch of more than 2^17 tiles (item order)."""
    sens = _sensors()
    items = [(scenes[j % 3], s, OUTS[kind] + ("t_end", "n_hits")) for j, (kind, s) in enumerate(sens)]
    res = salf.render_multi(items)
    for q, ((sc, s, outs), r) in enumerate(zip(items, res)):
        alone = salf.render(sc, sensor=s, outputs=outs)
        for k in outs:
            assert torch.equal(r[k], alone[k]), (q, k)
        _oracle_check(r, prepared[q % 3], s, sens[q][0], seed=100 + q)
    big = [(scenes[1], synth.pinhole(1920, 1080, 70.0, synth.look_at((7.0, -6.0, 4.0), (0, 0, 0)), (7.0, -6.0, 4.0)),
            ("rgb", "depth", "n_hits"))] * 5 + [(scenes[0], sens[7][1], ("depth", "intensity", "n_hits"))]
    for (sc, s, outs), r in zip(big, salf.render_multi(big)):
        alone = salf.render(sc, sensor=s, outputs=outs)
        for k in outs:
            assert torch.equal(r[k], alone[k]), k
    paper = salf.Scene.from_data(synth.random_scene(206), device=dev(), field="paper")
    with pytest.raises(salf.SalfError, match="UNSUPPORTED"):
        salf.render_multi([(paper, sens[0][1], ("rgb",))])
