"""Oracle evaluation of many rays of the driving scene in a pool of CPU worker processes (test
helper, not collected).  Each worker builds the oracle's own copy of the scene from the seeded
generator; workers never touch the GPU.  The pool holds at most 16 workers (one GPU's CPU share).
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_W = {}


def _init(kind):
    import oracle
    import synth
    data = synth.config1_scene() if kind == "driving" else None
    _W["ps"] = oracle.prepare(data)


def _work(args):
    import oracle
    o, d, samples, t_min = args
    ps = _W["ps"]
    opts = oracle.RenderOpts(samples=samples, t_min=t_min)
    hits, outs = [], []
    for r in range(o.shape[0]):
        h = oracle.hit_list(ps, o[r], d[r])
        hits.append(h)
        outs.append(oracle.render_ray(ps, o[r], d[r], opts, hits=h))
    return hits, outs


def workers():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class OraclePool:
    """pool.run(o, d) -> (hit lists, per-ray output dicts), in ray order."""

    def __init__(self, kind="driving"):
        ctx = mp.get_context("spawn")
        self.n = workers()
        self.pool = ctx.Pool(self.n, initializer=_init, initargs=(kind,))

    def run(self, o, d, samples=4, t_min=1e-6):
        o = np.ascontiguousarray(o, np.float32)
        d = np.ascontiguousarray(d, np.float32)
        parts = max(1, min(o.shape[0], 4 * self.n))
        chunks = np.array_split(np.arange(o.shape[0]), parts)
        res = self.pool.map(_work, [(o[c], d[c], samples, t_min) for c in chunks])
        hits = [h for part in res for h in part[0]]
        outs = [x for part in res for x in part[1]]
        return hits, outs

    def close(self):
        self.pool.close()
        self.pool.join()
