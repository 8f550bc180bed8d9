"""Schedule autotuner for the walk kernels.

The walk kernels run a work list of chunks (point, first walk, walk count),
one wave per chunk; the schedule sets the smallest chunk and how many chunks
there are per resident wave.  Fewer, larger chunks cost less per chunk but
balance uneven work worse; the best pair depends on the geometry (steps per
walk), the precision and the spread of walks per point.  ``tune`` times a
small grid of schedules on a seeded sample of the real work list with the
library's own timer (device events) and keeps the fastest; results are cached
in a JSON file keyed by device, domain kind, number of holes and precision.
Host-side orchestration only: every timed run is the library's walk kernel.
"""
import json
import os

import numpy as np
import torch

from . import dtn

CANDIDATES = [{"min_chunk": m, "oversub": o} for m in (256, 1024, 4096) for o in (2, 4, 8, 16)]
DEFAULT = {"min_chunk": 512, "oversub": 4}


def _key(geom, precision):
    d = geom.desc
    n_holes = int(np.asarray(d.get("holes", np.zeros((0, 6)))).reshape(-1, 6).shape[0])
    return f"{torch.cuda.get_device_name()}|{d['kind']}|{n_holes}|{precision}"


def tune(geom, pts, walks, precision="fp64", seed=0, sample_walks=2e8, reps=1, cache_path=None,
         candidates=None, walk_begin=None):
    """Pick the fastest schedule for work like (pts, walks).

    pts [n,3] and walks [n] are device tensors; a seeded sample of points with
    about ``sample_walks`` walks in all is timed under every candidate.
    Returns (schedule dict, {str(schedule): ms})."""
    cands = list(candidates or CANDIDATES)
    key = _key(geom, precision)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["best"], cache[key]["ms"]
    n = pts.shape[0]
    w = walks.detach().cpu().numpy()
    total = float(max(w.sum(), 1))
    frac = min(1.0, sample_walks / total)
    rng = np.random.default_rng(seed)
    idx = np.flatnonzero(rng.random(n) < frac) if frac < 1.0 else np.arange(n)
    if idx.size == 0:
        idx = np.arange(min(n, 1))
    I = torch.as_tensor(idx, device=pts.device)
    P = pts[I].contiguous()
    W = walks[I].contiguous()
    B = None if walk_begin is None else walk_begin[I].contiguous()
    ms, _ = dtn.time_schedules(geom, P, W, seed, cands, reps=reps, walk_begin=B, precision=precision)
    best = cands[int(np.argmin(ms))]
    table = {f"{c['min_chunk']}/{c['oversub']}": m for c, m in zip(cands, ms)}
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = {"best": best, "ms": table}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, table
