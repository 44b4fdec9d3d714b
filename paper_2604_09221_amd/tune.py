"""Autotuner for the persistent multi-triangulation launch.

The launch shape of patchwork_scheme_batch_multi -- masks per work item,
waves per block, blocks per CU, and for each degree 8..12 the lanes per
mask (1, 2 or 4: one lane per mask, or a lane group sharing one mask) -- is
chosen by timing candidates on the caller's own workload (device events
around each call, best of `repeats`): every (chunk, waves, blocks) shape
with the library's default lane groups, then, from the best of those, the
lane-group size of each degree in turn (coordinate descent).  The result is
cached per degree mix in tune_cache_gfx950.json next to this file (or the
file named by $PW_TUNE).  lookup_multi() returns the cached shape, or None
(the library defaults) if the mix was never tuned.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.environ.get("PW_TUNE", os.path.join(HERE, "tune_cache_gfx950.json"))

CHUNKS = (1024, 2048, 4096, 16384)
WAVES = (1, 2)
BLOCKS_PER_CU = (0, 2)
LANE_GROUP_DEGREES = (8, 9, 10, 11, 12)
LANE_GROUPS = (1, 2, 4)


def mix_key(degrees) -> str:
    ds = sorted(set(int(d) for d in degrees))
    return "multi:" + ",".join(str(d) for d in ds)


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup_multi(degrees):
    entry = _load().get(mix_key(degrees))
    if not entry:
        return None
    return tuple(entry["config"])


def call_timer(tris, masks128, offsets, hists=None):
    """ms of one patchwork_scheme_batch_multi call with a given shape (HIP
    events around the call on the current stream)."""
    import torch

    from . import patchwork as pw

    def run(cfg):
        if hists is not None:
            for h in hists:
                h.reset()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        pw.batch_multi(tris, masks128, offsets, hists=hists, config=cfg)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    return run


def tune_multi(tris, masks128, offsets, hists=None, repeats=2, save=True, log=print, timer=None):
    """Time candidate shapes on this workload; cache and return the fastest
    (chunk, waves_per_block, blocks_per_cu, lane_groups).  timer(cfg) -> ms
    (default: call_timer on this workload)."""
    from . import patchwork as pw

    run = timer or call_timer(tris, masks128, offsets, hists)

    def timed(cfg):
        best = min(run(cfg) for _ in range(repeats))
        if log:
            log(f"tune multi {cfg}: {best:.3f} ms")
        return best

    results = []
    for chunk in CHUNKS:
        for waves in WAVES:
            for bpc in BLOCKS_PER_CU:
                cfg = (chunk, waves, bpc, pw.DEFAULT_LANE_GROUPS)
                results.append((timed(cfg), cfg))
    results.sort()
    best_ms, best_cfg = results[0]
    # lanes per mask, one degree at a time
    groups = {d: pw.lane_groups_of(best_cfg[3]).get(d, 1) for d in LANE_GROUP_DEGREES}
    present = sorted({int(t.d) for t in tris} & set(LANE_GROUP_DEGREES))
    for d in present:
        for g in [x for x in LANE_GROUPS if x != groups[d]]:
            trial = {**groups, d: g}
            cfg = (*best_cfg[:3], pw.lane_groups_code(trial))
            ms = timed(cfg)
            results.append((ms, cfg))
            if ms < best_ms:
                best_ms, best_cfg, groups = ms, cfg, trial
    results.sort()
    if save:
        data = _load()
        data[mix_key([t.d for t in tris])] = {"config": list(best_cfg), "ms": best_ms,
                                              "candidates": [[list(c), ms] for ms, c in results]}
        with open(CACHE, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return best_cfg
