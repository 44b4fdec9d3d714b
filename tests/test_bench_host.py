"""Host-side logic of bench.py (no GPU): the Fig. 2 class representatives
and the merge of a sweep's parts against the printed histogram."""
from __future__ import annotations

import itertools
import json

import numpy as np

import bench


def test_fig2_fixed_bits_pick_one_mask_per_orbit():
    """sigma -> sigma + a + b i + c j (mod 2) is free; fixing sigma at (0,0),
    (1,1), (2,1) must leave exactly one mask of every orbit.  Checked on the
    three bits the action can change there, for d = 8."""
    d = 8
    fz = bench.fig2_fixed_bits(d)
    pts = [(i, j) for j in range(d + 1) for i in range(d + 1 - j)]
    bit = {p: k for k, p in enumerate(pts)}     # row-major by j, then i
    assert fz == (1 << bit[(0, 0)]) | (1 << bit[(1, 1)]) | (1 << bit[(2, 1)])
    seen = set()
    for a, b, c in itertools.product((0, 1), repeat=3):
        shift = tuple((a + b * i + c * j) % 2 for (i, j) in ((0, 0), (1, 1), (2, 1)))
        seen.add(shift)
    assert len(seen) == 8                        # the 8 group elements move the 3 fixed bits apart


def _part(tmp_path, name, first, count, hist):
    p = tmp_path / name
    p.write_text(json.dumps({"metric": "m", "tri": "rank016", "first": first, "count": count, "seconds": 1.0,
                             "masks_per_s": 1.0, "errors": 0, "hist": [[str(c), n] for c, n in hist]}) + "\n")
    return str(p)


def test_fig2_check_merges_parts_and_rounds_like_the_figure(tmp_path):
    """Two parts whose counts reproduce the printed rank016 shares; codes of
    k ovals are 2^(2k) + W (no J at even d)."""
    printed = np.loadtxt(bench.os.path.join(bench.os.path.dirname(bench.__file__), "tests", "golden",
                                            "fig2_rank016.hist"))
    scale = 1 << 42
    counts = {int(k): int(round(p / 100.0 * scale)) for k, p in printed}
    total = sum(counts.values())                 # the printed shares, rounded, need not sum to 100
    code_of = {k: (1 << (2 * k)) | 2 for k in counts if counts[k]}   # one code per oval count
    half = total // 2
    h0 = [(code_of[k], n // 2) for k, n in counts.items() if n]
    h1 = [(code_of[k], n - n // 2) for k, n in counts.items() if n]
    out = bench.fig2_check([_part(tmp_path, "a.json", 0, half, h0), _part(tmp_path, "b.json", half, total - half, h1)])
    assert out["classes"] == total and out["sum_counts"] == total
    assert out["distinct"] == len(code_of)
    assert out["max_abs_diff_pp_after_rounding"] < 1e-9
    assert not out["whole_sweep"]                # [0, total) is not all 2^42 classes
    # a share moved by a few units of the last printed decimal is seen
    delta = total // 10 ** 5                     # + 0.001 percentage points of 9-oval classes
    h2 = [(c, n + (delta if c == code_of[9] else 0)) for c, n in h1]
    off = bench.fig2_check([_part(tmp_path, "c.json", 0, half, h0),
                            _part(tmp_path, "d.json", half, total - half + delta, h2)])
    assert off["max_abs_diff_pp_after_rounding"] > 5e-4


def test_fig2_check_whole_sweep(tmp_path):
    """Parts that tile [0, 2^42) make a whole sweep; a gap does not."""
    h = [((1 << 4) | 2, 1 << 41)]
    whole = bench.fig2_check([_part(tmp_path, "a.json", 0, 1 << 41, h), _part(tmp_path, "b.json", 1 << 41, 1 << 41, h)])
    assert whole["whole_sweep"] and whole["classes"] == 1 << 42
    gap = bench.fig2_check([_part(tmp_path, "c.json", 0, (1 << 41) - 512, h),
                            _part(tmp_path, "d.json", 1 << 41, 1 << 41, h)])
    assert not gap["whole_sweep"]


def test_tuner_descends_over_lanes_per_mask(tmp_path, monkeypatch):
    """The autotuner's search, with a synthetic cost model in place of the
    GPU timer: it times every (chunk, waves, blocks) shape, then changes the
    lanes per mask of one degree at a time, keeps what is faster and caches
    the result per degree mix."""
    from paper_2604_09221_amd import patchwork as pw
    from paper_2604_09221_amd import tune

    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "tune.json"))
    best_groups = {8: 2, 9: 4, 10: 4, 11: 4, 12: 1}

    def cost(cfg):
        chunk, waves, bpc, code = cfg
        g = pw.lane_groups_of(code)
        ms = 100.0 + (0 if chunk == 2048 else 5) + (0 if waves == 2 else 3) + (0 if bpc == 0 else 2)
        return ms + sum(10.0 for d in range(8, 13) if g.get(d, 1) != best_groups[d])

    class T:
        def __init__(self, d):
            self.d = d

    tris = [T(d) for d in (4, 7, 8, 9, 10, 11, 12)]
    calls = []
    cfg = tune.tune_multi(tris, None, None, repeats=1, log=None, timer=lambda c: calls.append(c) or cost(c))
    assert cfg[:3] == (2048, 2, 0)
    assert pw.lane_groups_of(cfg[3]) == {d: g for d, g in best_groups.items() if g > 1}
    assert len(calls) == len(tune.CHUNKS) * len(tune.WAVES) * len(tune.BLOCKS_PER_CU) + 5 * 2
    assert tune.lookup_multi([t.d for t in tris]) == tuple(cfg)
