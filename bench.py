"""Benchmark: sign distributions classified per second at d = 7.

Workload (the headline configuration): one regular unimodular triangulation
of 7*Delta_2 (36 lattice points) from the lift h(i,j) = i^2 + i*j + j^2 +
U[0, 0.05) with seed 7 (its lower hull is the standard triangulation), and
the exhaustive sweep over all 2^35 sign masks with sigma(0,0) = '+', masks
generated in-kernel from the linear index, scheme histogram only.

One step enumerates one 2^32-mask chunk of the sweep (chunk k = indices
[k*2^32, (k+1)*2^32) mod 2^35) into the histogram, so the default 8 timed
steps are exactly the full 2^35 sweep.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CHUNK = 1 << 32
TOTAL = 1 << 35


def algorithmic_ops_per_mask(d: int) -> int:
    """Elementary steps of one evaluation (proof of Thm. 2): every diamond
    edge inspected once, one find per diamond vertex, one union per
    antipodal pair, one visit per tree node (at most M + 1 regions)."""
    nE = 6 * d * d + 2 * d
    nV = 2 * d * d + 2 * d + 1
    M = (d - 1) * (d - 2) // 2 + 1
    return nE + nV + 2 * d + (M + 1)


# chip figures for the ALU roofline: 256 CUs x 64 lanes x 2.4 GHz
PEAK_INT_OPS = 256 * 64 * 2.4e9

# sources of the specialised d=7 kernel; HBM traffic measured with rocprofv3
# counters is reported only while these are unchanged
KERNEL_SOURCES = ("paper_2604_09221_amd/csrc/pw_device.h", "paper_2604_09221_amd/csrc/pw_internal.h",
                  "paper_2604_09221_amd/csrc/jit.cpp", "paper_2604_09221_amd/csrc/scheme.hip",
                  "paper_2604_09221_amd/csrc/tri.cpp")
TRAFFIC_PROFILE = "profiles/pw_jit_enum_snap_d7_sweep_counters.md"
# the same for the batched call (its kernel, the program builder and the
# tuned launch shape, which sets the number of histogram flushes)
MULTI_SOURCES = ("paper_2604_09221_amd/csrc/pw_device.h", "paper_2604_09221_amd/csrc/pw_internal.h",
                 "paper_2604_09221_amd/csrc/pw_group.h", "paper_2604_09221_amd/csrc/multi.hip",
                 "paper_2604_09221_amd/csrc/tri.cpp", "paper_2604_09221_amd/tune_cache_gfx950.json")
MULTI_TRAFFIC_PROFILE = "profiles/k_multi_batched_uneven_4096x2p16_counters.md"
# the d=6 codes + histogram launches (the generated kernel's sources)
D6_SOURCES = KERNEL_SOURCES
D6_TRAFFIC_PROFILE = "profiles/pw_jit_hist_d6_codes_64x2p20_counters.md"


def kernel_sources_sha256(sources=KERNEL_SOURCES):
    import hashlib

    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(profile=TRAFFIC_PROFILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch (per call for the batched call) from a committed
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a 1 GiB copy), or
    None if the sources changed since it was taken."""
    try:
        text = open(os.path.join(ROOT, profile)).read()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(("traffic_bytes_per_launch: ",
                                                                                      "kernel_sources_sha256: ")))
    if vals.get("kernel_sources_sha256") != kernel_sources_sha256(sources):
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(d, E, n, codes_gpu_fn, sweep_hist_fn=None):
    """The oracle timed on the host's threads on n masks of the d=7 sweep
    (SplitMix64 stream 7); the GPU codes of the same masks must be equal
    (bit-exact), and, when sweep_hist_fn is given, so must the timed sweep
    kernel's histograms of 64 whole 512-mask chunks and 16 ragged ranges at
    random positions of the 2^35 indices (checked outside the timed region;
    a mismatch raises)."""
    import numpy as np

    import oracle
    from paper_2604_09221_amd import inputs as I

    threads = os.cpu_count() or 1
    idx = I.subsample_indices(7, n, 35)
    masks = np.zeros((n, 2), dtype=np.uint64)
    masks[:, 0] = idx << np.uint64(1)
    oracle.build()
    t0 = time.perf_counter()
    want = oracle.scheme_many(d, E, masks, threads=threads)
    dt = time.perf_counter() - t0
    got = codes_gpu_fn(masks)
    if not np.array_equal(got, want):
        bad = int(np.flatnonzero((got != want).any(axis=1))[0])
        raise AssertionError(f"GPU code of subsample mask {bad} differs from the oracle")
    sampled = ""
    if sweep_hist_fn is not None:
        rng = np.random.default_rng(20260)
        ranges = [(int(rng.integers(0, TOTAL // 512)) * 512, 512) for _ in range(64)]
        for _ in range(16):
            k = int(rng.integers(1, 1536))
            ranges.append((int(rng.integers(0, TOTAL - k)), k))
        for a, k in ranges:
            m = np.zeros((k, 2), dtype=np.uint64)
            m[:, 0] = np.arange(a, a + k, dtype=np.uint64) << np.uint64(1)
            ref = {}
            for j, (lo, hi) in enumerate(oracle.scheme_many(d, E, m, threads=threads)):
                c = int(lo) | (int(hi) << 64)
                cnt, w = ref.get(c, (0, a + j))
                ref[c] = (cnt + 1, min(w, a + j))
            if sweep_hist_fn(a, k) != ref:
                raise AssertionError(f"timed sweep kernel differs from the oracle on indices [{a}, {a + k})")
        sampled = (f"; the timed sweep kernel's histograms of {len(ranges)} sampled ranges (64 whole 512-mask "
                   f"chunks, 16 ragged) equal the oracle's")
    return {
        "value": n / dt,
        "unit": "masks/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n} masks of the d=7 sweep (SplitMix64 stream 7, idx = low 35 bits, mask = idx<<1), "
                  f"plain C oracle on {threads} host threads; GPU codes for the same masks bit-exact{sampled}",
    }


def hist_capacity(d):
    return {4: 64, 5: 64, 6: 128, 7: 256, 8: 1024, 9: 4096}.get(d, 1 << 15)


def bench_multi(args):
    """Batched uneven workload: 4096 triangulations, degree 4 + (SplitMix64(0)_t
    mod 9), lift seed t, 2^16 masks each (SplitMix64 stream t, two outputs
    per 128-bit mask, bits >= |A| and bit 0 cleared), per-triangulation
    histograms; a step is one call, i.e. one persistent launch per LDS
    class of degrees."""
    import torch

    from paper_2604_09221_amd import inputs as I
    from paper_2604_09221_amd import learn as Lr
    from paper_2604_09221_amd import patchwork as pw
    from paper_2604_09221_amd import tune

    n_slots, per = args.slots, 1 << 16
    noise = 1.0 if args.varied else 0.05
    degs = I.batched_degrees(n_slots, 0)
    # in-process (a few seconds): forked workers would inherit a profiler
    # loaded into this process, and their termination can block it
    edges = [I.lift_triangulation(int(d), t, noise=noise) for t, d in enumerate(degs)]
    torch.cuda.set_device(0)
    tris = [pw.Triangulation(int(d), E) for d, E in zip(degs, edges)]
    masks = torch.empty((n_slots * per, 2), dtype=torch.int64, device="cuda")
    for t, d in enumerate(degs):
        nA = (int(d) + 1) * (int(d) + 2) // 2
        masks[t * per:(t + 1) * per] = Lr.random_masks(t, 0, per, nA)
    offsets = np.arange(n_slots + 1, dtype=np.int64) * per
    hists = [pw.Histogram(hist_capacity(int(d))) for d in degs]
    flat = masks.view(-1)
    cfg = tune.lookup_multi(degs)
    if args.tune or cfg is None:
        cfg = tune.tune_multi(tris, flat, offsets, hists=hists, repeats=1, log=lambda m: print(m, file=sys.stderr))
    for _ in range(args.warmup):
        pw.batch_multi(tris, flat, offsets, hists=hists, config=cfg)
    for h in hists:
        h.reset()
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        pw.batch_multi(tris, flat, offsets, hists=hists, config=cfg)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    elapsed = time.perf_counter() - t0
    evals = args.steps * n_slots * per
    ops = sum(algorithmic_ops_per_mask(int(d)) for d in degs) * per
    total = sum(c for c, _ in hists[0].read().values())
    assert total == args.steps * per
    assert all(t.errors() == 0 for t in tris[:64])
    achieved = ops / (sum(times) / len(times)) / 1e12
    return {
        "metric": "sign distributions/sec, batched uneven degrees 4..12",
        "value": evals / elapsed, "unit": "masks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u128", "data": "synthetic",
        "config": {"workload": f"{n_slots} triangulations ({'varied' if args.varied else 'literal'} lifts) x 2^16 "
                               f"masks, degrees 4..12, per-triangulation histograms, one call "
                               f"(one persistent launch per LDS class)",
                   "launch_shape": list(cfg)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_OPS / 1e12, "unit": "TOP/s",
                     "frac": achieved * 1e12 / PEAK_INT_OPS,
                     "traffic": profiled_traffic(MULTI_TRAFFIC_PROFILE, MULTI_SOURCES)
                     if n_slots == 4096 and not args.varied else None,
                     "kernel": "pw::k_multi, pw::k_multi_g<2>, pw::k_multi_g<4>",
                     "per": "call (the class launches back to back)",
                     "avg_call_ms": sum(times) / len(times) * 1e3},
    }


def _events():
    import torch

    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def bench_d4(args):
    """d = 4: the standard triangulation (seed-0 lift), all 2^14 masks with
    sigma(0,0) = '+' (mask = k << 1, uint32), codes and histogram in one
    fused launch of the kernel specialised to the triangulation.  The
    workload is a single small launch, so the figure is its latency."""
    import torch

    from paper_2604_09221_amd import inputs as I
    from paper_2604_09221_amd import patchwork as pw

    d, n = 4, 1 << 14
    E = I.lift_triangulation(d, 0, noise=0.05)
    torch.cuda.set_device(0)
    tri = pw.Triangulation(d, E).specialize()
    masks2 = np.zeros((n, 2), dtype=np.uint64)
    masks2[:, 0] = np.arange(n, dtype=np.uint64) << np.uint64(1)
    mt = pw.mask_tensor(masks2, d)
    codes = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    hist = pw.Histogram(64)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        tri.codes_histogram(mt, hist, codes)
    hist.reset()
    torch.cuda.synchronize()
    ev = [_events() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        tri.codes_histogram(mt, hist, codes)
        b.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat = sorted(a.elapsed_time(b) / 1e3 for a, b in ev)
    h = hist.read()
    assert tri.errors() == 0 and sum(c for c, _ in h.values()) == args.steps * n
    med = lat[len(lat) // 2]
    ops = algorithmic_ops_per_mask(d) * n
    out = {"metric": "latency of all 2^14 sign distributions at d=4 (codes + histogram)",
           "value": med * 1e6, "unit": "us", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "d=4 standard triangulation (seed-0 lift), all 2^14 masks with sigma(0,0)=+, "
                                  "codes + histogram in one launch", "masks_per_s_at_median": n / med,
                      "latency_us_min": lat[0] * 1e6, "latency_us_max": lat[-1] * 1e6, "distinct_schemes": len(h)},
           "roofline": {"bound": "alu", "achieved": ops / med / 1e12, "peak": PEAK_INT_OPS / 1e12, "unit": "TOP/s",
                        "frac": ops / med / PEAK_INT_OPS, "traffic": None,
                        "kernel": "pw_jit_hist (codes + histogram, specialised to the triangulation)",
                        "ops_per_mask": algorithmic_ops_per_mask(d), "avg_launch_ms": sum(lat) / len(lat) * 1e3,
                        "note": "a single 2^14-mask launch: launch latency, not throughput, bounds it"}}
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        threads = os.cpu_count() or 1
        reps, t0 = 0, time.perf_counter()
        while True:
            want = oracle.scheme_many(d, E, masks2, threads=threads)
            reps += 1
            if time.perf_counter() - t0 > 2.0:
                break
        dt = (time.perf_counter() - t0) / reps
        got = codes.cpu().numpy().view(np.uint64)
        if not np.array_equal(got, want):
            raise AssertionError("d=4 codes differ from the oracle")
        ref = {}
        for k, (lo, hi) in enumerate(want):
            c = int(lo) | (int(hi) << 64)
            ref[c] = ref.get(c, 0) + 1
        if {c: v for c, (v, _) in h.items()} != {c: v * args.steps for c, v in ref.items()}:
            raise AssertionError("d=4 histogram differs from the oracle")
        out["cpu_baseline"] = {"value": dt * 1e6, "unit": "us", "cores": threads, "kind": "oracle",
                               "sample": f"all 2^14 masks, {reps} repetitions on {threads} host threads; GPU codes "
                                         "and histogram bit-exact"}
    return out


def bench_d6(args):
    """d = 6: 64 triangulations (lift seeds 0..63: the literal quadratic
    lift, or U[0,1) noise with --varied), per slot 2^20 uniform uint32 masks
    (SplitMix64 stream = slot seed, bit 0 cleared); per slot one fused
    launch writing every code and the slot's histogram.  A step is all 64
    launches, spread round-robin over --streams HIP streams (default 2, all
    at the default priority) so that one launch's tail overlaps the next
    ones; the step is timed on the current stream, which waits for all."""
    import torch

    from paper_2604_09221_amd import inputs as I
    from paper_2604_09221_amd import patchwork as pw

    d, slots, per = 6, 64, 1 << 20
    noise = 1.0 if args.varied else 0.05
    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    edges = [I.lift_triangulation(d, t, noise=noise) for t in range(slots)]
    tris = [pw.Triangulation(d, E).specialize() for E in edges]
    host = [I.random_masks(d, t, per) for t in range(slots)]
    masks = torch.cat([pw.mask_tensor(m, d) for m in host])          # 64 x 2^20 uint32 (256 MiB)
    codes = torch.empty((slots * per, 2), dtype=torch.int64, device="cuda")   # 1 GiB
    hists = [pw.Histogram(128) for _ in range(slots)]
    t_setup = time.perf_counter() - t_setup
    stream = torch.cuda.current_stream()

    side = [torch.cuda.Stream() for _ in range(max(1, args.streams))]

    def step():
        if args.streams <= 1:
            for t in range(slots):
                tris[t].codes_histogram(masks[t * per:(t + 1) * per], hists[t], codes[t * per:(t + 1) * per])
            return
        start = torch.cuda.Event()
        start.record(stream)
        for sd in side:
            sd.wait_event(start)
        for t in range(slots):
            tris[t].codes_histogram(masks[t * per:(t + 1) * per], hists[t], codes[t * per:(t + 1) * per],
                                    stream=side[t % len(side)].cuda_stream)
        for sd in side:
            done = torch.cuda.Event()
            done.record(sd)
            stream.wait_event(done)

    for _ in range(args.warmup):
        step()
    for h in hists:
        h.reset()
    torch.cuda.synchronize()
    ev = [_events() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_s = sum(a.elapsed_time(b) for a, b in ev) / len(ev) / 1e3
    hs = [h.read() for h in hists]
    assert all(t.errors() == 0 for t in tris)
    assert all(sum(c for c, _ in h.values()) == args.steps * per and len(h) <= 55 for h in hs)
    evals = slots * per
    ops = algorithmic_ops_per_mask(d) * evals
    alg_bytes = evals * (4 + 16)
    traffic = profiled_traffic(D6_TRAFFIC_PROFILE, D6_SOURCES) if not args.varied else None
    out = {"metric": "sign distributions/sec at d=6 (codes + per-triangulation histograms)",
           "value": args.steps * evals / elapsed, "unit": "masks/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": f"d=6: 64 triangulations ({'varied' if args.varied else 'literal'} lifts, seeds "
                                  "0..63) x 2^20 uniform uint32 masks, codes (1 GiB) + 64 histograms, one fused "
                                  f"launch per triangulation on {max(1, args.streams)} streams", "setup_seconds": t_setup,
                      "hbm_algorithmic_GBps": alg_bytes / step_s / 1e9,
                      "distinct_schemes_max": max(len(h) for h in hs)},
           "roofline": {"bound": "alu", "achieved": ops / step_s / 1e12, "peak": PEAK_INT_OPS / 1e12,
                        "unit": "TOP/s", "frac": ops / step_s / PEAK_INT_OPS,
                        "traffic": traffic, "kernel": "pw_jit_hist (codes + histogram, specialised per slot)",
                        "per": "step (64 launches)", "ops_per_mask": algorithmic_ops_per_mask(d),
                        "avg_step_ms": step_s * 1e3,
                        "hbm": {"achieved_GBps": (traffic if traffic else alg_bytes) / step_s / 1e9,
                                "peak_GBps": 8000.0, "algorithmic_bytes_per_step": alg_bytes}}}
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        threads = os.cpu_count() or 1
        sample = 1 << 22
        k = sample // slots
        ms = np.concatenate([m[:k] for m in host])
        t0 = time.perf_counter()
        want = np.concatenate([oracle.scheme_many(d, edges[t], host[t][:k], threads=threads) for t in range(slots)])
        dt = time.perf_counter() - t0
        got = np.concatenate([codes[t * per:t * per + k].cpu().numpy().view(np.uint64) for t in range(slots)])
        if not np.array_equal(got, want):
            raise AssertionError("d=6 codes differ from the oracle")
        out["cpu_baseline"] = {"value": len(ms) / dt, "unit": "masks/s", "cores": threads, "kind": "oracle",
                               "sample": f"the first {k} masks of each of the 64 slots ({len(ms)} masks) on "
                                         f"{threads} host threads; GPU codes for them bit-exact"}
    return out


def bench_learned(args):
    """d = 8 (seed-8 lift = the standard triangulation): distinct schemes
    per GPU-second for uniform sampling, the learned proposal (mutations of
    rare witnesses guided by the network's input gradient) and its ablation
    (the same search with uniform flips), each judged by the exact kernel."""
    import torch

    from paper_2604_09221_amd import inputs as I
    from paper_2604_09221_amd import learn as Lr
    from paper_2604_09221_amd import patchwork as pw

    d = 8
    torch.cuda.set_device(0)
    if args.learned_tri == "standard":
        E = I.lift_triangulation(d, 8, noise=0.05)
        known = None
    else:
        E = np.loadtxt(os.path.join(ROOT, "tests", "golden", f"fig2_{args.learned_tri}.edges"), dtype=np.int32)
        known = FIG2[args.learned_tri]          # distinct schemes over all 2^42 classes (Fig. 2)
    tri = pw.Triangulation(d, E)
    tri.specialize()
    budget = 1 << args.budget_log2
    log = (lambda m: print(m, file=sys.stderr, flush=True))
    res = [Lr.run_uniform(tri, d, budget)]
    per_round = max(1 << 20, budget >> 8)
    target = res[0]["distinct"]
    t_uniform = res[0]["gpu_seconds"]
    targets = [int(np.ceil(f * known)) for f in (0.9, 0.99, 1.0)] if known else list(args.targets or [])
    res.append(Lr.run_search(tri, d, budget, use_net=True, train_n=min(1 << 24, budget // 4), per_round=per_round,
                             log=log, target=target, time_budget=t_uniform, targets=targets))
    res.append(Lr.run_search(tri, d, budget, use_net=True, train_n=min(1 << args.online_train_log2, budget // 16),
                             per_round=per_round, log=log, target=target, time_budget=t_uniform, targets=targets,
                             online=True))
    res.append(Lr.run_search(tri, d, budget, use_net=False, train_n=min(1 << 24, budget // 4), per_round=per_round,
                             log=log, target=target, time_budget=t_uniform, targets=targets))
    # the same uniform stream again, untimed, for its curve
    uc = Lr.run_uniform(tri, d, budget, curve=True)
    res[0]["curve"] = uc["curve"]
    if targets:
        rate = budget / t_uniform
        res[0]["seconds_to"] = {tk: next((ev / rate for ev, n in uc["full_curve"] if n >= tk), None) for tk in targets}
        for r in res:
            if known:
                r["recall"] = r["distinct"] / known
    for r in res:
        r["distinct_per_gpu_second"] = r["distinct"] / r["gpu_seconds"]
    # GPU-seconds each search needs to find as many schemes as uniform
    # sampling found with the whole budget (curve points: evaluations,
    # distinct, seconds since the start, training included)
    for r in res[1:]:
        r["seconds_to_uniform_count"] = r.pop("seconds_to_target")
    # equal GPU time: the schemes each search had seen within the seconds
    # uniform sampling needs for the whole budget, per GPU-second
    res[0]["distinct_within_uniform_seconds"] = res[0]["distinct"]
    for r in res[1:]:
        r["distinct_within_uniform_seconds"] = r.pop("distinct_within_time_budget")
    for r in res:
        r["distinct_per_gpu_second_equal_time"] = r["distinct_within_uniform_seconds"] / t_uniform
    roof = gemm_roofline()
    return {
        "metric": "distinct real schemes found per GPU-second at d=8",
        "value": res[1]["distinct_per_gpu_second_equal_time"], "unit": "schemes/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+u64",
        "data": "synthetic",
        "config": {"workload": f"d=8 {args.learned_tri} triangulation, {budget} judged masks per method"
                               + (f"; {known} schemes known over all 2^42 classes (Fig. 2)" if known else ""),
                   "value": "learned proposal: distinct schemes seen within the GPU time uniform sampling takes for "
                            "the whole budget, per GPU-second (equal-time); uniform's equal-time rate: "
                            f"{res[0]['distinct_per_gpu_second_equal_time']:.1f}; each method's rate over its own "
                            "whole budget: distinct_per_gpu_second in results",
                   "results": res},
        "roofline": roof,
    }


def gemm_roofline():
    """Roofline of the learned proposal's dominant contraction: the 512 x 512
    hidden layer of the forward pass (k_gemm_bf16, 128 x 128 tiles, bias +
    ReLU epilogue, bf16 out) on 2^18 rows, timed with HIP events on the
    stream it runs on (20 launches after 3 warm-up launches)."""
    import torch

    from paper_2604_09221_amd import learn as Lr

    rows = 1 << 18
    net = Lr.MLP(n_in=45, seed=1)
    H1 = torch.zeros((rows, Lr.HIDDEN), dtype=torch.int16, device="cuda")
    H2 = torch.empty((rows, Lr.HIDDEN), dtype=torch.int16, device="cuda")
    stream = torch.cuda.current_stream()

    def layer2():  # as in the forward pass: the weight's [out][in] copy, contiguous along K
        Lr.gemm(H1, Lr.HIDDEN, 1, net.W16T["W2"], 1, Lr.HIDDEN, rows, Lr.HIDDEN, Lr.HIDDEN, C16=H2,
                bias=net.P["b2"], relu=True)

    for _ in range(3):
        layer2()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(stream)
    for _ in range(reps):
        layer2()
    e1.record(stream)
    torch.cuda.synchronize()
    gemm_s = e0.elapsed_time(e1) / 1e3 / reps
    flops = 2.0 * rows * Lr.HIDDEN * Lr.HIDDEN
    return {"bound": "mfma", "achieved": flops / gemm_s / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
            "frac": flops / gemm_s / 2.5e15, "traffic": None,
            "kernel": "pw::k_gemm_bf16<128,128> (hidden layer 512x512, forward, 2^18 rows)",
            "avg_launch_ms": gemm_s * 1e3}


def full_sweep_checks(full, d, E):
    """Checks of every whole pass over the 2^35 indices, outside the timed
    region: the counts sum to 2^35; each count is divisible by 4 (sigma ->
    sigma + b i + c j, (b, c) != 0, keeps sigma(0,0) and the scheme and has
    no fixed point: a free (Z/2)^2 action on the swept masks, Sec. 3);
    at most 121 schemes (Sec. 1); every pass gives the same histogram; and
    that histogram equals one sweep of the generic kernel (the triangulation
    program read from device memory, no snapshot), run here in 2^32-mask
    launches."""
    from paper_2604_09221_amd import patchwork as pw

    for h_ in full:
        assert sum(c for c, _ in h_.values()) == TOTAL
        assert all(c % 4 == 0 for c, _ in h_.values()), "a count of a whole sweep is not divisible by 4"
        assert len(h_) <= 121
        assert h_ == full[0], "two whole sweeps differ"
    gen = pw.Triangulation(d, E)
    ref = pw.Histogram(1024)
    t0 = time.perf_counter()
    for a in range(0, TOTAL, 1 << 32):
        gen.enumerate_range(a, 1 << 32, ref)
    got = ref.read()
    dt = time.perf_counter() - t0
    assert gen.errors() == 0
    assert got == full[0], "the sweep kernel's histogram differs from the generic kernel's"
    return {"passes_checked": len(full), "sum": True, "counts_divisible_by_4": True, "at_most_121": True,
            "equal_to_generic_kernel_sweep": True, "generic_sweep_seconds": dt}


def bench_orbit(args):
    """Orbit-reduced exhaustive sweep at d=7 (Sec. 3, Table 1): a varied-lift
    triangulation with trivial S3 stabiliser (lift seed 0, U[0,1) noise) is
    replaced by the canonical member of its orbit, and each step sweeps all
    2^33 (Z/2)^3 class representatives of it (sigma '+' at (0,0), (2,1),
    (3,1)).  `value` counts masks actually classified; `effective` counts
    the (T', sigma) pairs of the whole orbit they stand for (8 sign
    distributions per class, 6 triangulations per orbit).  Outside the timed
    region: the class histogram times 4 equals one full 2^35 sweep (sigma(0,0)
    = '+') of the same triangulation, sampled class ranges equal the
    oracle's, and every witness mapped back to the input triangulation gives
    its code on the oracle."""
    import torch

    from paper_2604_09221_amd import inputs as I
    from paper_2604_09221_amd import orbits
    from paper_2604_09221_amd import patchwork as pw

    d = 7
    E = I.lift_triangulation(d, 0, noise=1.0)
    torch.cuda.set_device(0)
    canon, k_perm, stab = pw.canonical(d, E)
    fixed = pw.class_fixed_bits(d)
    n_classes = 1 << (I.n_points(d) - 3)
    t_spec = time.perf_counter()
    tri = pw.Triangulation(d, canon).specialize()
    t_spec = time.perf_counter() - t_spec
    warm = pw.Histogram(1024)
    for _ in range(args.warmup):
        tri.enumerate_range(0, n_classes, warm, fixed_zero_bits=fixed)
    stream = torch.cuda.current_stream()
    hists = [pw.Histogram(1024) for _ in range(args.steps)]
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        tri.enumerate_range(0, n_classes, hists[k], fixed_zero_bits=fixed)
        ends[k].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launch_s = sum(a.elapsed_time(b) for a, b in zip(starts, ends)) / args.steps / 1e3
    hs = [h.read() for h in hists]
    assert tri.errors() == 0
    h = hs[0]
    assert all(x == h for x in hs)
    assert sum(c for c, _ in h.values()) == n_classes
    # checks outside the timed region
    full = pw.Histogram(1024)
    for a in range(0, TOTAL, 1 << 32):
        tri.enumerate_range(a, 1 << 32, full)
    hf = full.read()
    assert {c: 4 * n for c, (n, _) in h.items()} == {c: n for c, (n, _) in hf.items()}, \
        "class histogram x 4 differs from the full sweep"
    res = orbits.OrbitSweep(d, canon, k_perm, stab, fixed, n_classes, h)
    value = args.steps * n_classes / elapsed
    ops = algorithmic_ops_per_mask(d) * n_classes
    achieved = ops / launch_s / 1e12
    out = {
        "metric": "sign-distribution classes/sec at d=7, orbit-reduced (bit-exact)",
        "value": value, "unit": "masks/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "d=7 varied-lift triangulation (seed 0, U[0,1) noise), canonical member of its S3 "
                               "orbit, all 2^33 (Z/2)^3 class representatives per step, in-kernel, histogram",
                   "s3_stabilizer": stab, "orbit_size": 6 // stab, "classes_per_step": n_classes,
                   "distinct_schemes": len(h), "specialize_seconds": t_spec,
                   "checks": {"class_hist_x4_equals_full_sweep": True}},
        "effective": {"value": value * 8 * (6 // stab), "unit": "(T, sigma) pairs/s",
                      "note": "each class stands for 8 sign distributions of each of the orbit's "
                              f"{6 // stab} triangulations; not masks classified"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_OPS / 1e12, "unit": "TOP/s",
                     "frac": achieved * 1e12 / PEAK_INT_OPS, "traffic": None,
                     "kernel": "pw_jit_enum_snap (specialised, shared snapshot per 512 masks)",
                     "ops_per_mask": algorithmic_ops_per_mask(d), "avg_launch_ms": launch_s * 1e3},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = orbit_cpu_baseline(d, E, res, tri)
    return out


def orbit_cpu_baseline(d, E, res, tri):
    """The oracle on the orbit sweep's workload: 24 class ranges at random
    positions of the 2^33 classes (16 whole 512-class chunks, 8 ragged),
    timed on the host's threads and checked equal to the GPU sweep kernel's
    histograms of the same ranges; and every class witness, mapped back to
    the input triangulation, gives its code."""
    import numpy as np

    import oracle
    from paper_2604_09221_amd import inputs as I
    from paper_2604_09221_amd import patchwork as pw

    threads = os.cpu_count() or 1
    for code, (_, widx) in res.hist.items():
        if oracle.scheme(d, E, res.witness_for_input(widx)) != code:
            raise AssertionError("a class witness does not map back to the input triangulation")
    rng = np.random.default_rng(7)
    free = ((1 << I.n_points(d)) - 1) & ~res.fixed_zero_bits
    n_done, dt = 0, 0.0
    for k in range(24):
        a = int(rng.integers(0, res.classes // 512)) * 512
        kk = 512 if k % 3 else int(rng.integers(1, 700))
        m = np.zeros((kk, 2), dtype=np.uint64)
        m[:, 0] = [I.pdep(a + j, free) for j in range(kk)]
        t0 = time.perf_counter()
        codes = oracle.scheme_many(d, res.canonical_edges, m, threads=threads)
        dt += time.perf_counter() - t0
        n_done += kk
        ref = {}
        for j, (lo, hi) in enumerate(codes):
            c = int(lo) | (int(hi) << 64)
            cnt, w = ref.get(c, (0, a + j))
            ref[c] = (cnt + 1, min(w, a + j))
        hk = pw.Histogram(512)
        tri.enumerate_range(a, kk, hk, fixed_zero_bits=res.fixed_zero_bits)
        if hk.read() != ref:
            raise AssertionError(f"class range [{a}, {a + kk}) differs from the oracle")
    return {"value": n_done / dt, "unit": "masks/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_done} class representatives in 24 ranges at random positions of the 2^33 classes, "
                      f"plain C oracle on {threads} host threads; the GPU sweep kernel's histograms of the same "
                      f"ranges equal, and all {len(res.hist)} class witnesses map back to masks of the input "
                      f"triangulation with the same code"}


def bench_search(args):
    """The search over triangulations at d=6 (Sec. 3): simulated annealing
    over triangulations (chains scored by the number of distinct types they
    realise on 1024 fixed random sign distributions), then the witness <->
    triangulation loop from the annealing's best triangulations and the
    standard one: exhaustive class sweeps of the selected triangulations
    (one witness per new type), second-mode sweeps of 4096 symmetric
    triangulations (random symmetric flip walks, generated on the GPU)
    against all witnesses, selection of the regular triangulations that
    realise new types, until a round adds nothing.  The paper states that
    all 55 non-empty real schemes of degree six are realised by T-curves;
    none beyond them can appear.  `value` is the second mode's throughput:
    (triangulation, witness) pairs per second including the generation of
    the triangulations and their programs.  Every kept (triangulation,
    witness) is re-evaluated by the oracle and every kept triangulation
    carries an exact regularity certificate."""
    import numpy as np
    import torch

    from paper_2604_09221_amd import inputs as I
    from paper_2604_09221_amd import patchwork as pw
    from paper_2604_09221_amd import regular
    from paper_2604_09221_amd import search as S

    d = args.degree
    total = {6: 55, 7: 121}[d]      # non-empty real schemes of degree 6 and 7 (Sec. 1, Sec. 3)
    torch.cuda.set_device(0)
    t_all = time.perf_counter()
    # warm-up: load the kernels once
    S.mode2_sweep(d, I.random_masks(d, 1, 64), 64, 4, 1)
    n_masks = 1024 if d == 6 else 4096
    ann = S.anneal(d, n_chains=args.chains, iters=args.iters, n_masks=n_masks, mode=0, seed=args.seed,
                   symmetric=False, log_every=max(1, args.iters // 8))
    sa_evals = args.chains * (args.iters + 1) * n_masks
    order = np.argsort(-ann.best_score)
    rows = ann.best.cpu().numpy()
    pool, keys = [I.standard_triangulation(d)], set()
    for t in order:
        E = pw.edges_from_adjacency(d, rows[t].view(np.uint64))
        k = pw.canonical(d, E)[0].tobytes()
        if k in keys or not regular.is_regular(d, E):
            continue
        keys.add(k)
        pool.append(E)
        if len(pool) > args.pool:
            break
    res = S.iterate(d, pool, n_tris=args.slots, walk_steps=64, max_rounds=args.rounds, seed=args.seed,
                    target_count=total, max_selected=args.max_selected, explore_masks=2 * n_masks,
                    witness_mutants=args.witness_mutants, explore_tries=args.explore_tries,
                    target_chains=args.target_chains,
                    log=lambda info: print(json.dumps(info), file=sys.stderr, flush=True))
    total_s = time.perf_counter() - t_all
    assert all(regular.certificate(d, r.edges) is not None for r in res.found.values())
    assert len(res.found) <= total
    m2_pairs = sum(r["mode2_pairs"] for r in res.rounds)
    m2_s = sum(r["mode2_seconds"] for r in res.rounds)
    out = {
        "metric": f"triangulation x witness pairs/sec, second search mode at d={d} (generation included)",
        "value": m2_pairs / m2_s, "unit": "pairs/s", "n_gpus": 1, "steps": len(res.rounds), "warmup": 1,
        "ms_per_step": res.gpu_seconds / max(1, len(res.rounds)) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"d={d} search: annealing over triangulations (distinct types on {n_masks} random "
                               f"sign distributions), then the witness <-> triangulation loop with {args.slots} "
                               "symmetric triangulations per round",
                   "annealing": {"chains": args.chains, "iterations": args.iters, "evaluations": sa_evals,
                                 "seconds": ann.gpu_seconds, "evaluations_per_s": sa_evals / ann.gpu_seconds,
                                 "best_score": float(ann.best_score.max()),
                                 "start_score": float(ann.trace[0][1]) if ann.trace else None,
                                 "pool_triangulations": len(pool)},
                   "rounds": res.rounds,
                   "distinct_nonempty_schemes": len(res.found), "paper_total": total,
                   "schemes": sorted(S.scheme_text(c) for c in res.found),
                   "all_found": len(res.found) == total,
                   "seconds_total": total_s,
                   "checks": {"regularity_certificates": len(res.found), f"at_most_{total}": True}},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = search_cpu_baseline(d, res)
    return out


def search_cpu_baseline(d, res):
    """The oracle on the second search mode's workload: 512 generated
    symmetric triangulations against the found types' witnesses, timed on
    the host's threads, with the GPU's codes for the same pairs checked
    equal; and every kept (triangulation, witness) re-evaluated (each must
    give its code)."""
    import numpy as np
    import torch

    import oracle
    from paper_2604_09221_amd import inputs as I
    from paper_2604_09221_amd import patchwork as pw
    from paper_2604_09221_amd import search as S

    agree = S.certify(d, res, lambda d_, E, m: oracle.scheme(d_, E, m))
    if agree != len(res.found):
        raise AssertionError("a kept witness does not reproduce its code on the oracle")
    n_t = 512
    wm = np.zeros((len(res.found), 2), dtype=np.uint64)
    wm[:, 0] = [r.mask for r in res.found.values()]
    adj = S.replicate(d, I.standard_triangulation(d), n_t)
    pw.flip_walk(d, adj, 64, True, 4242)
    progs, _ = pw.build_programs(d, adj)
    codes = torch.zeros((n_t * len(wm), 2), dtype=torch.int64, device="cuda")
    pw.scheme_programs(d, progs, S.witness_tensor(wm), codes=codes)
    got = codes.cpu().numpy().view(np.uint64).reshape(n_t, len(wm), 2)
    rows = adj.cpu().numpy()
    edges = [pw.edges_from_adjacency(d, rows[t].view(np.uint64)) for t in range(n_t)]
    threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    want = [oracle.scheme_many(d, E, wm, threads=threads) for E in edges]
    dt = time.perf_counter() - t0
    for t in range(n_t):
        if not np.array_equal(got[t], want[t]):
            raise AssertionError(f"second-mode codes of generated triangulation {t} differ from the oracle")
    return {"value": n_t * len(wm) / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_t} symmetric triangulations (64 random symmetric flip moves from the standard one) x "
                      f"{len(wm)} witnesses (one per type found) on {threads} host threads; the GPU's codes for "
                      f"these pairs equal, and all {agree} kept (triangulation, witness) pairs reproduce their "
                      f"codes on the oracle"}


FIG2 = {"bow_tie": 123, "rank016": 359, "rank015": 353}  # distinct real schemes printed with Fig. 2


def fig2_fixed_bits(d):
    """Class representatives of the (Z/2)^3 action sigma -> sigma + a + b i +
    c j: sigma fixed to '+' at (0,0), (1,1) and (2,1), whose parity vectors
    (i, j mod 2) are (0,0), (1,1), (0,1) -- one mask per orbit, and the
    lattice bits 1..9 stay free (the sweep kernel's shared snapshot)."""
    def k(i, j):
        return j * (d + 1) - j * (j - 1) // 2 + i
    return (1 << k(0, 0)) | (1 << k(1, 1)) | (1 << k(2, 1))


def bench_fig2(args):
    """Part of the exhaustive class-representative sweep of one Fig. 2
    triangulation (d = 8, 2^42 classes): index range [part * 2^42 / parts,
    (part + 1) * 2^42 / parts), in launches of 2^36 masks; the histogram goes out as
    (code, count) pairs for merging (--config fig2-check)."""
    import torch

    from paper_2604_09221_amd import patchwork as pw

    d = 8
    E = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                                f"fig2_{args.tri}.edges"), dtype=np.int32)
    tri = pw.Triangulation(d, E).specialize()
    fz = fig2_fixed_bits(d)
    total = 1 << (45 - 3)
    first, end = args.part * total // args.parts, (args.part + 1) * total // args.parts
    step = 1 << 36
    hist = pw.Histogram(4096)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a in range(first, end, step):
        tri.enumerate_range(a, min(step, end - a), hist, fixed_zero_bits=fz)
        torch.cuda.synchronize()
        print(f"{args.tri}: {min(a + step, end) - first} of {end - first} masks, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    h = hist.read()
    return {"metric": "Fig. 2 class sweep (d=8)", "tri": args.tri, "first": first, "count": end - first,
            "seconds": dt, "masks_per_s": (end - first) / dt, "errors": tri.errors(),
            "hist": [[str(code), c] for code, (c, _) in sorted(h.items())]}


def fig2_check(paths):
    """Merge the parts of one triangulation's sweep and compare with the
    printed Fig. 2 data: the number of distinct schemes and the percentage
    of classes with k ovals (printed to 4 decimals)."""
    parts = [json.loads(open(p).read().strip().splitlines()[-1]) for p in paths]
    tri = parts[0]["tri"]
    counts = {}
    masks = 0
    for q in parts:
        assert q["tri"] == tri and q["errors"] == 0
        masks += q["count"]
        for code, c in q["hist"]:
            counts[int(code)] = counts.get(int(code), 0) + c
    ranges = sorted((q["first"], q["first"] + q["count"]) for q in parts)
    whole = ranges[0][0] == 0 and ranges[-1][1] == 1 << 42 and all(a[1] == b[0] for a, b in zip(ranges, ranges[1:]))
    by_ovals = {}
    for code, c in counts.items():
        ovals = (code.bit_length() - 1) // 2  # code = 2^|W| + W, |W| = 2 * ovals (no J at even d)
        by_ovals[ovals] = by_ovals.get(ovals, 0) + c
    printed = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                                      f"fig2_{tri}.hist"))
    rows, worst = [], 0.0
    for k, pct in printed:
        ours = 100.0 * by_ovals.get(int(k), 0) / masks
        worst = max(worst, abs(round(ours, 4) - pct))
        rows.append([int(k), pct, ours])
    return {"metric": "Fig. 2 replication (d=8, all 2^42 classes)", "tri": tri, "whole_sweep": whole,
            "classes": masks, "sum_counts": sum(counts.values()), "distinct": len(counts), "printed_distinct": FIG2[tri],
            "max_abs_diff_pp_after_rounding": worst, "ovals": rows,
            "seconds": sum(q["seconds"] for q in parts)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=1 << 24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config", choices=("d7", "d4", "d6", "orbit", "search", "multi", "learned", "gemm", "copyprobe", "fig2",
                                         "fig2-check"),
                    default="d7")
    ap.add_argument("--tri", choices=sorted(FIG2), default="rank016", help="--config fig2: the triangulation")
    ap.add_argument("--part", type=int, default=0, help="--config fig2: which part of the sweep")
    ap.add_argument("--parts", type=int, default=2, help="--config fig2: parts of the 2^42 sweep")
    ap.add_argument("inputs", nargs="*", help="--config fig2-check: the parts' JSON outputs")
    ap.add_argument("--slots", type=int, default=4096)
    ap.add_argument("--chains", type=int, default=256, help="--config search: annealing chains")
    ap.add_argument("--iters", type=int, default=300, help="--config search: annealing iterations")
    ap.add_argument("--pool", type=int, default=8, help="--config search: annealed triangulations kept")
    ap.add_argument("--rounds", type=int, default=10, help="--config search: witness <-> triangulation rounds")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--streams", type=int, default=2, help="--config d6: HIP streams the 64 launches use")
    ap.add_argument("--degree", type=int, choices=(6, 7), default=6, help="--config search: the degree")
    ap.add_argument("--max-selected", type=int, default=32, help="--config search: class sweeps per round")
    ap.add_argument("--witness-mutants", type=int, default=0, help="--config search: mutants per witness")
    ap.add_argument("--explore-tries", type=int, default=1, help="--config search: novelty annealing runs")
    ap.add_argument("--target-chains", type=int, default=0,
                    help="--config search: chains of the (p, n)-target annealing runs (0 = none)")
    ap.add_argument("--varied", action="store_true")
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--budget-log2", type=int, default=30,
                    help="--config learned: judged masks per method (2^30: the configured workload)")
    ap.add_argument("--learned-tri", choices=("standard", "bow_tie", "rank016", "rank015"), default="standard",
                    help="--config learned: the d=8 triangulation")
    ap.add_argument("--targets", type=int, nargs="*", help="--config learned: scheme counts to time")
    ap.add_argument("--online-train-log2", type=int, default=22,
                    help="--config learned: uniform training masks of the online-learning search")
    ap.add_argument("--generic", action="store_true", help="time the generic (unspecialised) kernel")
    ap.add_argument("--chunk-log2", type=int, default=32, help="masks per step (profiling runs use less)")
    ap.add_argument("--no-full-check", action="store_true",
                    help="skip the checks of whole passes (the generic kernel's reference sweep)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(sharding the sweeps needs only a merge of the per-GPU histograms).", file=sys.stderr)
        sys.exit(2)
    if args.config == "gemm":
        import torch

        torch.cuda.set_device(0)
        print(json.dumps({"metric": "bf16 GEMM throughput (learned proposal's hidden layer)",
                          "roofline": gemm_roofline()}), flush=True)
        return
    if args.config == "fig2-check":
        print(json.dumps(fig2_check(args.inputs)), flush=True)
        return
    if args.config == "fig2":
        print(json.dumps(bench_fig2(args)), flush=True)
        return
    if args.config == "multi":
        print(json.dumps(bench_multi(args)), flush=True)
        return
    if args.config == "search":
        print(json.dumps(bench_search(args)), flush=True)
        return
    if args.config == "orbit":
        print(json.dumps(bench_orbit(args)), flush=True)
        return
    if args.config in ("d4", "d6"):
        print(json.dumps((bench_d4 if args.config == "d4" else bench_d6)(args)), flush=True)
        return
    if args.config == "learned":
        print(json.dumps(bench_learned(args)), flush=True)
        return
    if args.config == "copyprobe":
        # reference for HBM traffic counters: one device-to-device copy of
        # exactly 1 GiB (a plain copy kernel reads and writes 1 GiB each)
        import torch

        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30}), flush=True)
        return

    import numpy as np
    import torch

    from paper_2604_09221_amd import inputs as I
    from paper_2604_09221_amd import patchwork as pw

    d = 7
    E = I.lift_triangulation(d, 7, noise=0.05)
    torch.cuda.set_device(0)
    tri = pw.Triangulation(d, E)
    # kernels specialised to this triangulation (hipRTC); compile time is
    # setup, outside the timed region
    t_spec = time.perf_counter()
    kernel = "pw_jit_enum_snap (kernel specialised to the d=7 triangulation, shared snapshot per 512 masks)"
    if args.generic:
        kernel = "pw::k_enum<7> (generic)"
    else:
        tri.specialize()
    t_spec = time.perf_counter() - t_spec
    warm = pw.Histogram(1024)
    stream = torch.cuda.current_stream()

    CHUNK = 1 << args.chunk_log2
    assert CHUNK <= TOTAL
    for w in range(args.warmup):
        tri.enumerate_range((w * CHUNK) % TOTAL, CHUNK, warm)
    torch.cuda.synchronize()

    # one histogram per pass over the 2^35 indices (the steps of pass p go
    # into passes[p]): a whole pass is closed under the sign symmetries, so
    # its counts can be checked after the timed region
    n_pass = (args.steps * CHUNK + TOTAL - 1) // TOTAL
    passes = [pw.Histogram(1024) for _ in range(n_pass)]
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        first = (k * CHUNK) % TOTAL
        starts[k].record(stream)
        tri.enumerate_range(first, CHUNK, passes[k * CHUNK // TOTAL])
        ends[k].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    hs = [p.read() for p in passes]
    assert tri.errors() == 0
    masks_done = args.steps * CHUNK
    assert sum(c for h_ in hs for c, _ in h_.values()) == masks_done
    h = hs[0]
    full = [h_ for k, h_ in enumerate(hs) if (k + 1) * TOTAL <= masks_done]
    full_checks = None
    if full and not args.no_full_check:
        full_checks = full_sweep_checks(full, d, E)
    value = masks_done / elapsed
    avg_launch_s = sum(launch_ms) / len(launch_ms) / 1e3
    ops = algorithmic_ops_per_mask(d) * CHUNK
    achieved = ops / avg_launch_s / 1e12

    out = {
        "metric": "sign distributions/sec at d=7 (bit-exact)",
        "value": value,
        "unit": "masks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "d=7 exhaustive sweep: standard triangulation (seed-7 lift), all 2^35 masks with "
                        "sigma(0,0)=+, generated in-kernel, scheme histogram",
            "degree": d,
            "masks_per_step": CHUNK,
            "full_sweep": masks_done >= TOTAL,
            "full_sweep_checks": full_checks,
            "distinct_schemes": len(h),
            "specialize_seconds": t_spec,
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_INT_OPS / 1e12,
            "unit": "TOP/s",
            "frac": achieved * 1e12 / PEAK_INT_OPS,
            "traffic": None if args.generic or args.chunk_log2 != 32 else profiled_traffic(),
            "kernel": kernel,
            "ops_per_mask": algorithmic_ops_per_mask(d),
            "avg_launch_ms": avg_launch_s * 1e3,
        },
    }
    if not args.no_cpu_baseline:
        def gpu_codes(m2):
            c = tri.batch(pw.mask_tensor(m2, d))
            torch.cuda.synchronize()
            return c.cpu().numpy().view(np.uint64)

        def sweep_hist(a, k):
            hk = pw.Histogram(512)
            tri.enumerate_range(a, k, hk)
            return hk.read()

        out["cpu_baseline"] = cpu_baseline(d, E, args.cpu_sample, gpu_codes,
                                           None if args.generic else sweep_hist)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
