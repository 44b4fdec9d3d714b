"""Search over triangulations (Sec. 3), orchestrated on the host, computed
on the device.

* ``mode2_sweep``: the second search mode -- many triangulations (random
  walks in the flip graph, optionally keeping the (i, j) -> (j, i)
  symmetry) judged against a pool of witness sign distributions.  Walks,
  programs and evaluation all run on the GPU (``pw_flip_walk``,
  ``pw_build_programs``, ``patchwork_scheme_programs``); only the
  histogram of codes comes back.
* ``anneal``: simulated annealing over triangulations, each chain scored by
  the number of distinct types it realises on a fixed sample of sign
  distributions, or by how many of them reach a target (p, n); proposals
  are single (symmetric) flip moves, accepted by the Metropolis rule
  (``pw_tri_objective``, ``pw_anneal_accept``).
* ``iterate``: the witness <-> triangulation loop: sweep every sign class of
  the selected triangulations (one witness per new type), sweep generated
  triangulations against the accumulated witnesses, select the
  triangulations that realise new types, repeat until nothing new appears.

Types count as realised only with a regular triangulation (Viro's
patchworking needs a convex one; ``regular.certificate`` gives an exact
certificate), and every witness kept is re-evaluated by the exact kernel.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I
from . import orbits
from . import patchwork as pw
from . import regular


def _torch():
    import torch

    return torch


def replicate(d: int, edges, n: int, device="cuda"):
    """n copies of one triangulation as device adjacency rows (n, 64) int64."""
    torch = _torch()
    rows = pw.adjacency_from_edges(d, edges).view(np.int64)
    return torch.from_numpy(np.tile(rows, (n, 1))).to(device)


def edges_of(d: int, adj_row) -> np.ndarray:
    """Edge list of one device (or host) adjacency row block."""
    r = adj_row.cpu().numpy() if hasattr(adj_row, "cpu") else np.asarray(adj_row)
    return pw.edges_from_adjacency(d, r.view(np.uint64))


def witness_tensor(masks2, device="cuda"):
    """(n, 2) uint64 host masks -> flat int64 device tensor."""
    torch = _torch()
    return torch.from_numpy(I.masks128(np.asarray(masks2, dtype=np.uint64).reshape(-1, 2))).to(device)


@dataclass
class Mode2Result:
    d: int
    n_tris: int
    n_w: int
    hist: dict                      # code -> (count over all pairs, smallest pair index t * n_w + w)
    adj: object                     # the batch's adjacency rows (device)
    gpu_seconds: float

    def pair(self, code):
        """(triangulation index, witness index) of a code's witness pair."""
        gi = self.hist[code][1]
        return gi // self.n_w, gi % self.n_w


def mode2_sweep(d: int, witnesses, n_tris: int, walk_steps: int, seed: int, start=None, symmetric: bool = True,
                capacity: int = 1 << 14, adj=None) -> Mode2Result:
    """Generate n_tris triangulations by `walk_steps` random (symmetric)
    flip moves from `start` (default: the standard triangulation), or take
    the device batch `adj`, and judge each against every witness."""
    torch = _torch()
    if adj is None:
        adj = replicate(d, start if start is not None else I.standard_triangulation(d), n_tris)
        t0 = time.perf_counter()
        pw.flip_walk(d, adj, walk_steps, symmetric, seed)
    else:
        t0 = time.perf_counter()
    progs, bad = pw.build_programs(d, adj)
    wt = witness_tensor(witnesses, adj.device)
    h = pw.Histogram(capacity)
    _, err = pw.scheme_programs(d, progs, wt, hist=h)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if int(bad.max().item()) != 0 or int(err.item()) != 0:
        raise pw.PatchworkError(pw.PW_ERR_INTERNAL, "a generated triangulation failed its program or evaluation checks")
    return Mode2Result(d, adj.shape[0], len(np.asarray(witnesses).reshape(-1, 2)), h.read(), adj, dt)


@dataclass
class AnnealResult:
    d: int
    best: object                    # (n_chains, 64) device adjacency of each chain's best state
    best_score: np.ndarray
    final_score: np.ndarray
    accepted: np.ndarray
    masks: np.ndarray               # the fixed sample of sign distributions the score is taken on
    gpu_seconds: float
    trace: list = field(default_factory=list)   # (iteration, max score, mean score)


def accept_table(temperature: float, n: int = 64) -> np.ndarray:
    """floor(2^24 exp(-k / temperature)) for k = 1..n (uint32)."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return np.floor((1 << 24) * np.exp(-k / max(temperature, 1e-9))).astype(np.uint32)


def score_batch(d, adj, masks_t, n_w, mode, target, known=None):
    progs, bad = pw.build_programs(d, adj)
    n = adj.shape[0]
    torch = _torch()
    codes = torch.empty((n * n_w, 2), dtype=torch.int64, device=adj.device)
    _, err = pw.scheme_programs(d, progs, masks_t, codes=codes)
    score = pw.tri_objective(d, codes, n, n_w, mode, target, known=known)
    return score, codes, bad, err


def known_tensor(codes, device="cuda"):
    """Sorted low words of scheme codes (d <= 9), for objective mode 2."""
    torch = _torch()
    lo = np.array(sorted({int(c) & ((1 << 64) - 1) for c in codes}), dtype=np.uint64)
    return torch.from_numpy(lo.view(np.int64)).to(device)


def anneal(d: int, n_chains: int, iters: int, n_masks: int = 1024, mode: int = 0, target=(0, 0),
           t_start: float = 4.0, t_end: float = 0.25, seed: int = 1, symmetric: bool = False, start=None,
           scramble: int = 64, log_every: int = 0, known=None, extra_masks=None) -> AnnealResult:
    """Simulated annealing over triangulations of degree d (<= 9), n_chains
    chains in parallel, maximising `mode` (0: distinct types on the sample,
    1: sample masks whose scheme has (p, n) = target, 2: distinct types on
    the sample not among the codes `known`).  The temperature falls
    geometrically from t_start to t_end; the chains start from `start` (a
    triangulation or a list of them, shared round-robin; default standard)
    after `scramble` random moves.  `extra_masks` ((k, 2) uint64, e.g.
    mutants of known witnesses) join the random sample."""
    torch = _torch()
    dev = "cuda"
    masks = I.random_masks(d, 0xA77 + seed, n_masks)
    if extra_masks is not None and len(extra_masks):
        masks = np.concatenate([masks, np.asarray(extra_masks, dtype=np.uint64).reshape(-1, 2)])[:8192]
        n_masks = len(masks)
    mt = witness_tensor(masks, dev)
    kt = known_tensor(known, dev) if (mode == 2 and known) else None
    starts = start if isinstance(start, list) else [start if start is not None else I.standard_triangulation(d)]
    reps = [replicate(d, E, (n_chains - k + len(starts) - 1) // len(starts), dev) for k, E in enumerate(starts)]
    cur = torch.cat(reps, 0)[:n_chains].contiguous()
    t0 = time.perf_counter()
    if scramble:
        pw.flip_walk(d, cur, scramble, symmetric, seed ^ 0x5C, step0=0)
    prop = cur.clone()
    best = cur.clone()
    score_cur, _, bad, err = score_batch(d, cur, mt, n_masks, mode, target, kt)
    score_best = score_cur.clone()
    n_acc = torch.zeros(n_chains, dtype=torch.int32, device=dev)
    tables = np.stack([accept_table(t_start * (t_end / t_start) ** (k / max(1, iters - 1))) for k in range(iters)])
    tables_t = torch.from_numpy(tables.view(np.int32)).to(dev)
    trace = []
    for it in range(iters):
        pw.flip_walk(d, prop, 1, symmetric, seed, step0=1 << 20 | it)
        score_prop, _, bad_p, err_p = score_batch(d, prop, mt, n_masks, mode, target, kt)
        pw.anneal_accept(cur, prop, score_cur, score_prop, best, score_best, tables_t[it], seed, it, n_acc)
        if log_every and (it % log_every == 0 or it == iters - 1):
            s = score_cur.cpu().numpy()
            trace.append((it, float(s.max()), float(s.mean())))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if int(bad.max().item()) or int(err.item()) or int(bad_p.max().item()) or int(err_p.item()):
        raise pw.PatchworkError(pw.PW_ERR_INTERNAL, "a chain's triangulation failed its program or evaluation checks")
    return AnnealResult(d, best, score_best.cpu().numpy(), score_cur.cpu().numpy(),
                        n_acc.cpu().numpy(), masks, dt, trace)


@dataclass
class Realised:
    edges: np.ndarray
    mask: int
    regular: bool


@dataclass
class IterateResult:
    d: int
    found: dict                     # code -> Realised (a regular triangulation and a witness)
    rounds: list                    # per round: dict of counts and seconds
    gpu_seconds: float


def _canon_key(d, E):
    c, _, _ = pw.canonical(d, E)
    return c.tobytes()


def mutants(d: int, witnesses, per: int, seed: int):
    """`per` mutants of every witness (1 to 3 random flips each, bit 0
    kept; the device mutation kernel), as (k, 2) uint64 host masks."""
    from . import learn

    torch = _torch()
    if not len(witnesses) or per <= 0:
        return np.zeros((0, 2), dtype=np.uint64)
    par = witness_tensor(witnesses).view(-1, 2)
    out = [learn.mutate(par, per * len(witnesses), I.n_points(d), f, seed * 7 + f).cpu().numpy()
           for f in (1, 2, 3)]
    return np.concatenate(out).view(np.uint64)


def explore(d: int, found: dict, starts, n_chains: int, iters: int, n_masks: int, seed: int, keep: int = 8,
            witnesses=None):
    """Annealing for novelty: chains from `starts` scored by the number of
    types not yet found that they realise on a sample of random masks and
    mutants of the known witnesses; the regular triangulations of the best
    chains with a positive score (distinct up to S3, at most `keep`)."""
    extra = None
    if witnesses is not None and len(witnesses):
        extra = mutants(d, witnesses, max(1, n_masks // (3 * len(witnesses))), seed)
    ann = anneal(d, n_chains, iters, n_masks=n_masks, mode=2, seed=seed, start=list(starts), known=list(found),
                 scramble=16, extra_masks=extra)
    rows = ann.best.cpu().numpy()
    out = {}
    for t in np.argsort(-ann.best_score):
        if ann.best_score[t] <= 0 or len(out) >= keep:
            break
        E = edges_of(d, rows[t])
        k = _canon_key(d, E)
        if k not in out and regular.is_regular(d, E):
            out[k] = E
    return out, ann


def code_pn(code: int):
    """(p, n) of a scheme code: ovals at odd depth (outermost = 1) and at
    even depth, read off the code's bit string ('1' opens a node)."""
    bits = bin(code & ((1 << 127) - 1))[3:]
    depth = p = n = 0
    for ch in bits:
        if ch == "1":
            depth += 1
            if depth % 2:
                p += 1
            else:
                n += 1
        else:
            depth -= 1
    return p, n


def explore_targets(d: int, found: dict, starts, n_chains: int, iters: int, seed: int, witnesses, keep: int = 8,
                    span: int = 2, max_targets: int = 24):
    """Annealing toward (p, n) pairs no found type has, at the highest oval
    counts reached (the top `span` + 1 totals): for each pair, chains from
    `starts` scored by how many masks of a sample reach it; the sample is
    mutants of the witnesses of the types with the most ovals and of the
    Harnack distribution, where such types live.  Returns the regular
    triangulations of the best chains with a positive score (distinct up to
    S3, at most `keep` per target) and the targets tried."""
    have = {code_pn(c) for c in found}
    tot = {c: sum(code_pn(c)) for c in found}
    top = max(tot.values()) if tot else 0
    targets = [(p, t - p) for t in range(top + 1, top - span - 1, -1) for p in range(t + 1)
               if (p, t - p) not in have][:max_targets]
    rich = [r.mask for c, r in sorted(found.items(), key=lambda kv: -tot[kv[0]])[:32]]
    base = np.zeros((len(rich) + 1, 2), dtype=np.uint64)
    for k, m in enumerate(rich + [I.harnack_mask(d)]):
        base[k, 0] = m & ((1 << 64) - 1)
        base[k, 1] = m >> 64
    sample = mutants(d, base, max(1, 2048 // (3 * len(base))), seed)
    out = {}
    for k, tg in enumerate(targets):
        ann = anneal(d, n_chains, iters, n_masks=256, mode=1, target=tg, seed=seed * 101 + k, start=list(starts),
                     scramble=16, extra_masks=sample)
        rows = ann.best.cpu().numpy()
        got = 0
        for t in np.argsort(-ann.best_score):
            if ann.best_score[t] <= 0 or got >= keep:
                break
            E = edges_of(d, rows[t])
            key = _canon_key(d, E)
            if key not in out and regular.is_regular(d, E):
                out[key] = E
                got += 1
    return out, targets


def iterate(d: int, pool, n_tris: int = 4096, walk_steps: int = 64, max_rounds: int = 8, seed: int = 0,
            symmetric: bool = True, capacity: int = 1 << 14, max_selected: int = 32, log=None,
            explore_chains: int = 256, explore_iters: int = 200, explore_masks: int = 2048,
            target_count=None, witness_mutants: int = 0, explore_tries: int = 1,
            target_chains: int = 0, target_iters: int = 150) -> IterateResult:
    """The witness <-> triangulation loop of Sec. 3 from an initial pool of
    triangulations.  Each round: (1) every (Z/2)^3 class of each selected
    triangulation is swept (its orbit-canonical member), one witness kept
    per new type; (2) n_tris triangulations generated by random
    (symmetric) walks from the selected and pool triangulations are judged
    against all witnesses; (3) those realising new types, once certified
    regular, are selected for the next round.  When a round adds nothing,
    an annealing run for novelty (``explore``) proposes the next selection
    (up to explore_tries runs); the loop stops when that finds nothing
    either, after max_rounds, or once target_count types are known.  With
    witness_mutants > 0 the second mode also judges that many mutants of
    every witness (1-3 flips each) against the generated triangulations.
    With target_chains > 0, a round without news whose novelty runs find
    nothing anneals toward the (p, n) pairs missing at the highest oval
    counts (``explore_targets``) before giving up."""
    found: dict = {}
    witnesses: list = []
    rounds = []
    selected = {}
    for E in pool:
        selected.setdefault(_canon_key(d, E), np.asarray(E))
    starts = list(selected.values())
    t_all = 0.0
    for r in range(max_rounds):
        info = {"round": r, "swept": len(selected)}
        t0 = time.perf_counter()
        new_from_sweeps = 0
        for E in list(selected.values())[:max_selected]:
            res = orbits.orbit_sweep(d, E, capacity=capacity, specialize=False)
            for code, (_, widx) in res.hist.items():
                if code in found:
                    continue
                m = res.class_mask(widx)
                found[code] = Realised(res.canonical_edges, m, True)
                witnesses.append(m)
                new_from_sweeps += 1
        t_sweep = time.perf_counter() - t0
        info["new_from_class_sweeps"] = new_from_sweeps
        wm = np.zeros((len(witnesses), 2), dtype=np.uint64)
        wm[:, 0] = [m & ((1 << 64) - 1) for m in witnesses]
        if witness_mutants:
            wm = np.concatenate([wm, mutants(d, wm, witness_mutants, seed * 31 + r)])
        # generated triangulations: walks from the triangulations met so far
        per = max(1, n_tris // max(1, len(starts)))
        torch = _torch()
        adj = torch.cat([replicate(d, E, per) for E in starts], 0)
        pw.flip_walk(d, adj, walk_steps, symmetric, seed * 1000 + r)
        m2 = mode2_sweep(d, wm, adj.shape[0], 0, 0, adj=adj, capacity=capacity)
        info["mode2_pairs"] = adj.shape[0] * len(wm)
        info["mode2_seconds"] = m2.gpu_seconds
        nxt = {}
        new_regular = 0
        for code, (_, gi) in m2.hist.items():
            if code in found:
                continue
            t, w = gi // m2.n_w, gi % m2.n_w
            E = edges_of(d, adj[t])
            if not regular.is_regular(d, E):
                continue
            found[code] = Realised(E, int(wm[w, 0]) | (int(wm[w, 1]) << 64), True)
            nxt.setdefault(_canon_key(d, E), E)
            new_regular += 1
        info["new_from_mode2"] = new_regular
        info["sweep_seconds"] = t_sweep
        info["distinct"] = len(found)
        t_all += time.perf_counter() - t0
        rounds.append(info)
        if log:
            log(info)
        if target_count is not None and len(found) >= target_count:
            break
        if not nxt and new_from_sweeps == 0:
            if not explore_chains:
                break
            t1 = time.perf_counter()
            for k in range(explore_tries):
                nxt, ann = explore(d, found, starts, explore_chains, explore_iters, explore_masks,
                                   seed * 7919 + r * 13 + k, witnesses=wm[:len(witnesses)])
                if nxt:
                    break
            info["explore_best"] = float(ann.best_score.max())
            if not nxt and target_chains:
                nxt, tried = explore_targets(d, found, starts, target_chains, target_iters, seed * 7 + r,
                                             wm[:len(witnesses)])
                info["targets_tried"] = len(tried)
            info["explore_seconds"] = time.perf_counter() - t1
            info["explore_selected"] = len(nxt)
            t_all += info["explore_seconds"]
            if not nxt:
                break
        selected = nxt
        starts = (starts + list(nxt.values()))[-64:]
    return IterateResult(d, found, rounds, t_all)


def scheme_text(code: int) -> str:
    """Display form of a scheme code (Rohlin-Viro style, display only):
    '<J + 1<2> + 5>'; k empty ovals side by side are written k."""
    bits = bin(code & ((1 << 127) - 1))[3:]
    pos = 0

    def forest():
        nonlocal pos
        kids = []
        while pos < len(bits) and bits[pos] == "1":
            pos += 1
            kids.append(forest())
            pos += 1  # the closing '0'
        return kids

    def fmt(f):
        empty = sum(1 for t in f if not t)
        parts, seen = [], {}
        for t in f:
            if t:
                k = fmt(t)
                seen[k] = seen.get(k, 0) + 1
        parts = [f"{n}<{k}>" for k, n in seen.items()]
        if empty:
            parts.append(str(empty))
        return " + ".join(parts) if parts else "0"

    body = fmt(forest())
    if code >> 127:
        body = "J" if body == "0" else "J + " + body
    return f"<{body}>"


def certify(d: int, res: IterateResult, check) -> int:
    """Re-evaluate every kept (triangulation, witness) with `check(d, edges,
    mask) -> code` and return how many agree."""
    return sum(check(d, r.edges, r.mask) == code for code, r in res.found.items())


__all__ = ["replicate", "edges_of", "mode2_sweep", "anneal", "iterate", "accept_table", "Mode2Result",
           "AnnealResult", "IterateResult", "math"]
