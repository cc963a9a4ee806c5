"""Autotuner of the build's speed knobs.

The knobs -- the cutover C below which a subarray is finished on-chip, the
number of workgroups of the persistent on-chip finish, how the level-0 rank
records are completed, the radix digit width and tile size of the presort,
(learned form) which sorts use the learned buckets, and (plain form) the
level form: k-1 arrays moved per level, one multi-level split per level, or
(k >= 5) deferred partitioning -- change speed only.  tune() times every candidate configuration on the caller's input, and
checks that each one returns exactly the output of the default
configuration (a difference would be a bug, and raises); the fastest is
cached per (form, k, dtype, log2 n) in a JSON file, from which
best_options() reads it back.  Timing uses HIP events on the build's stream.
"""
from __future__ import annotations

import json
import math
import os

DEFAULTS = {"cutover": 1024, "leaf_blocks": 2048, "records": 0}
CANDIDATES = [{"cutover": c, "leaf_blocks": b, "records": r} for c in (1024, 2048, 4096)
              for b in (1024, 2048, 4096) for r in (1, 2)]
# the learned form also chooses which sorts go through the learned buckets:
# all of them, or only the first (the multi-word sort, where the buckets save
# the most passes)
LEARNED_SORTS = (0, 1)
# level forms of a single tree: 4 (one multi-level split per level; the
# default from k = 3 on) and 1 (every level moves k-1 arrays); deferred partitioning (form 3) saves
# (k-1)(k-2)/2 array moves for the price of one radix split per array j >= 2,
# measured to lose at k <= 4, so only k >= 5 try it
LEVEL_FORMS = (4, 1)
DEFERRED_MIN_K = 5
# radix geometry: digit width (8 or 11 bits: four or three passes per key
# word) and keys per tile
DIGIT_BITS = (8, 11)
SORT_TILES = (4096, 8192)


def knob_values(form: str, k: int | None = None) -> dict:
    """The values every knob of a form may take (the first is its default)."""
    v = {"cutover": (1024, 2048, 4096), "leaf_blocks": (2048, 1024, 4096), "records": (0, 1, 2),
         "digit_bits": DIGIT_BITS, "sort_tile": SORT_TILES}
    if form == "plain":
        v["level"] = LEVEL_FORMS + ((3,) if k is not None and k >= DEFERRED_MIN_K else ())
    if form == "learned":
        v["learned_sorts"] = LEARNED_SORTS
    return v


def candidates_for(form: str, k: int | None = None) -> list:
    """Every combination of cutover, finish grid and record completion, with
    the form's own knob (learned sorts; level form of the plain form)."""
    if form == "learned":
        return [dict(c, learned_sorts=m) for c in CANDIDATES for m in LEARNED_SORTS]
    if form == "plain":
        levels = LEVEL_FORMS + ((3,) if k is not None and k >= DEFERRED_MIN_K else ())
        return [dict(c, level=lv) for lv in levels for c in CANDIDATES]
    return list(CANDIDATES)


def cache_path() -> str:
    return os.environ.get("KD_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1410_5420_amd",
                                       "tune.json"))


def cache_key(form: str, n: int, k: int, dtype: str) -> str:
    """Inputs of similar size share an entry: n is bucketed by log2."""
    return f"{form}|k={k}|{dtype}|log2n={int(round(math.log2(max(n, 1))))}"


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(entries: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def best_options(form: str, n: int, k: int, dtype: str, path: str | None = None) -> dict:
    """The cached best configuration, or the defaults."""
    e = load(path).get(cache_key(form, n, k, dtype))
    return dict(e["config"]) if e else dict(DEFAULTS)


def select(results: list) -> dict:
    """The fastest of [{"config": ..., "ms": ...}], ties to the earlier one."""
    if not results:
        raise ValueError("no candidate was timed")
    return min(results, key=lambda r: r["ms"])


def coordinate_order(form: str, k: int | None = None) -> list:
    """The knobs in the order coordinate descent sweeps them."""
    order = ["level", "cutover", "leaf_blocks", "records", "digit_bits", "sort_tile",
             "learned_sorts"]
    vals = knob_values(form, k)
    return [(name, vals[name]) for name in order if name in vals]


def tune(tuples, form: str = "plain", offsets=None, models=None, candidates=None, reps: int = 5,
         warmup: int = 1, path: str | None = None, record: bool = True,
         strategy: str = "coordinate") -> dict:
    """Time configurations on ``tuples`` (a device tensor) and cache the
    fastest.  form: "plain", "learned" (needs ``models``) or "batched" (needs
    ``offsets``).  With ``candidates`` (a list of configurations) every one
    is timed; otherwise strategy "coordinate" sweeps one knob at a time from
    the defaults, keeping the best value found so far (knob_values), and
    "exhaustive" times candidates_for(form).  Every configuration's output
    must equal the default's.  Returns {"config", "ms", "results"}."""
    import torch

    from . import BatchedBuilder, Builder, LearnedBuilder

    n, k = tuples.shape
    dev = tuples.device
    dtype = str(tuples.dtype).replace("torch.", "")

    def make(cfg):
        if form == "plain":
            b = Builder(max(n, 1), k, tuples.dtype, dev, **cfg)
            return b, lambda perm: b.build(tuples, perm)
        if form == "learned":
            b = LearnedBuilder(max(n, 1), k, tuples.dtype, dev, **cfg)
            return b, lambda perm: b.build(tuples, perm, models=models)
        if form == "batched":
            b = BatchedBuilder(offsets, k, tuples.dtype, dev, **cfg)
            return b, lambda perm: b.build(tuples, perm)
        raise ValueError(form)

    ref_builder, run = make(dict(DEFAULTS))
    ref = torch.full((max(n, 1),), -1, dtype=torch.int32, device=dev)
    run(ref)
    torch.cuda.synchronize()
    ref_nu = ref_builder.n_unique.clone()
    del ref_builder

    results = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_cfg(cfg):
        b, run = make(dict(cfg))
        perm = torch.full_like(ref, -1)
        for _ in range(warmup):
            run(perm)
        torch.cuda.synchronize()
        if not (torch.equal(perm, ref) and torch.equal(b.n_unique, ref_nu)):
            raise RuntimeError(f"configuration {cfg} changed the output: the knobs must not")
        times = []
        for _ in range(reps):
            ev0.record()
            run(perm)
            ev1.record()
            torch.cuda.synchronize()
            times.append(ev0.elapsed_time(ev1))
        times.sort()
        res = {"config": dict(cfg), "ms": times[len(times) // 2]}
        results.append(res)
        del b
        return res

    if candidates is not None or strategy == "exhaustive":
        for cfg in candidates or candidates_for(form, k):
            time_cfg(cfg)
        best = select(results)
    elif strategy == "coordinate":
        cur = {name: vals[0] for name, vals in coordinate_order(form, k)}
        best = time_cfg(cur)
        for name, vals in coordinate_order(form, k):
            for v in vals:
                if v == best["config"][name]:
                    continue
                r = time_cfg(dict(best["config"], **{name: v}))
                if r["ms"] < best["ms"]:
                    best = r
    else:
        raise ValueError(strategy)
    if record:
        entries = load(path)
        entries[cache_key(form, n, k, dtype)] = {"config": best["config"], "ms": best["ms"]}
        save(entries, path)
    return {"config": best["config"], "ms": best["ms"], "results": results}
