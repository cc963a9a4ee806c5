"""Benchmark: balanced k-d tree build throughput on one MI355X.

Headline workload: k = 3, n = 2^24 int32 tuples uniform over the full signed
range with 0.1% exact copies, one tree.  A step is one whole build -- presort
by the three cyclic super keys, duplicate removal and the level-by-level
partition -- with the tuples already resident in HBM and a preallocated
workspace.  value = n / (time per step), in tuples/s.

Beside it (all on the same GPU, all bit-exact against the plain build):
  * presort and partition phase times, and per-kernel-class time per step
    (HIP events the library records around its own launches);
  * the roofline of the dominant kernel class: algorithmic bytes per launch
    over its average launch time, with HBM traffic from profiler counters
    when they were taken for the current kernel sources;
  * the learned-presort form on the headline input and on the 2^26 float32
    Gaussian mixture, against the plain build on the same inputs;
  * the batched form on 4096 point-cloud trees, against a host loop of plain
    builds and as a replayed HIP graph;
  * the CPU oracle timed on the host.

Prints exactly one JSON line.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tuples/sec k-d build (k=3, n=2^24, bit-exact) plain vs batched/learned; % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---- algorithmic byte model ----------------------------------------------------------

def onesweep_bytes(n: int, nu: int, k: int):
    """(total algorithmic bytes, launches) of all radix passes of one plain
    build (each pass counts as one launch of the class).  Array 0 is sorted
    over all n rows by its first word alone (k > 1): every pass moves that
    key word and k payload words (the row id, made by the first pass, and the
    other key words), read from the planes the rows were canonicalised into.  The
    complete word-by-word sort of array 0 is also enqueued, gated on the tie
    step's flag: its k * 4 passes move nothing unless a run of equal first
    words is too long, and count as launches of no bytes.  Each of the k-1
    chain sorts runs over the n_unique rows and moves its key word and k-1
    payload words (the ranks known so far, the first made by its first pass
    as the input position, and the key words of the later sorts); its last
    pass drops the key.  Every word read or written counts 4 bytes."""
    P = 4  # 8-bit digit passes per 32-bit word
    words = 0
    launches = 0
    if k > 1:
        for ps in range(P):
            words += n * ((k if ps == 0 else k + 1) + (k + 1))
        launches += P + k * P
    else:
        for ps in range(P):
            words += n * ((1 if ps == 0 else 2) + 2)
        launches += P
    for _ in range(k - 1, 0, -1):
        for ps in range(P):
            words += nu * ((k - 1 if ps == 0 else k) + (k - 1 if ps == P - 1 else k))
        launches += P
    return 4 * words, launches


def level_write_masks(k: int, levels: int):
    """The planes each level's move writes (per array), walking back from the
    on-chip finish exactly as the library does: later levels and the finish
    read, of a split array p, plane 0 and (p != 0) its order-0 plane; of a
    moving array, the side-deciding plane and every plane it writes; the
    finish reads the order-0 plane of arrays 1 .. k-1."""
    need = [0] * k
    for j in range(1, k):
        need[j] = 1 << (k - 1 - j)
    masks = [None] * levels
    for d in range(levels - 1, -1, -1):
        p = d % k
        masks[d] = {j: need[j] for j in range(k) if j != p}
        for j in range(k):
            if j == p:
                need[j] |= 1
                if p != 0:
                    need[j] |= 1 << ((k - p - 1) % k)
            elif need[j]:
                need[j] |= 1 << ((p - j - 1 + 2 * k) % k)
    return masks


def level_bytes(nu: int, k: int, cutover: int):
    """(total algorithmic bytes, launches) of the global partition levels:
    every moving array reads the plane that decides the side and the planes
    it moves, and writes the planes later levels or the on-chip finish read
    (all k-1 rank planes except near the end; row ids stay in the level-0
    records)."""
    levels = 0
    while (nu >> levels) > cutover:
        levels += 1
    total = 0
    for d, m in enumerate(level_write_masks(k, levels)):
        p = d % k
        for j, w in m.items():
            if not w:
                continue
            cp = (p - j - 1 + 2 * k) % k
            total += nu * 4 * (bin(w | (1 << cp)).count("1") + bin(w).count("1"))
    return total, levels


# The byte model fixed before measuring (the scope's measurement section):
# per tuple, a word-sort of the chain presort moves 8 + 16 (P - 1) + 12 bytes
# over its P = 4 digit passes (17 B per pass on average), a global level moves
# 5 + 9 (k - 1) bytes (a side-flag design: the split array's index read and
# flag write, each other array's index read, flag gather and index write), and
# the whole build at k = 3, n = 2^24 (r = 8, C = 4096) moves 672 B per tuple.
SURVEY_PASS_BYTES = 17
SURVEY_WHOLE_BUILD_BYTES_PER_TUPLE = 672


def survey_level_bytes(k: int) -> int:
    return 5 + 9 * (k - 1)


def survey_whole_build_bytes(n: int, k: int, nu: int) -> int:
    """B_model of the whole build, P = 4, C = 4096: chain presort (2k - 1)
    word-sorts of 68 B, duplicate removal 8 + 4k, ceil(log2(n_u / 4096))
    levels of 5 + 9 (k - 1), the on-chip finish and emission 8k + 12 (672 B
    per tuple at k = 3, n = 2^24)."""
    levels = 0
    while (nu >> levels) > 4096:
        levels += 1
    per = (2 * k - 1) * 68 + (8 + 4 * k) + levels * survey_level_bytes(k) + (8 * k + 12)
    return per * n


def survey_bytes_per_launch(kernel: str, n: int, nu: int, k: int, cutover: int):
    """(algorithmic bytes per launch, description) under the fixed model:
    a level moves n_u tuples, a radix pass 17 B per row it sorts (word 0
    passes over n rows, the chain's over n_u; gated passes count as launches
    of no bytes, as in the design model)."""
    if kernel == "level":
        return survey_level_bytes(k) * nu, f"{survey_level_bytes(k)} B x n_unique per level (5 + 9(k-1))"
    if kernel == "onesweep":
        _, launches = onesweep_bytes(n, nu, k)
        P = 4
        rows = P * n + (k - 1) * P * nu if k > 1 else P * n
        return SURVEY_PASS_BYTES * rows / launches, (f"17 B per sorted row per pass over the "
                                                     f"{launches} passes, averaged")
    if kernel == "leaf":
        return (8 * k + 12) * nu, f"{8 * k + 12} B x n_unique (8k + 12)"
    raise ValueError(kernel)


def roll_depth(L: int, j: int, k: int) -> int:
    return j + k * ((L - 1 - j) // k) + 1 if L > j else 0


def split_bytes(nu: int, k: int, cutover: int):
    """(total algorithmic bytes, levels) of level form 4: at level L >= 1 the
    array L mod k splits from its last layout to depth L; its count reads
    the planes the walk compares and writes a key per element (1 byte, 2 at
    k = 8), its move reads the key and the planes it writes and writes them
    (write masks from the library's own plan); after the last level the
    arrays the on-chip finish reads split to its depth."""
    from paper_1410_5420_amd import _lib

    levels = 0
    while (nu >> levels) > cutover:
        levels += 1
    lm, fm = _lib.level_plan(k, levels) if k > 1 else ([], [])
    kb = 2 if k >= 8 else 1

    def one(q, frm, to, mask):
        deciding = {((l % k) - q - 1 + 2 * k) % k for l in range(frm, to)}
        w = bin(mask).count("1")
        return nu * (4 * len(deciding) + kb + kb + 8 * w)

    total = 0
    for L in range(1, levels):
        q = L % k
        total += one(q, roll_depth(L, q, k), L, lm[L])
    for j in range(1, k):
        a = roll_depth(levels, j, k)
        if levels >= 1 and a < levels:
            total += one(j, a, levels, fm[j])
    return total, levels


def byte_model(kernel: str, n: int, nu: int, k: int, cutover: int, level_form: int = 1):
    """Algorithmic bytes of one launch of a kernel class (averaged over the
    build's launches of that class; a global level counts as one launch),
    and how they arise."""
    if kernel == "level" and level_form == 4:
        total, levels = split_bytes(nu, k, cutover)
        return total / max(levels, 1), (f"{levels} levels, one multi-level split per level: count "
                                        f"reads the compared rank planes and writes a key, move reads "
                                        f"the key and moves the written planes (library's write masks)")
    if kernel == "level":
        total, launches = level_bytes(nu, k, cutover)
        return total / max(launches, 1), (f"{launches} levels: per level (k-1) arrays x (k-1) ranks "
                                          f"x 4 B, read + write, x n_unique; near the end only the "
                                          f"planes later levels and the on-chip finish read")
    if kernel == "onesweep":
        total, launches = onesweep_bytes(n, nu, k)
        return total / launches, f"radix key + payload words of the build's {launches} passes, averaged"
    if kernel == "leaf":
        per_unit = 4 * k + 4  # order-0 rank of k-1 arrays + row id in, perm out
        return per_unit * nu, f"{per_unit} B x n_unique elements"
    raise ValueError(kernel)


# ---- profiler traffic ------------------------------------------------------------------

def source_digest() -> str:
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1410_5420_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch from a committed counter summary, if it was taken
    for the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"source digest:\s*`?([0-9a-f]+)", text)
    m_val = re.search(r"traffic bytes per launch:\s*([0-9]+)", text)
    if not m_sha or not m_val or m_sha.group(1) != source_digest():
        return None
    return int(m_val.group(1))


# ---- CPU baseline -------------------------------------------------------------------

def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(t: np.ndarray):
    """The oracle as it stands, median of 3 runs in each of two modes: one
    thread on a bounded sample (the first quarter of the rows), and q =
    2^floor(log2 nproc) threads (the paper's parent/child scheme allows only
    powers of two) on the whole input, nproc capped at the 16 CPUs a GPU's
    share of the host provides."""
    import oracle

    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = min(16, nproc)
    q = 1
    while q * 2 <= cores:
        q *= 2

    def median_rate(x, threads):
        runs = []
        for _ in range(3):
            t0 = time.perf_counter()
            r = oracle.build_tree(x, threads=threads, children=False)
            runs.append((time.perf_counter() - t0, r["times"]))
        runs.sort(key=lambda v: v[0])
        dt, times = runs[1]
        return x.shape[0] / dt, dt, times

    sample = t[: t.shape[0] // 4]
    r1, d1, t1 = median_rate(sample, 1)
    rq, dq, tq = median_rate(t, q)
    return {"value": round(rq, 1), "unit": "tuples/s", "cores": q, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": nproc,
            "one_thread": {"value": round(r1, 1), "unit": "tuples/s", "cores": 1,
                           "rows": int(sample.shape[0]), "median_s": round(d1, 3),
                           "presort_s": round(t1[0], 3), "partition_s": round(t1[1], 3)},
            "sample": f"median of 3 whole builds of the same {t.shape[0]}-row input at q={q} threads "
                      f"({dq:.2f} s; presort {tq[0]:.2f} s, partition {tq[1]:.2f} s; paper's parent/"
                      f"child threads); one_thread: median of 3 builds of its first "
                      f"{sample.shape[0]} rows on one thread ({d1:.2f} s)"}


# ---- timing helpers ----------------------------------------------------------------

def time_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cutover", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the learned and batched forms")
    ap.add_argument("--no-tune", action="store_true", help="use the default knobs instead of autotuning")
    ap.add_argument("--knobs", type=str, default=None,
                    help="JSON object of build knobs for the plain build (no autotuning), e.g. the "
                         "config a tuned run reported, so a profiled run repeats it")
    ap.add_argument("--no-queries", action="store_true", help="skip the tree searches on the C2 tree")
    ap.add_argument("--no-select", action="store_true",
                    help="skip the comparison builder's k sweep on the C3 inputs")
    ap.add_argument("--n", type=int, default=1 << 24, help=argparse.SUPPRESS)
    ap.add_argument("--calibrate", action="store_true",
                    help="first run one plain 256 MiB device copy (a reference for profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the build runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    import kdgen
    import paper_1410_5420_amd as kd
    from paper_1410_5420_amd import _lib

    n, k = args.n, 3
    log(f"generating n={n} k={k}")
    t_host = kdgen.c2_full_range(n)
    dev = torch.device("cuda:0")
    t = torch.from_numpy(t_host).to(dev)
    tuned = None
    if args.cutover:
        knobs = {"cutover": args.cutover, "leaf_blocks": None, "records": None}
    elif args.knobs:
        knobs = {"cutover": None, "leaf_blocks": None, "records": None}
        knobs.update(json.loads(args.knobs))
    elif args.no_tune:
        knobs = {"cutover": None, "leaf_blocks": None, "records": None}
    else:
        from paper_1410_5420_amd import autotune

        log("autotuning the knobs on this input")
        tuned = autotune.tune(t, "plain", reps=3, record=False)
        knobs = dict(tuned["config"])
    cutover = knobs["cutover"] or 1024
    level_form = knobs.get("level") or 4  # the library's default for one tree of k >= 3
    b = kd.Builder(n, k, torch.int32, dev, **knobs)
    perm = torch.full((n,), -1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    if args.calibrate:
        ref = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        ref.fill_(1)
        _ = ref.clone()
        torch.cuda.synchronize()
        del ref, _
    for _ in range(args.warmup):
        b.build(t, perm)
    torch.cuda.synchronize()
    nu = int(b.n_unique.item())
    log(f"warmup done, n_unique={nu}")

    # timed region: K whole builds, nothing else enqueued between them
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.build(t, perm)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    log(f"{args.steps} steps, {ms_per_step:.3f} ms/step")
    b.status()  # raises if a kernel reported inconsistent counts

    # every kernel class over its own (untimed) builds: the library records
    # HIP events around that class's launches on the build's stream
    durations = {}
    for cls in ("level", "onesweep", "leaf", "records", "dedup"):
        reps = max(3, args.steps // 4)
        c2 = 64 * reps
        _lib.probe_start(cls, c2)
        for _ in range(reps):
            b.build(t, perm)
        torch.cuda.synchronize()
        durations[cls] = _lib.probe_stop(c2)
        durations[cls + "_reps"] = reps
    class_ms = {}
    for cls in ("level", "onesweep", "leaf", "records", "dedup"):
        class_ms[cls] = round(float(np.sum(durations[cls])) / durations[cls + "_reps"], 4)

    # phase split, measured separately with events on the same stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    pre_ms, part_ms = [], []
    for _ in range(max(3, args.steps // 2)):
        ev[0].record(stream)
        b.presort(t)
        ev[1].record(stream)
        b.partition(t, perm)
        ev[2].record(stream)
        torch.cuda.synchronize()
        pre_ms.append(ev[0].elapsed_time(ev[1]))
        part_ms.append(ev[1].elapsed_time(ev[2]))

    levels = 0
    while (nu >> levels) > cutover:
        levels += 1

    def roofline_of(cls):
        # achieved: the fixed model's algorithmic bytes per launch over the
        # class's average launch time; the design's own byte model beside it.
        # A global level is one launch of the level class: its time is the
        # class's time per build over the levels (the library records its
        # launch groups separately, two or three per level).
        bytes_per_launch, unit_desc = survey_bytes_per_launch(cls, n, nu, k, cutover)
        design_bytes, design_desc = byte_model(cls, n, nu, k, cutover, level_form)
        real = [d for d in durations[cls] if d > 0.002]  # no-op launches (levels past the cutover) excluded
        avg_ms = float(np.mean(real)) if real else float("nan")
        if cls == "level":
            avg_ms = class_ms["level"] / max(levels, 1)
            real = [0] * levels
        achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        design_achieved = design_bytes / (avg_ms * 1e-3) / 1e9
        traffic = recorded_traffic(cls, "c2")
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": cls,
                "avg_launch_ms": round(avg_ms, 4), "launches": len(real),
                "bytes_per_launch": int(bytes_per_launch), "byte_model": unit_desc,
                "design_model": {"bytes_per_launch": int(design_bytes), "byte_model": design_desc,
                                 "achieved": round(design_achieved, 1),
                                 "frac": round(design_achieved / HBM_PEAK_GBS, 4)}}

    B_model = survey_whole_build_bytes(n, k, nu)
    wb_gbs = B_model / (ms_per_step * 1e-3) / 1e9
    whole_build = {"bytes_per_tuple": round(B_model / n, 1), "B_model": int(B_model),
                   "ms_per_step": round(ms_per_step, 4), "achieved": round(wb_gbs, 1),
                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(wb_gbs / HBM_PEAK_GBS, 4),
                   "bar": 0.40,
                   "byte_model": "fixed before measuring: chain presort (2k-1) x 68 B, dedup 8 + 4k, "
                                 "ceil(log2(n_u/4096)) levels x (5 + 9(k-1)), finish 8k + 12 "
                                 "(672 B per tuple at k = 3, n = 2^24)"}
    log(f"whole build: {B_model / 1e9:.2f} GB model bytes in {ms_per_step:.3f} ms = "
        f"{wb_gbs / HBM_PEAK_GBS:.3f} of HBM peak")
    dominant = max(("level", "onesweep"), key=lambda c: class_ms[c])
    roofline = roofline_of(dominant)
    secondary = roofline_of("onesweep" if dominant == "level" else "level")

    out = {
        "metric": METRIC,
        "value": round(n / (ms_per_step * 1e-3), 1),
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "k=3, n=2^24 int32 uniform over the full signed range, 0.1% exact "
                               "copies (seeded); one plain build (presort + dedup + partition)",
                   "k": k, "n": n, "n_unique": nu, "tuple_dtype": "int32", "cutover": cutover,
                   "leaf_blocks": knobs["leaf_blocks"] or 2048,
                   "records": knobs["records"] or 0,
                   "level_form": level_form,
                   "digit_bits": knobs.get("digit_bits") or 8,
                   "sort_tile": knobs.get("sort_tile") or 4096,
                   "autotuned": tuned is not None,
                   "presort_ms": round(float(np.median(pre_ms)), 4),
                   "partition_ms": round(float(np.median(part_ms)), 4),
                   "kernel_class_ms_per_step": class_ms},
        "roofline": roofline,
        "roofline_secondary": secondary,
        "whole_build": whole_build,
    }

    if not args.no_queries:
        out["queries"] = queries_c2(torch, kd, _lib, kdgen, t, t_host, perm, b.n_unique, nu, args)

    if not args.no_select:
        out["select_c3"] = select_c3(torch, kd, kdgen, args)

    if not args.no_forms:
        plain_perm = perm.clone()
        out["forms"] = {"learned_c2": learned_form(torch, kd, t, plain_perm, nu, args, "c2 (same input)",
                                                   knobs),
                        "deferred_c2": deferred_form(torch, kd, t, plain_perm, nu, args, knobs)}
        del b, t, perm, plain_perm
        torch.cuda.empty_cache()
        out["forms"]["learned_c5"] = learned_c5(torch, kd, kdgen, args)
        torch.cuda.empty_cache()
        out["forms"]["batched_c4"] = batched_c4(torch, kd, kdgen, args)
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(t_host)
    print(json.dumps(out), flush=True)


def queries_c2(torch, kd, _lib, kdgen, t, t_host, perm, n_nodes, nu, args):
    """Batched searches over the C2 tree just built: 2^20 nearest-neighbour
    queries (m = 8) and 2^20 box counts over the node coordinates gathered
    once into tree-position order, each kernel timed over its launches with
    the library's probe (HIP events on the launch stream).  Bytes: every
    visited node reads its coordinates (4k B); the visits are counted by the
    kernels.  The CPU oracle runs a sample of the same queries."""
    n, k = t.shape
    nq = 1 << 20
    pts, lo, hi = kdgen.c2_queries(t_host, nq)
    dp, dlo, dhi = (torch.from_numpy(a).to(t.device) for a in (pts, lo, hi))
    reps = 5
    res = {"workload": "C2 tree (k=3, 2^24 int32 rows); 2^20 points within 1000 of a random row "
                       "(m = 8 nearest) and 2^20 boxes of half-width 2^26 around random rows"}
    visits = torch.zeros(1, dtype=torch.int64, device=t.device)
    _lib.probe_start("query", 1)
    nodes = kd.gather_nodes(t, perm, n_nodes)
    torch.cuda.synchronize()
    res["gather_nodes_ms"] = round(float(_lib.probe_stop(1)[0]), 4)
    _lib.probe_start("query", 1)
    bounds = kd.subtree_bounds(nodes, n_nodes)
    torch.cuda.synchronize()
    res["subtree_bounds_ms"] = round(float(np.sum(_lib.probe_stop(1))), 4)
    runs = {"nearest_m8": lambda v: kd.nearest(t, perm, n_nodes, dp, 8, visits=v, nodes=nodes),
            "box_count": lambda v: kd.region_count(t, perm, n_nodes, dlo, dhi, visits=v, nodes=nodes,
                                                   bounds=bounds),
            "box_count_no_bounds": lambda v: kd.region_count(t, perm, n_nodes, dlo, dhi, visits=v,
                                                             nodes=nodes)}
    outs = {}
    for name, fn in runs.items():
        fn(None)
        visits.zero_()
        outs[name] = fn(visits)
        torch.cuda.synchronize()
        per_query = int(visits.item()) / nq
        _lib.probe_start("query", reps)
        for _ in range(reps):
            fn(None)
        torch.cuda.synchronize()
        ms = float(np.mean(_lib.probe_stop(reps)))
        gbs = per_query * nq * (4 * k) / (ms * 1e-3) / 1e9
        res[name] = {"ms_per_batch": round(ms, 4), "queries_per_s": round(nq / (ms * 1e-3), 1),
                     "visits_per_query": round(per_query, 2), "node_bytes_gbs": round(gbs, 1),
                     "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"queries {name}: {ms:.3f} ms per 2^20, {per_query:.1f} visits per query")
    res["box_mean_count"] = round(float(outs["box_count"].float().mean().item()), 2)
    res["box_bounds_same_counts"] = bool(torch.equal(outs["box_count"], outs["box_count_no_bounds"]))
    # every node as a query (m = 8, itself excluded), then the reverse lists
    visits.zero_()
    _lib.probe_start("query", 1)
    near = kd.all_nearest(t, perm, n_nodes, 8, visits=visits, nodes=nodes)
    torch.cuda.synchronize()
    all_ms = float(_lib.probe_stop(1)[0])
    all_visits = int(visits.item()) / nu
    _lib.probe_start("query", 1)
    offs, _lists = kd.reverse_nearest(perm, n_nodes, near)
    torch.cuda.synchronize()
    rev_ms = float(_lib.probe_stop(1)[0])
    res["all_nearest_m8"] = {"ms": round(all_ms, 3), "nodes_per_s": round(nu / (all_ms * 1e-3), 1),
                             "visits_per_query": round(all_visits, 2)}
    res["reverse_lists"] = {"ms": round(rev_ms, 3), "entries": int(offs[-1].item())}
    log(f"queries all nearest: {all_ms:.2f} ms over {nu} nodes; reverse lists {rev_ms:.2f} ms")
    del near, offs, _lists
    # spot check against the oracle on a few queries
    from oracle import queries as oq

    p = perm[:nu].cpu().numpy()
    nn_rows = outs["nearest_m8"].cpu().numpy()
    counts = outs["box_count"].cpu().numpy()
    ok = True
    for q in range(4):
        od = [d for d, _ in oq.nearest_neighbors(t_host, p, [int(v) for v in pts[q]], 8)]
        x = t_host[nn_rows[q]].astype(object)
        gd = [sum((int(a) - int(b)) ** 2 for a, b in zip(r, pts[q])) for r in x]
        ok = ok and od == gd
        ok = ok and len(oq.region_search(t_host, p, lo[q].tolist(), hi[q].tolist())) == counts[q]
    res["spot_check_vs_oracle"] = bool(ok)
    if not args.no_cpu:
        # the oracle as it stands, on a sample of the same queries
        t0 = time.perf_counter()
        s_nn = 2000
        for q in range(s_nn):
            oq.nearest_neighbors(t_host, p, [int(v) for v in pts[q]], 8)
        nn_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        s_box = 200
        for q in range(s_box):
            oq.region_search(t_host, p, lo[q].tolist(), hi[q].tolist())
        box_s = time.perf_counter() - t0
        res["cpu_baseline"] = {"kind": "oracle", "cores": 1,
                               "nearest_m8_queries_per_s": round(s_nn / nn_s, 1),
                               "box_count_queries_per_s": round(s_box / box_s, 1),
                               "sample": f"the first {s_nn} points and {s_box} boxes of the same "
                                         f"batches ({nn_s + box_s:.1f} s, one Python thread)"}
        log(f"queries cpu oracle: {s_nn / nn_s:.0f} nn/s, {s_box / box_s:.0f} boxes/s")
    return res


def select_c3(torch, kd, kdgen, args):
    """The paper's comparison (its Fig. 7 varies k): the presort builder
    against the comparison builder (per-level median selection) on the C3
    inputs (n = 2^22, 256 Gaussian clusters, 10% copies) for k in
    {2, 3, 4, 6, 8}, and the presort builder with deferred partitioning
    (level form 3); all produce the same tree, checked here."""
    res = {"workload": "C3: k in {2,3,4,6,8}, n=2^22 int32 from 256 Gaussian clusters "
                       "(sigma 2^12), 10% exact copies", "per_k": {}}
    reps = max(3, args.steps // 4)
    for k in (2, 3, 4, 6, 8):
        x = kdgen.c3_clustered(k)
        t = torch.from_numpy(x).cuda()
        n = t.shape[0]
        b = kd.Builder(n, k, torch.int32)
        db = kd.Builder(n, k, torch.int32, level=3)
        sb = kd.SelectBuilder(n, k, torch.int32)
        p1 = torch.full((n,), -1, dtype=torch.int32, device=t.device)
        p2 = torch.full((n,), -1, dtype=torch.int32, device=t.device)
        p3 = torch.full((n,), -1, dtype=torch.int32, device=t.device)
        plain_ms = time_steps(torch, lambda: b.build(t, p1), reps, 1)
        def_ms = time_steps(torch, lambda: db.build(t, p3), reps, 1)
        sel_ms = time_steps(torch, lambda: sb.build(t, p2), reps, 1)
        nu = int(b.n_unique.item())
        same = int(sb.n_unique.item()) == nu and torch.equal(p1[:nu], p2[:nu])
        dsame = int(db.n_unique.item()) == nu and torch.equal(p1[:nu], p3[:nu])
        res["per_k"][str(k)] = {"presort_builder_ms": round(plain_ms, 3),
                                "deferred_partitioning_ms": round(def_ms, 3),
                                "select_builder_ms": round(sel_ms, 3),
                                "ratio": round(sel_ms / plain_ms, 2),
                                "same_tree": bool(same and dsame)}
        log(f"c3 k={k}: presort builder {plain_ms:.2f} ms, deferred partitioning {def_ms:.2f} ms, "
            f"per-level selection builder {sel_ms:.2f} ms, same={same} {dsame}")
        del b, db, sb, p1, p2, p3, t
        torch.cuda.empty_cache()
    return res


def deferred_form(torch, kd, t, plain_perm, nu, args, knobs):
    """Deferred partitioning (level form 3) on the same input: build time and
    equality with the plain perm."""
    n, k = t.shape
    kn = {key: v for key, v in knobs.items() if key != "level"}
    db = kd.Builder(n, k, t.dtype, level=3, **kn)
    perm = torch.full((n,), -1, dtype=torch.int32, device=t.device)
    ms = time_steps(torch, lambda: db.build(t, perm), max(5, args.steps // 2), 2)
    same = int(db.n_unique.item()) == nu and torch.equal(perm[:nu], plain_perm[:nu])
    log(f"deferred partitioning c2: {ms:.3f} ms, same={same}")
    return {"workload": "c2 (same input)", "build_ms": round(ms, 3), "same_tree": bool(same)}


def learned_form(torch, kd, t, plain_perm, nu, args, label, knobs=None):
    """Learned build on an input already built plainly: training time, build
    time, fallbacks, equality with the plain perm."""
    n, k = t.shape
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    models = kd.train_cdf(t)
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - t0) * 1e3
    knobs = dict(knobs or {})
    if not args.no_tune:
        from paper_1410_5420_amd import autotune

        cands = [dict(knobs, learned_sorts=m) for m in autotune.LEARNED_SORTS]
        knobs = autotune.tune(t, "learned", models=models, candidates=cands, reps=3,
                              record=False)["config"]
    lb = kd.LearnedBuilder(n, k, t.dtype, **knobs)
    perm = torch.full((n,), -1, dtype=torch.int32, device=t.device)
    ms = time_steps(torch, lambda: lb.build(t, perm, models=models), max(3, args.steps // 2), 2)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    pre = []
    for _ in range(3):
        ev[0].record()
        lb.presort(t, models=models)
        ev[1].record()
        torch.cuda.synchronize()
        pre.append(ev[0].elapsed_time(ev[1]))
    lb.build(t, perm, models=models)
    torch.cuda.synchronize()
    same = int(lb.n_unique.item()) == nu and torch.equal(perm[:nu], plain_perm[:nu])
    res = {"workload": label, "n": n, "knobs": knobs, "train_ms": round(train_ms, 3),
           "ms_per_build": round(ms, 4),
           "ms_per_build_with_training": round(ms + train_ms, 4),
           "tuples_per_s": round(n / (ms * 1e-3), 1), "presort_ms": round(float(np.median(pre)), 4),
           "fell_back": lb.fell_back.cpu().numpy().tolist(), "bit_exact_vs_plain": bool(same)}
    log(f"learned {label}: {ms:.3f} ms/build, presort {res['presort_ms']} ms, fell_back {res['fell_back']}")
    return res


def learned_c5(torch, kd, kdgen, args):
    log("generating the 2^26 float32 mixture")
    x = kdgen.c5_mixture()
    t = torch.from_numpy(x).cuda()
    del x
    n, k = t.shape
    knobs = {}
    if not args.no_tune:
        from paper_1410_5420_amd import autotune

        knobs = autotune.tune(t, "plain", reps=2, record=False)["config"]
        log(f"c5 plain knobs {knobs}")
    b = kd.Builder(n, k, torch.float32, **knobs)
    perm = torch.full((n,), -1, dtype=torch.int32, device=t.device)
    reps = max(3, args.steps // 4)
    plain_ms = time_steps(torch, lambda: b.build(t, perm), reps, 2)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    pre = []
    for _ in range(3):
        ev[0].record()
        b.presort(t)
        ev[1].record()
        torch.cuda.synchronize()
        pre.append(ev[0].elapsed_time(ev[1]))
    nu = int(b.n_unique.item())
    del b
    torch.cuda.empty_cache()
    res = learned_form(torch, kd, t, perm, nu, args, "k=3, n=2^26 float32 mixture of 64 anisotropic Gaussians",
                       knobs)
    res["plain_knobs"] = knobs
    res["plain_ms_per_build"] = round(plain_ms, 4)
    res["plain_presort_ms"] = round(float(np.median(pre)), 4)
    res["speedup_vs_plain"] = round(plain_ms / res["ms_per_build"], 3)
    res["speedup_vs_plain_with_training"] = round(plain_ms / res["ms_per_build_with_training"], 3)
    log(f"c5 plain {plain_ms:.3f} ms, learned {res['ms_per_build']} ms "
        f"({res['ms_per_build_with_training']} ms with training)")
    res["reuse"] = learned_reuse(torch, kd, kdgen, t, knobs, res["knobs"], args)
    return res


def learned_reuse(torch, kd, kdgen, t_a, plain_knobs, learned_knobs, args):
    """The learned form as it is meant to be used: a model trained once, on
    draw A of the mixture, then reused for a build of draw B (same
    distribution, other rows), against the plain build of draw B.  Both
    builds are timed alternately, reps each, and the spread is reported."""
    log("reuse: model trained on draw A, builds of draw B")
    models = kd.train_cdf(t_a)
    torch.cuda.synchronize()
    xb = kdgen.c5_mixture(draw=1)
    tb = torch.from_numpy(xb).cuda()
    del xb
    n, k = tb.shape
    b = kd.Builder(n, k, torch.float32, **plain_knobs)
    lb = kd.LearnedBuilder(n, k, torch.float32, **learned_knobs)
    pp = torch.full((n,), -1, dtype=torch.int32, device=tb.device)
    pl = torch.full((n,), -1, dtype=torch.int32, device=tb.device)
    for _ in range(2):
        b.build(tb, pp)
        lb.build(tb, pl, models=models)
    torch.cuda.synchronize()
    plain, learned = [], []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for _ in range(max(5, args.steps // 2)):
        for builder, out, times, kw in ((b, pp, plain, {}), (lb, pl, learned, {"models": models})):
            ev[0].record()
            builder.build(tb, out, **kw)
            ev[1].record()
            torch.cuda.synchronize()
            times.append(ev[0].elapsed_time(ev[1]))
    nu = int(b.n_unique.item())
    same = int(lb.n_unique.item()) == nu and torch.equal(pp[:nu], pl[:nu])
    b.status()
    lb.status()
    fb = lb.fell_back.cpu().numpy().tolist()
    res = {"workload": "model trained on draw A of the C5 mixture, builds of draw B (same mixture, "
                       "other rows)",
           "plain_ms_median": round(float(np.median(plain)), 4),
           "learned_ms_median": round(float(np.median(learned)), 4),
           "plain_ms_min_max": [round(min(plain), 4), round(max(plain), 4)],
           "learned_ms_min_max": [round(min(learned), 4), round(max(learned), 4)],
           "speedup_vs_plain": round(float(np.median(plain)) / float(np.median(learned)), 3),
           "fell_back": fb, "bit_exact_vs_plain": bool(same), "reps": len(plain)}
    log(f"reuse: plain {res['plain_ms_median']} ms, learned {res['learned_ms_median']} ms, "
        f"fell_back {fb}, same={same}")
    del b, lb, pp, pl, tb
    torch.cuda.empty_cache()
    return res


def batched_c4(torch, kd, kdgen, args):
    log("generating 4096 point-cloud trees")
    x, offsets = kdgen.c4_batched()
    t = torch.from_numpy(x).cuda()
    total = int(offsets[-1])
    B = len(offsets) - 1
    knobs = {}
    if not args.no_tune:
        from paper_1410_5420_amd import autotune

        knobs = autotune.tune(t, "batched", offsets=offsets, reps=3, record=False)["config"]
        log(f"batched knobs {knobs}")
    bb = kd.BatchedBuilder(offsets, 3, torch.float32, **knobs)
    perm_b = torch.full((total,), -1, dtype=torch.int32, device=t.device)
    reps = max(3, args.steps // 4)
    batched_ms = time_steps(torch, lambda: bb.build(t, perm_b), reps, 2)

    # the same build captured once into a HIP graph and replayed
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bb.build(t, perm_b)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        bb.build(t, perm_b)
    graph_ms = time_steps(torch, g.replay, reps, 1)
    nub = bb.n_unique.clone()

    # a host loop of plain builds, one per tree, on the same stream
    maxn = int(np.max(np.diff(offsets)))
    pb = kd.Builder(maxn, 3, torch.float32)
    perm_l = torch.full((total,), -1, dtype=torch.int32, device=t.device)
    views = [(t[int(offsets[i]):int(offsets[i + 1])], perm_l[int(offsets[i]):int(offsets[i + 1])])
             for i in range(B)]

    def loop():
        for tv, pv in views:
            pb.build(tv, pv)

    loop_ms = time_steps(torch, loop, 1, 1)
    torch.cuda.synchronize()
    # bit-exact: every tree of the batch equals its plain build (positions
    # past n_unique stay -1 on both sides)
    perm_b.fill_(-1)
    bb.build(t, perm_b)
    torch.cuda.synchronize()
    same = torch.equal(perm_b, perm_l) and torch.equal(bb.n_unique, nub)
    res = {"workload": f"{B} float32 point-cloud trees, n_i log-uniform in [64, 65536], k=3",
           "trees": B, "rows": total, "knobs": knobs, "ms_per_build": round(batched_ms, 4),
           "tuples_per_s": round(total / (batched_ms * 1e-3), 1),
           "graph_replay_ms": round(graph_ms, 4),
           "host_loop_of_plain_builds_ms": round(loop_ms, 3),
           "speedup_vs_loop": round(loop_ms / batched_ms, 2), "bit_exact_vs_loop": bool(same)}
    log(f"batched: {batched_ms:.3f} ms (graph {graph_ms:.3f}), loop {loop_ms:.1f} ms, same={same}")
    return res


if __name__ == "__main__":
    main()
