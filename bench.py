"""Benchmark: balanced k-d tree build throughput on one MI355X.

Workload (the headline configuration): k = 3, n = 2^24 int32 tuples uniform
over the full signed range with 0.1% exact copies, one tree.  A step is one
whole build -- presort by the three cyclic super keys, duplicate removal and
the level-by-level partition -- with the tuples already resident in HBM and a
preallocated workspace.  value = n / (time per step), in tuples/s.

Beside it: presort and partition phase times (measured on their own), the
roofline of the dominant kernel (algorithmic bytes per launch over its average
launch time, from HIP events the library records around that kernel on its own
stream during the timed steps), and the CPU oracle timed on the host.

Prints exactly one JSON line.
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

METRIC = "tuples/sec k-d build (k=3, n=2^24, bit-exact) plain vs batched/learned; % HBM peak"
HBM_PEAK_GBS = 8000.0


def onesweep_bytes(n: int, nu: int, k: int):
    """(total algorithmic bytes, launches) of all radix scatter passes of one build.

    Array 0 is sorted over all n rows, word by word; every pass moves its key
    word and k payload words (the row id and the other key words), the first
    one reading the tuple rows themselves.  Each of the k-1 chain sorts runs
    over the n_unique rows and moves its key word and k payload words (row id,
    ranks known so far, key words of the later sorts); its last pass drops the
    key.  Every word read or written counts 4 bytes.
    """
    P = 4  # 8-bit digit passes per 32-bit word
    words = 0
    for w in range(k - 1, -1, -1):
        for ps in range(P):
            words += n * ((k if (w == k - 1 and ps == 0) else k + 1) + (k + 1))
    for _ in range(k - 1, 0, -1):
        for ps in range(P):
            words += nu * ((k if ps == 0 else k + 1) + (k if ps == P - 1 else k + 1))
    return 4 * words, 2 * k * P - P


def level_bytes(nu: int, k: int, cutover: int):
    """(total algorithmic bytes, launches) of the global partition levels:
    every array but the split one is read once and written once; records hold
    k-1 ranks, plus the row id in array 0's."""
    R = k - 1
    levels = 0
    while (nu >> levels) > cutover:
        levels += 1
    total = 0
    for L in range(levels):
        p = L % k
        words = sum(R + (1 if j == 0 else 0) for j in range(k) if j != p)
        total += nu * words * 4 * 2
    return total, levels


def byte_model(kernel: str, n: int, nu: int, k: int, cutover: int):
    """Algorithmic bytes of one launch of a kernel class (averaged over the
    build's launches of that class), and how they arise."""
    if kernel == "level":
        total, launches = level_bytes(nu, k, cutover)
        return total / max(launches, 1), (f"{launches} levels: per level (k-1) arrays x (k-1) ranks "
                                          f"(+ row id in array 0) x 4 B, read + write, x n_unique")
    if kernel == "onesweep":
        total, launches = onesweep_bytes(n, nu, k)
        return total / launches, f"radix key + payload words of the build's {launches} passes, averaged"
    if kernel == "leaf":
        per_unit = 4 * k + 4  # order-0 rank of k-1 arrays + row id in, perm out
        return per_unit * nu, f"{per_unit} B x n_unique elements"
    raise ValueError(kernel)


def cpu_baseline(t: np.ndarray):
    import oracle

    cores = min(16, os.cpu_count() or 1)
    q = 1
    while q * 2 <= cores:
        q *= 2
    t0 = time.perf_counter()
    r = oracle.build_tree(t, threads=q, children=False)
    dt = time.perf_counter() - t0
    return {"value": t.shape[0] / dt, "unit": "tuples/s", "cores": q, "kind": "oracle",
            "sample": f"one whole build of the same {t.shape[0]}-row input "
                      f"({dt:.1f} s; presort {r['times'][0]:.1f} s, partition {r['times'][1]:.1f} s), "
                      f"paper's parent/child threads, q={q}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--probe", default="level", choices=["level", "onesweep", "leaf"])
    ap.add_argument("--cutover", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
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
    print(f"[bench] generating n={n} k={k}", file=sys.stderr, flush=True)
    t_host = kdgen.c2_full_range(n)
    dev = torch.device("cuda:0")
    t = torch.from_numpy(t_host).to(dev)
    b = kd.Builder(n, k, torch.int32, dev, cutover=args.cutover)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
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
    print(f"[bench] warmup done, n_unique={nu}", file=sys.stderr, flush=True)

    # timed region: K whole builds; the probe records the dominant kernel's launches
    launches_per_step = {"level": 64, "onesweep": 4 * (2 * k - 1), "leaf": 1}[args.probe]
    cap = launches_per_step * args.steps
    _lib.probe_start(args.probe, cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.build(t, perm)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    durations = _lib.probe_stop(cap)
    ms_per_step = elapsed * 1e3 / args.steps
    print(f"[bench] {args.steps} steps, {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

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

    bytes_per_launch, unit_desc = byte_model(args.probe, n, nu, k, args.cutover or 1024)
    # no-op launches (levels below the cutover for this n_unique) do not count
    real = [d for d in durations if d > 0.002]
    avg_ms = float(np.mean(real)) if real else float("nan")
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": args.probe, "avg_launch_ms": round(avg_ms, 4), "launches": len(real),
                "bytes_per_launch": int(bytes_per_launch), "byte_model": unit_desc}

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
                   "k": k, "n": n, "n_unique": nu, "tuple_dtype": "int32",
                   "cutover": args.cutover or 1024,
                   "presort_ms": round(float(np.median(pre_ms)), 4),
                   "partition_ms": round(float(np.median(part_ms)), 4)},
        "roofline": roofline,
    }
    if not args.no_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(t_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
