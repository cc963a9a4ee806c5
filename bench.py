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


def byte_model(kernel: str, n: int, nu: int, k: int, R: int):
    """Algorithmic bytes of every launch of one kernel class in one build.

    Returns (bytes per launch, unit description).  Streams count 4 bytes per
    element word read or written; a gathered word counts 4 bytes.
    """
    P = 4  # 8-bit digit passes per 32-bit word
    if kernel == "level":
        # k-1 arrays of R rank planes, each read once and written once
        per_unit = (k - 1) * R * 4 * 2
        return per_unit * nu, f"{per_unit} B x n_unique elements"
    if kernel == "onesweep":
        total = 0
        for w in range(k):  # array 0: all n rows, LSD over k words
            first = w == 0
            total += n * ((4 if first else 8) + 8)  # pass 0: key (+id) in, pair out
            total += n * 16 * (P - 2)  # middle passes: pair in, pair out
            total += n * (8 + (8 if w == k - 1 else 4))  # last pass: pair in, id (+key) out
        for _ in range(k - 1):  # chain: n_unique rows, one word each
            total += nu * (8 + 8) + nu * 16 * (P - 2) + nu * (8 + 4)
        launches = k * P + (k - 1) * P
        return total / launches, "radix pair traffic averaged over the build's passes"
    if kernel == "leaf":
        per_unit = 4 * k + 4 + 4  # plane-0 ranks of k arrays in, perm out, row id gathered
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

    R = k
    bytes_per_launch, unit_desc = byte_model(args.probe, n, nu, k, R)
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
                   "cutover": args.cutover or 2048,
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
