"""Pins of the CPU oracle against facts that do not come from the oracle.

* the paper's 15-tuple worked example (Sec. 2.1, stated facts only);
* np.lexsort (stable presort) and np.unique (duplicate removal);
* the "sort at every node" definition of the balanced tree;
* the k = 1 closed form (in-order layout == sorted unique order);
* invariants: depth balance, super-key order at every node, complete
  permutation of the unique representatives, child positions;
* IEEE totalOrder on a hand-ordered list of special float32 values;
* region and nearest-neighbour queries against linear scans.
"""
import json
import os

import numpy as np
import pytest

import bruteforce as bf
import kdgen
import oracle
from oracle import queries

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")


def worked_example():
    g = json.load(open(GOLDEN))
    rows = dict(g["tuples_stated"])
    rows.update({k: v for k, v in g["completion_used"].items() if k != "note"})
    t = np.array([rows[str(i)] for i in range(15)], dtype=np.int32)
    return t, g


def test_worked_example_presort():
    t, g = worked_example()
    arrays, nu = oracle.presort(t)
    assert nu == 15
    names = ["xyz", "yzx", "zxy"]
    for d, name in enumerate(names):
        first, last = g["initial_first_two_last_two"][name]
        assert list(arrays[d, :2]) == first, name
        assert list(arrays[d, -2:]) == last, name
    assert arrays[0, g["xyz_median"]["address"]] == g["xyz_median"]["value"]
    assert list(arrays[1, 2:6]) == g["yzx_initial_2_to_5"]["values"]


def test_worked_example_splits():
    t, g = worked_example()
    # after one level the storage of A[0] holds the partitioned yzx array
    r1 = oracle.build_tree(t, max_depth=1, arrays=True, children=False)
    yzx1 = r1["arrays"][0]
    facts = g["yzx_after_first_split"]
    for addr, val in facts.items():
        if addr in ("absent", "cite"):
            continue
        assert yzx1[int(addr)] == val
    lower_upper = np.concatenate([yzx1[:7], yzx1[8:]])
    assert facts["absent"] not in lower_upper
    for addr, val in g["yzx_after_first_split_medians"].items():
        if addr != "cite":
            assert yzx1[int(addr)] == val
    # after two levels A[0] holds the partitioned zxy array
    r2 = oracle.build_tree(t, max_depth=2, arrays=True, children=False)
    zxy2 = r2["arrays"][0]
    for addr, val in g["zxy_after_second_split"].items():
        if addr != "cite":
            assert zxy2[int(addr)] == val


def test_worked_example_tree():
    t, g = worked_example()
    r = oracle.build_tree(t)
    perm, lo, hi = r["perm"], r["lo"], r["hi"]
    tree = g["tree"]
    root = 7
    assert perm[root] == tree["root"]
    assert [perm[lo[root]], perm[hi[root]]] == tree["children"]
    for child_pos in (lo[root], hi[root]):
        want = tree["grandchildren"][str(perm[child_pos])]
        assert [perm[lo[child_pos]], perm[hi[child_pos]]] == want
    bf.check_invariants(t, perm, lo, hi)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8])
@pytest.mark.parametrize("seed", [0, 1])
def test_presort_matches_lexsort_unique(k, seed):
    # few distinct values per column -> many ties and exact duplicates
    t = kdgen.uniform_int(700, k, -3, 4, 0.2, seed)
    arrays, nu = oracle.presort(t)
    want = bf.presort_dedup(t)
    assert nu == want.shape[1]
    assert np.array_equal(arrays, want)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_build_matches_sort_at_every_node(k, seed):
    lohi = [(-4, 5), (0, 1 << 20), (-(2 ** 31), 2 ** 31)][seed]
    t = kdgen.uniform_int(1500 + 37 * seed, k, lohi[0], lohi[1], 0.05, seed)
    r = oracle.build_tree(t)
    assert np.array_equal(r["perm"].astype(np.int64), bf.sort_at_every_node(t))
    bf.check_invariants(t, r["perm"], r["lo"], r["hi"])


def test_build_float32_matches_definition():
    g = kdgen.rng(5)
    t = g.normal(size=(900, 3)).astype(np.float32)
    t[100:150] = t[:50]  # exact copies
    r = oracle.build_tree(t)
    assert np.array_equal(r["perm"].astype(np.int64), bf.sort_at_every_node(t))
    bf.check_invariants(t, r["perm"], r["lo"], r["hi"])


def test_k1_closed_form():
    t = kdgen.uniform_int(1000, 1, -50, 50, 0.3, 3)
    r = oracle.build_tree(t)
    reps = bf.unique_representatives(t)
    want = reps[np.argsort(t[reps, 0], kind="stable")]
    assert np.array_equal(r["perm"].astype(np.int64), want)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 7, 8])
def test_tiny_sizes(n):
    t = kdgen.uniform_int(n, 3, 0, 100, 0.0, 11 + n)
    r = oracle.build_tree(t)
    assert r["n_unique"] == len(bf.unique_representatives(t))
    if n:
        assert np.array_equal(r["perm"].astype(np.int64), bf.sort_at_every_node(t))
        bf.check_invariants(t, r["perm"], r["lo"], r["hi"])


def test_all_duplicates():
    t = np.tile(np.array([[7, -1, 3]], dtype=np.int32), (257, 1))
    r = oracle.build_tree(t)
    assert r["n_unique"] == 1 and list(r["perm"]) == [0]


def test_extreme_int_values():
    lo, hi = np.iinfo(np.int32).min, np.iinfo(np.int32).max
    base = np.array([[lo, hi, 0], [hi, lo, 0], [lo, lo, lo], [hi, hi, hi], [0, 0, 0], [-1, 1, -1],
                     [1, -1, 1], [lo, hi, 0]], dtype=np.int32)
    r = oracle.build_tree(base)
    assert r["n_unique"] == 7
    assert np.array_equal(r["perm"].astype(np.int64), bf.sort_at_every_node(base))


def test_float_total_order_special_values():
    # ascending IEEE-754 totalOrder, written out by hand
    bits = [0xFFC00000,  # -NaN (quiet)
            0xFF800000,  # -inf
            0xFF7FFFFF,  # -max
            0xBF800000,  # -1.0
            0x80000001,  # -min subnormal
            0x80000000,  # -0.0
            0x00000000,  # +0.0
            0x00000001,  # +min subnormal
            0x3F800000,  # 1.0
            0x7F7FFFFF,  # +max
            0x7F800000,  # +inf
            0x7FC00000]  # +NaN (quiet)
    vals = np.array(bits, dtype=np.uint32).view(np.float32).reshape(-1, 1)
    shuffled = np.ascontiguousarray(vals[::-1][[3, 0, 7, 11, 1, 9, 5, 2, 10, 4, 6, 8]])
    arrays, nu = oracle.presort(shuffled)
    assert nu == 12
    got = shuffled[arrays[0], 0].view(np.uint32)
    assert [int(b) for b in got] == bits


def test_threads_do_not_change_result():
    t = kdgen.uniform_int(5000, 3, 0, 1000, 0.05, 9)
    a = oracle.build_tree(t, threads=1)
    b = oracle.build_tree(t, threads=8)
    assert np.array_equal(a["perm"], b["perm"])
    assert np.array_equal(a["lo"], b["lo"]) and np.array_equal(a["hi"], b["hi"])


@pytest.mark.parametrize("depth", [1, 2, 3, 4])
def test_level_state_arrays(depth):
    """After `depth` levels every subarray of storage A[r] holds exactly the
    subtree's elements sorted by super key (depth + r) mod k (Sec. 2.1)."""
    t = kdgen.uniform_int(600, 3, 0, 50, 0.05, 21)
    r = oracle.build_tree(t, max_depth=depth, arrays=True, children=False)
    full = oracle.build_tree(t)
    nu = full["n_unique"]
    cols = bf.order_columns(t)
    segs = [(0, nu - 1)]
    for _ in range(depth):
        nxt = []
        for s, e in segs:
            if e < s:
                continue
            m = s + (e - s) // 2
            nxt += [(s, m - 1), (m + 1, e)]
        segs = nxt
    for s, e in segs:
        if e < s:
            continue
        members = np.sort(full["perm"][s:e + 1])
        for rr in range(3):
            seg = r["arrays"][rr, s:e + 1].astype(np.int64)
            assert np.array_equal(np.sort(seg), members)
            want = bf.lexsort_superkey(cols, seg, (depth + rr) % 3)
            assert np.array_equal(seg, want)


def test_c1_workload_is_fast_and_correct():
    t = kdgen.c1_small_uniform()
    r = oracle.build_tree(t)
    assert r["n_unique"] == 4014
    assert sum(r["times"]) < 1.0
    assert np.array_equal(r["perm"].astype(np.int64), bf.sort_at_every_node(t))


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_region_and_nn_queries(dtype):
    g = kdgen.rng(33)
    if dtype == np.int32:
        t = g.integers(0, 64, size=(400, 3)).astype(np.int32)
    else:
        t = g.normal(size=(400, 3)).astype(np.float32)
    r = oracle.build_tree(t)
    perm = r["perm"]
    for _ in range(25):
        if dtype == np.int32:
            a = g.integers(0, 64, size=3)
            b = g.integers(0, 64, size=3)
            q = [int(v) for v in g.integers(0, 64, size=3)]
        else:
            a = g.normal(size=3)
            b = g.normal(size=3)
            q = [float(v) for v in g.normal(size=3)]
        lower, upper = np.minimum(a, b).tolist(), np.maximum(a, b).tolist()
        assert queries.region_search(t, perm, lower, upper) == bf.region_scan(t, perm.astype(np.int64), lower, upper)
        got = [d for d, _ in queries.nearest_neighbors(t, perm, q, 7)]
        assert got == bf.knn_scan_distances(t, perm.astype(np.int64), q, 7)


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_all_nearest_and_reverse_lists(dtype):
    # every node as a query, itself excluded; reverse lists are the transpose
    # (inputs without distance ties, so the neighbour sets are unique)
    g = kdgen.rng(34)
    if dtype == np.int32:
        t = g.integers(-10**6, 10**6, size=(300, 3)).astype(np.int32)
    else:
        t = g.normal(size=(300, 3)).astype(np.float32)
    r = oracle.build_tree(t)
    perm = r["perm"]
    m = 4
    near = queries.all_nearest(t, perm, m)
    assert len(near) == len(perm)
    scan_rows = []
    for pos, row in enumerate(perm):
        others = np.array([int(x) for x in perm if int(x) != int(row)], dtype=np.int64)
        want = bf.knn_scan_distances(t, others, t[int(row)].tolist(), m)
        assert [d for d, _ in near[pos]] == want
        assert int(row) not in [rr for _, rr in near[pos]]
        # brute-force neighbour rows (ties absent): the m smallest distances
        if dtype == np.int32:
            d = [sum((int(a) - int(b)) ** 2 for a, b in zip(t[o], t[int(row)])) for o in others]
        else:
            d = [float(np.sum((t[o].astype(np.float64) - t[int(row)].astype(np.float64)) ** 2)) for o in others]
        order = np.argsort(np.array(d), kind="stable")[:m]
        scan_rows.append([int(others[i]) for i in order])
        assert sorted(rr for _, rr in near[pos]) == sorted(scan_rows[-1])
    rev = queries.reverse_lists(perm, [[rr for _, rr in nb] for nb in near])
    want = {}
    for pos, rows in enumerate(scan_rows):
        for rr in rows:
            want.setdefault(rr, []).append(int(perm[pos]))
    assert rev == {k: sorted(v) for k, v in want.items()}
    assert sum(len(v) for v in rev.values()) == m * len(perm)


def test_region_search_with_nan_coordinates():
    # a NaN coordinate is never inside a box, and a NaN split value does not
    # prune the subtrees below it: the search equals a linear scan
    g = kdgen.rng(35)
    t = g.normal(size=(500, 3)).astype(np.float32)
    # positive and negative NaNs, dense enough that some split values are NaN
    t[g.integers(0, 500, size=60), g.integers(0, 3, size=60)] = np.nan
    t[g.integers(0, 500, size=30), g.integers(0, 3, size=30)] = -np.nan
    r = oracle.build_tree(t)
    perm = r["perm"]
    nodes = t[perm]
    for _ in range(30):
        a, b = g.normal(size=3) * 1.5, g.normal(size=3) * 1.5
        lower, upper = np.minimum(a, b).astype(np.float32), np.maximum(a, b).astype(np.float32)
        with np.errstate(invalid="ignore"):
            inside = np.all((nodes >= lower) & (nodes <= upper), axis=1)
        want = sorted(int(v) for v in perm[inside])
        assert queries.region_search(t, perm, lower.tolist(), upper.tolist()) == want
    everything = queries.region_search(t, perm, [-1e9] * 3, [1e9] * 3)
    assert len(everything) == int((~np.isnan(nodes).any(axis=1)).sum())
