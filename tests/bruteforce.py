"""Independent brute-force checkers that pin the oracle (numpy only).

None of these call the oracle.  They restate what the build must produce from
plain definitions and library routines:

* presort by a super key  == ``np.lexsort`` over the rotated columns (stable);
* duplicate removal       == ``np.unique(rows, axis=0, return_index=True)``;
* the tree                == "sort at every node": sort the subset by the
  super key of its depth, take the element of rank floor((size-1)/2), recurse
  on the elements before and after it;
* queries                 == linear scans.
"""
from __future__ import annotations

import numpy as np


def order_columns(tuples: np.ndarray) -> np.ndarray:
    """Columns as int64 values whose numeric order is the coordinate order.

    int32: the values.  float32: only finite values without -0.0 are
    supported here, where IEEE totalOrder equals numeric order; special values
    are pinned separately by an explicit list.
    """
    if tuples.dtype == np.int32:
        return tuples.astype(np.int64)
    assert tuples.dtype == np.float32
    f = tuples.astype(np.float64)
    assert np.all(np.isfinite(f)) and not np.any((f == 0) & np.signbit(f))
    # rank of each value among all values of its column preserves numeric order
    out = np.empty(tuples.shape, dtype=np.int64)
    for d in range(tuples.shape[1]):
        _, inv = np.unique(f[:, d], return_inverse=True)
        out[:, d] = inv
    return out


def lexsort_superkey(cols: np.ndarray, rows: np.ndarray, p: int) -> np.ndarray:
    """Stable sort of ``rows`` by the super key p : p+1 : ... (mod k)."""
    k = cols.shape[1]
    sub = cols[rows]
    keys = [sub[:, (p + i) % k] for i in range(k - 1, -1, -1)]  # last key is primary
    return rows[np.lexsort(keys)]


def unique_representatives(tuples: np.ndarray) -> np.ndarray:
    """Smallest row index of every distinct (bitwise) row, ascending."""
    bits = np.ascontiguousarray(tuples).view(np.int32)
    _, idx = np.unique(bits, axis=0, return_index=True)
    return np.sort(idx).astype(np.int64)


def presort_dedup(tuples: np.ndarray):
    """The k deduplicated presorted index arrays, by lexsort + unique."""
    cols = order_columns(tuples)
    reps = unique_representatives(tuples)
    n, k = tuples.shape
    return np.stack([lexsort_superkey(cols, reps, d) for d in range(k)]) if n else np.zeros((k, 0), np.int64)


def sort_at_every_node(tuples: np.ndarray) -> np.ndarray:
    """In-order layout of the balanced tree by the plain definition."""
    cols = order_columns(tuples)
    reps = unique_representatives(tuples)
    k = tuples.shape[1]
    perm = np.full(reps.shape[0], -1, dtype=np.int64)

    stack = [(0, reps, 0)]
    while stack:
        base, rows, depth = stack.pop()
        if rows.shape[0] == 0:
            continue
        srt = lexsort_superkey(cols, rows, depth % k)
        r = (srt.shape[0] - 1) // 2
        perm[base + r] = srt[r]
        stack.append((base, srt[:r], depth + 1))
        stack.append((base + r + 1, srt[r + 1:], depth + 1))
    return perm


def check_invariants(tuples: np.ndarray, perm: np.ndarray, lo=None, hi=None):
    """Depth balance, super-key order at every node, complete permutation of
    the unique representatives, and (optionally) child positions."""
    cols = order_columns(tuples)
    k = tuples.shape[1]
    nu = perm.shape[0]
    reps = unique_representatives(tuples)
    assert np.array_equal(np.sort(perm.astype(np.int64)), reps), "perm is not the set of representatives"
    height = 0
    stack = [(0, nu - 1, 0)]
    while stack:
        s, e, depth = stack.pop()
        if e < s:
            continue
        height = max(height, depth + 1)
        m = s + (e - s) // 2
        size_l, size_r = m - s, e - m
        assert size_l <= size_r <= size_l + 1, "not depth balanced"
        p = depth % k
        order = [(p + i) % k for i in range(k)]
        node = cols[perm[m]][order]
        for side, (a, b) in ((-1, (s, m - 1)), (1, (m + 1, e))):
            if b < a:
                continue
            sub = cols[perm[a:b + 1]][:, order]
            # lexicographic compare of every row against the node
            diff = sub - node
            nz = diff != 0
            first = np.where(nz.any(axis=1), nz.argmax(axis=1), -1)
            assert np.all(first >= 0), "equal super keys in a subtree"
            sign = np.sign(diff[np.arange(diff.shape[0]), first])
            assert np.all(sign == side), "super-key order violated"
        if lo is not None:
            lm = (s + (m - 1 - s) // 2) if m - 1 >= s else -1
            hm = (m + 1 + (e - m - 1) // 2) if e >= m + 1 else -1
            assert lo[m] == lm and hi[m] == hm, "child positions wrong"
        stack.append((s, m - 1, depth + 1))
        stack.append((m + 1, e, depth + 1))
    if nu:
        assert height == int(np.floor(np.log2(nu))) + 1, "height is not floor(log2 n)+1"


def region_scan(tuples: np.ndarray, rows: np.ndarray, lower, upper):
    x = tuples[rows].astype(np.float64 if tuples.dtype == np.float32 else np.int64)
    inside = np.all((x >= np.asarray(lower)) & (x <= np.asarray(upper)), axis=1)
    return sorted(int(r) for r in rows[inside])


def knn_scan_distances(tuples: np.ndarray, rows: np.ndarray, query, m: int):
    if tuples.dtype == np.int32:
        d = [sum((int(v) - int(q)) ** 2 for v, q in zip(tuples[r], query)) for r in rows]
    else:
        d = [float(np.sum((tuples[r].astype(np.float64) - np.asarray(query, np.float64)) ** 2)) for r in rows]
    return sorted(d)[:m]
