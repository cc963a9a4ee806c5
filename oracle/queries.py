"""Tree queries over the oracle's in-order layout (test infrastructure).

The paper names two searches over the built tree: all points inside a
k-dimensional hyper-rectangle (Appendix, "Source Code for Optimized
Algorithms") and the m nearest neighbours of a query point kept in a
priority queue (Appendix, "Nearest Neighbors").  Both walk the implicit tree
of the in-order layout: the node of ``[s, e]`` is at ``s + (e - s) // 2`` and
splits on dimension ``depth mod k``.

Every element of a "less than" subtree has a super key below the node's, so
its coordinate in the split dimension is <= the node's (ties are possible when
the split coordinates are equal and a later portion decides); symmetrically
">=" for the "greater than" subtree.  The searches prune with those
non-strict bounds.  Coordinates are handled exactly: Python ints for int32,
float64 for float32.
"""
from __future__ import annotations

import heapq

import numpy as np


class _coords:
    """Exact coordinates of a row, converted when first read (Python ints for
    int32, float64 for float32), so a search costs what it visits."""

    def __init__(self, tuples: np.ndarray):
        self.t = tuples
        self.cache = {}

    def __getitem__(self, row: int):
        x = self.cache.get(row)
        if x is None:
            r = self.t[row]
            if self.t.dtype == np.int32:
                x = tuple(int(v) for v in r)
            else:
                x = tuple(float(v) for v in r.astype(np.float64))
            self.cache[row] = x
        return x


def region_search(tuples: np.ndarray, perm: np.ndarray, lower, upper):
    """Rows of all tree nodes with ``lower[d] <= x[d] <= upper[d]`` for every d."""
    pts = _coords(tuples)
    k = tuples.shape[1]
    found = []

    def visit(s, e, depth):
        if e < s:
            return
        m = s + (e - s) // 2
        row = int(perm[m])
        x = pts[row]
        if all(lower[d] <= x[d] <= upper[d] for d in range(k)):
            found.append(row)
        p = depth % k
        # a side is skipped only when the split value proves the box misses it
        # (a NaN split value proves nothing)
        if not lower[p] > x[p]:
            visit(s, m - 1, depth + 1)
        if not upper[p] < x[p]:
            visit(m + 1, e, depth + 1)

    visit(0, len(perm) - 1, 0)
    return sorted(found)


def nearest_neighbors(tuples: np.ndarray, perm: np.ndarray, query, m: int, exclude=None):
    """The m nearest tree nodes to ``query`` as ``[(sq_distance, row), ...]``
    in increasing distance, found with a bounded max-priority queue.  The node
    of row ``exclude`` (if given) is not a candidate."""
    pts = _coords(tuples)
    k = tuples.shape[1]
    q = tuple(query)
    heap = []  # max-heap on distance via negation

    def sqd(x):
        return sum((x[d] - q[d]) * (x[d] - q[d]) for d in range(k))

    def visit(s, e, depth):
        if e < s:
            return
        mid = s + (e - s) // 2
        row = int(perm[mid])
        x = pts[row]
        dist = sqd(x)
        if row == exclude:
            pass
        elif len(heap) < m:
            heapq.heappush(heap, (-dist, -row))
        elif dist < -heap[0][0]:
            heapq.heapreplace(heap, (-dist, -row))
        p = depth % k
        diff = q[p] - x[p]
        near, far = ((s, mid - 1), (mid + 1, e)) if diff <= 0 else ((mid + 1, e), (s, mid - 1))
        visit(near[0], near[1], depth + 1)
        if len(heap) < m or diff * diff <= -heap[0][0]:
            visit(far[0], far[1], depth + 1)

    visit(0, len(perm) - 1, 0)
    return sorted((-d, -r) for d, r in heap)


def all_nearest(tuples: np.ndarray, perm: np.ndarray, m: int):
    """Every node's m nearest other nodes (Appendix, "Nearest Neighbors":
    each point of the tree taken as a query point), as one list of
    ``[(sq_distance, row), ...]`` per tree position."""
    return [nearest_neighbors(tuples, perm, tuples[int(r)].tolist(), m, exclude=int(r))
            for r in perm]


def reverse_lists(perm: np.ndarray, near_rows):
    """Reverse nearest neighbours: for every row, the rows of the nodes that
    have it among their nearest (``near_rows[pos]``: the neighbour rows of
    the node at tree position pos), ascending."""
    out = {}
    for pos, rows in enumerate(near_rows):
        for r in rows:
            out.setdefault(int(r), []).append(int(perm[pos]))
    return {r: sorted(v) for r, v in out.items()}
