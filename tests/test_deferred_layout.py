"""Layout rules of level forms 1 and 3 (deferred partitioning), on the CPU.

Two models of what the library computes, checked against definitions:
- the bucket numbering of the split (Appendix, "Deferred Merge Sort and
  Partitioning"): a stable sort of array j, in its presorted order, by each
  element's in-order bucket among the subarrays and nodes of depth D must
  give exactly the layout that D levels of stable partitioning give;
- the buffer accounting: the number of writes into array j's records before
  a depth (the plain count less j - 1 once array j is split, one write before
  that) must make every read of a level, of a split and of the on-chip finish
  find the layout of its depth with the planes it needs.
Both rules are also read from the compiled library (kd_level_masks) and
replayed from there, so the model and the library cannot drift apart.
"""
import random

import pytest


def moves_before(depth, j, k):
    as_split = (depth - j + k - 1) // k if depth > j else 0
    return depth - as_split


def array_moves(defer, depth, j, k):
    if not defer or j < 2:
        return moves_before(depth, j, k)
    return moves_before(depth, j, k) - (j - 1) if depth >= j else 1


def buffer_of(moves):
    return 0 if moves == 0 else (1 if moves & 1 else 2)


def write_masks(k, levels, defer):
    need = [0] * k
    for j in range(1, k):
        need[j] = 1 << (k - 1 - j)
    masks = [0] * levels
    for d in range(levels - 1, -1, -1):
        p = d % k
        m = 0
        for j in range(k):
            if j != p and not (defer and j >= 2 and d < j):
                m |= need[j] << (8 * j)
        masks[d] = m
        for j in range(k):
            if j == p:
                need[j] |= 1
                if p != 0:
                    need[j] |= 1 << ((k - p - 1) % k)
            elif need[j]:
                need[j] |= 1 << ((p - j - 1 + 2 * k) % k)
    return masks


def replay(k, levels, deepest, defer, plan=None):
    """Every read finds the layout of its depth with the planes it needs.
    plan: (masks, moves[depth][j]) to replay instead of this file's rules
    (the compiled library's, from kd_level_masks)."""
    if plan is not None:
        lib_masks, lib_moves = plan

        def array_moves(defer_, d, j, k_):  # noqa: F811
            return lib_moves[d][j]
    else:
        lib_masks = None
        array_moves = globals()["array_moves"]
    state = {(0, j): (0, 0xFF) for j in range(k)}  # (buffer, array) -> (depth, planes)
    have_nodes = set()

    def read(d, j, planes):
        got = state.get((buffer_of(array_moves(defer, d, j, k)), j))
        assert got is not None and got[0] == d and got[1] & planes == planes, (k, levels, deepest, d, j)

    def split(j):
        depth = min(j, deepest)
        assert all(x in have_nodes for x in range(depth))
        state[(1, j)] = (depth, 0xFF)

    masks = lib_masks if lib_masks is not None else (write_masks(k, levels, defer) if levels else [])
    for d in range(levels):
        if defer and 2 <= d < k:
            split(d)
        if defer and d <= k - 2 and d < deepest:
            read(d, d, 1)
            have_nodes.add(d)
        if d >= deepest:
            continue
        p = d % k
        read(d, p, 1 | ((1 << ((k - p - 1) % k)) if p else 0))
        bp = buffer_of(array_moves(defer, d, p, k))
        state[(bp, p)] = (d + 1, state[(bp, p)][1])  # the split array is already partitioned
        for j in range(k):
            w = (masks[d] >> (8 * j)) & 0xFF
            if j == p or not w:
                continue
            read(d, j, w | (1 << ((p - j - 1 + 2 * k) % k)))
            state[(buffer_of(array_moves(defer, d, j, k) + 1), j)] = (d + 1, w)
    if defer:
        for j in range(max(levels, 2), k):
            split(j)
    for j in range(1, k):
        read(deepest, j, 1 << (k - 1 - j))


def test_buffer_accounting():
    for k in range(2, 9):
        for levels in range(0, 18):
            for deepest in range(0, levels + 1):
                replay(k, levels, deepest, 0)
                if k >= 3:
                    replay(k, levels, deepest, 1)


@pytest.fixture(scope="module")
def L():
    from paper_1410_5420_amd import _lib

    return _lib


def test_rules_equal_the_compiled_plan(L):
    """The rules above are the library's own (kd_level_masks: the host's
    write masks and the move count that picks each array's buffer)."""
    for k in range(2, 9):
        for levels in range(0, 21):
            for defer in ((0, 1) if k >= 3 else (0,)):
                masks, moves = L.level_masks(k, levels, defer)
                assert masks == (write_masks(k, levels, defer) if levels else []), (k, levels, defer)
                for d in range(levels + 1):
                    for j in range(k):
                        assert moves[d][j] == array_moves(defer, d, j, k), (k, levels, defer, d, j)


def test_buffer_accounting_of_the_compiled_plan(L):
    for k in range(2, 9):
        for levels in range(0, 18):
            for defer in ((0, 1) if k >= 3 else (0,)):
                plan = L.level_masks(k, levels, defer)
                for deepest in range(0, levels + 1):
                    replay(k, levels, deepest, defer, plan)


def test_buffer_accounting_catches_a_wrong_count():
    """A plain move count for a deferred array must fail the replay."""
    global array_moves
    good = array_moves
    try:
        array_moves = lambda defer, depth, j, k: moves_before(depth, j, k)  # noqa: E731
        failed = False
        try:
            replay(4, 10, 10, 1)
        except AssertionError:
            failed = True
        assert failed
    finally:
        array_moves = good


def bucket(ranks, node_rank, x, D):
    q = 0
    for d in range(D):
        r, nr = ranks[d][x], node_rank[(d, q)]
        if r == nr:
            return q * (2 << (D - d)) + (1 << (D - d)) - 1
        q = 2 * q + (1 if r > nr else 0)
    return 2 * q


def test_bucket_split_equals_level_partition():
    for seed in range(25):
        rnd = random.Random(seed)
        for k in range(3, 9):
            for j in range(2, k):
                for D in range(0, j + 1):
                    nu = rnd.randrange(1 << (D + 1), 300)
                    ranks = [rnd.sample(range(nu), nu) for _ in range(k)]
                    order = [sorted(range(nu), key=lambda x, o=o: ranks[o][x]) for o in range(k)]
                    arrays = [list(a) for a in order]
                    node_rank = {}
                    subs = [(0, nu - 1, 0)]
                    for d in range(D):
                        p = d % k
                        nxt_arrays = [list(a) for a in arrays]
                        nxt = []
                        for s, e, q in subs:
                            m = s + (e - s) // 2
                            med = arrays[p][m]
                            node_rank[(d, q)] = ranks[p][med]
                            for o in range(k):
                                if o == p:
                                    continue
                                part = arrays[o][s:e + 1]
                                lo = [x for x in part if ranks[p][x] < ranks[p][med]]
                                hi = [x for x in part if ranks[p][x] > ranks[p][med]]
                                nxt_arrays[o][s:m] = lo
                                nxt_arrays[o][m + 1:e + 1] = hi
                            nxt += [(s, m - 1, 2 * q), (m + 1, e, 2 * q + 1)]
                        arrays, subs = nxt_arrays, nxt
                    got = sorted(order[j], key=lambda x: bucket(ranks, node_rank, x, D))
                    assert max(bucket(ranks, node_rank, x, D) for x in range(nu)) <= 254
                    for s, e, _ in subs:
                        assert got[s:e + 1] == arrays[j][s:e + 1], (seed, k, j, D)


def test_level_masks_rejects_bad_arguments(L):
    import ctypes

    wm = (ctypes.c_uint64 * 32)()
    mv = (ctypes.c_int32 * 512)()
    assert L.lib.kd_level_masks(1, 3, 0, wm, mv) == -1
    assert L.lib.kd_level_masks(3, 3, 2, wm, mv) == -1
    assert L.lib.kd_level_masks(3, 3, 0, wm, None) == -1
    assert L.lib.kd_level_masks(3, 3, 0, None, mv) == -1
    assert L.lib.kd_level_masks(9, 3, 0, wm, mv) == -4
    assert L.lib.kd_level_masks(3, 31, 0, wm, mv) == -4
