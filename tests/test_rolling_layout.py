"""CPU replay of level form 4 (one multi-level split per level).

The replay runs the form's steps on rank records exactly as the kernels
define them: which array splits at each level, from which depth, through which
medians, from which buffer into which, and which record planes each split
writes (the masks come from the compiled library, kd_level_plan).  Every
buffer starts out poisoned, so a read of a plane no earlier step wrote fails.
The tree it produces -- nodes recorded level by level, the last layouts the
on-chip finish reads, and the subtrees below the cutover built from them --
must equal the oracle's.  The device may stop above the host's level count
(duplicates shrink the tree after the host has sized the launches), so every
device depth up to the host's is replayed with the host's masks.
"""
import numpy as np
import pytest

import kdgen
import oracle

POISON = -1


@pytest.fixture(scope="module")
def L():
    from paper_1410_5420_amd import _lib

    return _lib


def roll_depth(L, j, k):
    return j + k * ((L - 1 - j) // k) + 1 if L > j else 0


def roll_moves(L, j, k):
    if j == 0:
        return (L - 1) // k if L >= 1 else 0
    return (L - 1 - j) // k + 1 if L > j else 0


def plane_of(j, o, k):
    return (o - j - 1 + 2 * k) % k


def cutover_depth(nu, C):
    d = 0
    while (nu >> d) > C:
        d += 1
    return d


def subarray(nu, depth, c):
    """Range of subarray c (left to right) at `depth` of a tree of nu nodes."""
    s, e = 0, nu - 1
    for l in range(depth - 1, -1, -1):
        m = s + (e - s) // 2
        if (c >> l) & 1:
            s = m + 1
        else:
            e = m - 1
    return s, e


def descend(s, e, b, levels):
    for l in range(levels - 1, -1, -1):
        m = s + (e - s) // 2
        if (b >> l) & 1:
            s = m + 1
        else:
            e = m - 1
    return s, e


def brute_subtree(elems, rank, k, depth, s, perm):
    """Sort-at-every-node definition below the cutover (ranks order the super keys)."""
    if not elems:
        return
    o = depth % k
    srt = sorted(elems, key=lambda x: rank[o][x])
    mid = (len(srt) - 1) // 2
    perm[s + mid] = srt[mid]
    brute_subtree(srt[:mid], rank, k, depth + 1, s, perm)
    brute_subtree(srt[mid + 1:], rank, k, depth + 1, s + mid + 1, perm)


def replay(t, C, host_levels, lm, fm):
    n, k = t.shape
    arrays, nu = oracle.presort(t)
    rows = arrays[0]
    rank = np.zeros((k, n), dtype=np.int64)
    for o in range(k):
        rank[o, arrays[o]] = np.arange(nu)
    bufs = [np.full((k, k - 1, max(nu, 1)), POISON, dtype=np.int64) for _ in range(3)]
    for j in range(k):
        for c in range(k - 1):
            bufs[0][j, c, :nu] = rank[(j + 1 + c) % k, arrays[j]]
    D = cutover_depth(nu, C)
    assert D <= host_levels

    def buf(m):
        return bufs[0 if m == 0 else (1 if m % 2 else 2)]

    med = {}
    perm = np.full(nu, -1, dtype=np.int64)

    def split(q, frm, to, moves, wmask):
        src, dst = buf(moves)[q], buf(moves + 1)[q]
        sl = to - frm
        for c0 in range(1 << frm):
            s, e = subarray(nu, frm, c0)
            buckets = [[] for _ in range(1 << sl)]
            for i in range(s, e + 1):
                h, drop = 1, False
                for l in range(frm, to):
                    r = src[plane_of(q, l % k, k), i]
                    assert r != POISON, f"split of array {q}: plane for level {l} never written"
                    c = (c0 << (l - frm)) + (h - (1 << (l - frm)))
                    nr = med[(l, c)]
                    if r == nr:
                        drop = True
                        break
                    h = 2 * h + (1 if r > nr else 0)
                if not drop:
                    buckets[h - (1 << sl)].append(i)
            for b, lst in enumerate(buckets):
                ds, de = descend(s, e, b, sl)
                assert len(lst) == de - ds + 1, "bucket size differs from the subtree's"
                for off, i in enumerate(lst):
                    for c in range(k - 1):
                        if (wmask >> c) & 1:
                            assert src[c, i] != POISON, f"array {q} moves plane {c}, never written"
                            dst[c, ds + off] = src[c, i]

    for Lv in range(host_levels):
        if Lv >= D:
            continue  # the device skips levels past its own count
        p = Lv % k
        if Lv >= 1:
            split(p, roll_depth(Lv, p, k), Lv, roll_moves(Lv, p, k), lm[Lv])
        arr = buf(roll_moves(Lv, p, k) + (1 if Lv >= 1 else 0))[p]
        for c in range(1 << Lv):
            s, e = subarray(nu, Lv, c)
            m = s + (e - s) // 2
            r1 = arr[0, m]
            assert r1 != POISON
            rp = bufs[0][(p + 1) % k, k - 2, r1]
            med[(Lv, c)] = rp
            r0 = rp if p == 0 else arr[plane_of(p, 0, k), m]
            assert r0 != POISON
            perm[m] = rows[r0]
    if D >= 1:
        for j in range(1, k):
            a = roll_depth(D, j, k)
            if a < D:
                split(j, a, D, roll_moves(D, j, k), fm[j])
    # the on-chip finish: arrays 1 .. k-1 at depth D, their order-0 plane
    layouts = {}
    for j in range(1, k):
        moves = roll_moves(D, j, k) + (1 if D >= 1 and roll_depth(D, j, k) < D else 0)
        layouts[j] = buf(moves)[j, plane_of(j, 0, k)]
    for c in range(1 << D):
        s, e = subarray(nu, D, c)
        if e < s:
            continue
        elems = None
        for j in range(1, k):
            r0 = layouts[j][s:e + 1]
            assert np.all(r0 != POISON), f"finish reads an unwritten order-0 plane of array {j}"
            ej = [int(rows[r]) for r in r0]
            assert all(rank[j][ej[i]] < rank[j][ej[i + 1]] for i in range(len(ej) - 1)), \
                f"array {j} is not in its order inside subarray {c} at depth {D}"
            if elems is None:
                elems = ej
            assert sorted(ej) == sorted(elems)
        if elems is None:  # k = 1 does not reach here
            continue
        brute_subtree(elems, rank, k, D, s, perm)
    return perm, nu


CASES = [(2, 300, 0.3, 4), (3, 700, 0.4, 4), (3, 2000, 0.05, 8), (4, 900, 0.3, 2), (5, 600, 0.2, 4),
         (6, 500, 0.3, 2), (7, 400, 0.1, 2), (8, 700, 0.3, 2), (3, 5, 0.0, 4), (4, 1, 0.0, 4)]


@pytest.mark.parametrize("k,n,dup,C", CASES)
def test_rolling_replay_matches_oracle(L, k, n, dup, C):
    t = kdgen.uniform_int(n, k, -1000, 1000, dup, 4000 + 17 * k + n)
    want = oracle.build_tree(t, children=False)
    nu = want["n_unique"]
    D = cutover_depth(nu, C)
    for host_levels in sorted({D, D + 1, D + 2, cutover_depth(n, C), D + k}):
        lm, fm = L.level_plan(k, host_levels)
        perm, nu2 = replay(t, C, host_levels, lm, fm)
        assert nu2 == nu
        assert np.array_equal(perm, want["perm"]), (k, n, host_levels)


def test_level_plan_moves_less_than_form1(L):
    """Planes moved per element by the levels of form 4 against form 1 (two
    reads/writes per plane): at k = 3, 14 levels, form 4 moves each array
    once per level it splits in."""
    lm, fm = L.level_plan(3, 14)
    moved4 = sum(bin(m).count("1") for m in lm) + sum(bin(m).count("1") for m in fm)
    assert moved4 <= 14 * 2 and moved4 >= 13
    lm8, _ = L.level_plan(8, 12)
    assert sum(bin(m).count("1") for m in lm8) <= 12 * 7


def test_level_plan_rejects_bad_arguments(L):
    import ctypes

    fm = (ctypes.c_uint32 * 8)()
    lm = (ctypes.c_uint32 * 32)()
    assert L.lib.kd_level_plan(1, 3, lm, fm) == -1
    assert L.lib.kd_level_plan(9, 3, lm, fm) == -4
    assert L.lib.kd_level_plan(3, -1, lm, fm) == -1
    assert L.lib.kd_level_plan(3, 31, lm, fm) == -4
    assert L.lib.kd_level_plan(3, 3, lm, None) == -1


@pytest.mark.parametrize("k,n", [(3, 2000), (5, 1500)])
def test_replay_catches_a_dropped_plane(L, k, n):
    """The replay is a check of the plan, not a copy of it: a level whose write
    mask loses one plane that a later split or the finish reads must fail."""
    t = kdgen.uniform_int(n, k, -1000, 1000, 0.0, 777 + k)
    want = oracle.build_tree(t, children=False)
    C = 4
    host_levels = cutover_depth(want["n_unique"], C)
    lm, fm = L.level_plan(k, host_levels)
    caught = 0
    for lv in range(1, host_levels):
        for c in range(k - 1):
            if not (lm[lv] >> c) & 1:
                continue
            bad = list(lm)
            bad[lv] &= ~(1 << c)
            try:
                perm, _ = replay(t, C, host_levels, bad, fm)
            except AssertionError:
                caught += 1
                continue
            # a plane nobody reads again may be dropped harmlessly, but then
            # the tree must still be right
            assert np.array_equal(perm, want["perm"])
    assert caught > 0
