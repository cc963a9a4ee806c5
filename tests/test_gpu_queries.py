"""GPU parity of the tree searches (region search and m nearest neighbours)
through the C ABI.

The trees are built on the GPU (their layouts are bit-exact against the
oracle in test_gpu_build.py).  Region searches must return exactly the
oracle's rows, in increasing tree position; nearest-neighbour searches must
return the m nodes smallest in (squared distance, row), which is unique, and
their distances must equal the oracle's.  At larger sizes the reference is a
brute-force scan over the tree's nodes with the same arithmetic (exact
integers; float64 sums in dimension order).
"""
import numpy as np
import pytest

import kdgen
from oracle import queries as oq

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1410_5420_amd as kd

    return kd


def gpu_tree(kd, t: np.ndarray):
    dt = torch.from_numpy(t).cuda()
    perm, nu = kd.build(dt)
    return dt, perm, nu


def boxes(g, t: np.ndarray, nq: int):
    """Boxes around random tuples with random extents (some empty, some
    degenerate points, some covering everything)."""
    n, k = t.shape
    lo_all, hi_all = t.min(axis=0).astype(np.float64), t.max(axis=0).astype(np.float64)
    span = np.maximum(hi_all - lo_all, 1.0)
    centre = t[g.integers(0, n, size=nq)].astype(np.float64)
    ext = span * g.uniform(0.0, 0.4, size=(nq, k)) ** 2
    lower, upper = centre - ext, centre + ext
    lower[0::17] = centre[0::17]  # a point box on a tuple
    upper[0::17] = centre[0::17]
    lower[5::23], upper[5::23] = lo_all - 1, hi_all + 1  # everything
    lower[7::29], upper[7::29] = centre[7::29] + 1, centre[7::29] - 1  # empty
    if t.dtype == np.int32:
        lo = np.clip(np.floor(lower), -2**31, 2**31 - 1).astype(np.int32)
        hi = np.clip(np.ceil(upper), -2**31, 2**31 - 1).astype(np.int32)
    else:
        lo, hi = lower.astype(np.float32), upper.astype(np.float32)
    return lo, hi


def query_points(g, t: np.ndarray, nq: int):
    n, k = t.shape
    base = t[g.integers(0, n, size=nq)].astype(np.float64)
    span = np.maximum(t.max(axis=0).astype(np.float64) - t.min(axis=0), 1.0)
    p = base + g.normal(size=(nq, k)) * span * 0.01
    p[::11] = base[::11]  # exactly on a tuple
    if t.dtype == np.int32:
        return np.clip(np.rint(p), -2**31, 2**31 - 1).astype(np.int32)
    return p.astype(np.float32)


def exact_sq_dist(t: np.ndarray, rows: np.ndarray, q: np.ndarray):
    """Squared distances of tuples[rows] to q with the searches' arithmetic:
    Python ints for int32, float64 summed over d in order for float32."""
    if t.dtype == np.int32:
        x = t[rows].astype(object)
        return [sum((int(a) - int(b)) ** 2 for a, b in zip(row, q)) for row in x]
    x = t[rows].astype(np.float64)
    qq = q.astype(np.float64)
    acc = np.zeros(len(rows))
    for d in range(t.shape[1]):
        diff = x[:, d] - qq[d]
        acc = acc + diff * diff
    return acc.tolist()


def brute_nearest(t: np.ndarray, nodes: np.ndarray, q: np.ndarray, m: int):
    d = exact_sq_dist(t, nodes, q)
    order = sorted(range(len(nodes)), key=lambda i: (d[i], int(nodes[i])))[:m]
    return [int(nodes[i]) for i in order], [d[i] for i in order]


def check_region(kd, t, dt, perm, nu, lo, hi, with_oracle=True):
    p = perm.cpu().numpy()
    pos = np.empty(t.shape[0], dtype=np.int64)
    pos[p] = np.arange(nu)
    dlo, dhi = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    nodes = kd.gather_nodes(dt, perm, nu)
    assert np.array_equal(nodes[:nu].cpu().numpy(), t[p])
    counts = kd.region_count(dt, perm, nu, dlo, dhi, nodes=nodes).cpu().numpy()
    assert np.array_equal(kd.region_count(dt, perm, nu, dlo, dhi).cpu().numpy(), counts)
    bounds = kd.subtree_bounds(nodes, nu)
    check_bounds(t[p], bounds[:nu].cpu().numpy())
    assert np.array_equal(kd.region_count(dt, perm, nu, dlo, dhi, nodes=nodes, bounds=bounds).cpu().numpy(),
                          counts)
    rows_b, offs_b = kd.region_rows(dt, perm, nu, dlo, dhi, nodes=nodes, bounds=bounds)
    rows, offs = kd.region_rows(dt, perm, nu, dlo, dhi, nodes=nodes)
    assert torch.equal(rows_b, rows) and torch.equal(offs_b, offs)
    rows, offs = rows.cpu().numpy(), offs.cpu().numpy()
    assert np.array_equal(np.diff(offs), counts)
    nodes = t[p]
    for q in range(lo.shape[0]):
        got = rows[offs[q]:offs[q + 1]]
        assert np.all(np.diff(pos[got]) > 0), "rows not in increasing tree position"
        inside = np.all((nodes >= lo[q]) & (nodes <= hi[q]), axis=1)
        assert sorted(got.tolist()) == sorted(p[inside].tolist()), f"box {q}"
        if with_oracle:
            assert sorted(got.tolist()) == oq.region_search(t, p, lo[q].tolist(), hi[q].tolist())


def check_bounds(nodes: np.ndarray, bounds: np.ndarray):
    """Every subtree's box is the min / max over its contiguous range."""
    nu, k = nodes.shape

    def walk(s, e):
        if e < s:
            return
        m = s + (e - s) // 2
        sub = nodes[s:e + 1]
        assert np.array_equal(bounds[m, :k], sub.min(axis=0)), (s, e)
        assert np.array_equal(bounds[m, k:], sub.max(axis=0)), (s, e)
        walk(s, m - 1)
        walk(m + 1, e)

    if nu <= 4096:
        walk(0, nu - 1)


def check_nearest(kd, t, dt, perm, nu, pts, m, with_oracle=True):
    p = perm.cpu().numpy()
    got = kd.nearest(dt, perm, nu, torch.from_numpy(pts).cuda(), m).cpu().numpy()
    for q in range(pts.shape[0]):
        want_rows, want_d = brute_nearest(t, p, pts[q], m)
        row = got[q]
        assert row[:len(want_rows)].tolist() == want_rows, f"query {q}"
        assert np.all(row[len(want_rows):] == -1)
        if with_oracle:
            qv = [int(v) for v in pts[q]] if t.dtype == np.int32 else [float(v) for v in pts[q]]
            od = [d for d, _ in oq.nearest_neighbors(t, p, qv, m)]
            assert od == want_d


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_queries_match_oracle(kd, k, dtype):
    g = kdgen.rng(900 + k)
    n = 1500
    if dtype == "i32":
        t = kdgen.uniform_int(n, k, -2**31, 2**31, 0.05, 910 + k)
    else:
        t = g.normal(size=(n, k)).astype(np.float32)
        t[g.integers(0, n, size=40)] = t[g.integers(0, n, size=40)]  # exact copies
    print(f"[gpu case] queries k={k} dtype={dtype} n={n}", flush=True)
    dt, perm, nu = gpu_tree(kd, t)
    lo, hi = boxes(g, t, 60)
    check_region(kd, t, dt, perm, nu, lo, hi)
    pts = query_points(g, t, 40)
    for m in (1, 5, 16):
        check_nearest(kd, t, dt, perm, nu, pts, m)


def test_queries_small_coordinates_with_ties(kd):
    # many equal coordinates: the non-strict pruning bounds matter
    g = kdgen.rng(931)
    t = g.integers(0, 6, size=(3000, 3)).astype(np.int32)
    print("[gpu case] queries ties n=3000", flush=True)
    dt, perm, nu = gpu_tree(kd, t)
    lo = g.integers(0, 6, size=(80, 3)).astype(np.int32)
    hi = np.minimum(lo + g.integers(0, 3, size=(80, 3)), 5).astype(np.int32)
    check_region(kd, t, dt, perm, nu, lo, hi)
    pts = g.integers(-1, 7, size=(50, 3)).astype(np.int32)
    for m in (1, 7, 64):
        check_nearest(kd, t, dt, perm, nu, pts, m)


def test_queries_degenerate_trees(kd):
    print("[gpu case] queries degenerate trees", flush=True)
    for n in (1, 2, 3, 7):
        t = kdgen.uniform_int(n, 3, -100, 100, 0.0, 940 + n)
        dt, perm, nu = gpu_tree(kd, t)
        lo = np.full((3, 3), -200, dtype=np.int32)
        hi = np.full((3, 3), 200, dtype=np.int32)
        hi[1] = -150  # empty
        check_region(kd, t, dt, perm, nu, lo, hi)
        pts = np.zeros((4, 3), dtype=np.int32)
        check_nearest(kd, t, dt, perm, nu, pts, 5)  # m > nodes: -1 padding
    # a tree of identical rows has one node
    t = np.tile(np.array([[3, 1, 4]], dtype=np.int32), (50, 1))
    dt, perm, nu = gpu_tree(kd, t)
    assert nu == 1
    check_nearest(kd, t, dt, perm, nu, np.array([[0, 0, 0]], dtype=np.int32), 3)
    # zero nodes: every count 0, every row -1
    dt = torch.from_numpy(t).cuda()
    empty = torch.zeros(1, dtype=torch.int32, device="cuda")
    c = kd.region_count(dt, empty, 0, torch.zeros((2, 3), dtype=torch.int32, device="cuda"),
                        torch.ones((2, 3), dtype=torch.int32, device="cuda"))
    assert c.cpu().tolist() == [0, 0]
    r = kd.nearest(dt, empty, 0, torch.zeros((2, 3), dtype=torch.int32, device="cuda"), 4)
    assert (r.cpu().numpy() == -1).all()
    # no queries
    assert kd.region_count(dt, perm, nu, torch.zeros((0, 3), dtype=torch.int32, device="cuda"),
                           torch.zeros((0, 3), dtype=torch.int32, device="cuda")).numel() == 0


def test_visit_counter(kd):
    t = kdgen.uniform_int(5000, 3, -2**31, 2**31, 0.0, 950)
    print("[gpu case] queries visit counter", flush=True)
    dt, perm, nu = gpu_tree(kd, t)
    v = torch.zeros(1, dtype=torch.int64, device="cuda")
    everything = np.array([[-2**31] * 3], dtype=np.int32), np.array([[2**31 - 1] * 3], dtype=np.int32)
    kd.region_count(dt, perm, nu, torch.from_numpy(everything[0]).cuda(),
                    torch.from_numpy(everything[1]).cuda(), visits=v)
    assert int(v.item()) == nu  # a box around everything visits every node once
    v.zero_()
    nodes = kd.gather_nodes(dt, perm, nu)
    c = kd.region_count(dt, perm, nu, torch.from_numpy(everything[0]).cuda(),
                        torch.from_numpy(everything[1]).cuda(), visits=v, nodes=nodes,
                        bounds=kd.subtree_bounds(nodes, nu))
    assert int(v.item()) == 1 and int(c.item()) == nu  # with bounds: the root's box is inside
    v.zero_()
    kd.nearest(dt, perm, nu, torch.from_numpy(t[:3]).cuda(), 1, visits=v)
    assert 3 <= int(v.item()) < 3 * nu


@pytest.mark.parametrize("dtype", ["i32", "f32"])
def test_queries_large_brute_force(kd, dtype):
    # 2^20 rows, 2^16 queries; 1000 boxes and 256 nearest-neighbour queries
    # of them are checked against a scan
    g = kdgen.rng(960)
    n = 1 << 20
    if dtype == "i32":
        t = kdgen.uniform_int(n, 3, -2**31, 2**31, 0.001, 961)
    else:
        t = kdgen.gaussian_mixture_f32(n, 3, 16, 962)
    print(f"[gpu case] queries large dtype={dtype} n={n}", flush=True)
    dt, perm, nu = gpu_tree(kd, t)
    p = perm.cpu().numpy()
    nodes = t[p]
    nq = 1 << 16
    lo, hi = boxes(g, t, nq)
    counts = kd.region_count(dt, perm, nu, torch.from_numpy(lo).cuda(),
                             torch.from_numpy(hi).cuda()).cpu().numpy()
    pts = query_points(g, t, nq)
    got = kd.nearest(dt, perm, nu, torch.from_numpy(pts).cuda(), 8).cpu().numpy()
    dn = kd.gather_nodes(dt, perm, nu)
    counts_b = kd.region_count(dt, perm, nu, torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda(),
                               nodes=dn, bounds=kd.subtree_bounds(dn, nu)).cpu().numpy()
    assert np.array_equal(counts_b, counts)
    # scan of each box over the nodes in the slab of its first coordinate
    # (nodes sorted by that coordinate once; every node of the slab checked)
    order = np.argsort(nodes[:, 0], kind="stable")
    by_x = nodes[order]
    for q in g.choice(nq, size=1000, replace=False):
        a = np.searchsorted(by_x[:, 0], lo[q, 0], side="left")
        b = np.searchsorted(by_x[:, 0], hi[q, 0], side="right")
        slab = by_x[a:b]
        inside = np.all((slab >= lo[q]) & (slab <= hi[q]), axis=1)
        assert counts[q] == int(inside.sum()), f"box {q}"
    for q in g.choice(nq, size=256, replace=False):
        want_rows, _ = brute_nearest_fast(t, p, pts[q], 8)
        assert got[q].tolist() == want_rows, f"query {q}"


def brute_nearest_fast(t, nodes, q, m):
    """brute_nearest over many nodes: candidates by float64 distance, then
    the exact order on a generous candidate set."""
    x = t[nodes].astype(np.float64)
    approx = ((x - q.astype(np.float64)) ** 2).sum(axis=1)
    c = max(64, 8 * m)
    cand = nodes[np.argpartition(approx, c)[:c]] if len(nodes) > c else nodes
    return brute_nearest(t, cand, q, m)


@pytest.mark.parametrize("k,dtype,n", [(3, "i32", 700), (2, "f32", 600), (5, "i32", 500),
                                       (3, "i32", 1)])
def test_all_nearest_and_reverse(kd, k, dtype, n):
    g = kdgen.rng(970 + k + n)
    if dtype == "i32":
        t = kdgen.uniform_int(n, k, -2**31, 2**31, 0.05, 971 + k)
    else:
        t = g.normal(size=(n, k)).astype(np.float32)
    print(f"[gpu case] all nearest k={k} dtype={dtype} n={n}", flush=True)
    dt, perm, nu = gpu_tree(kd, t)
    p = perm.cpu().numpy()
    m = 6
    near = kd.all_nearest(dt, perm, nu, m)
    got = near.cpu().numpy()
    assert got.shape == (n, m)
    for pos in range(nu):
        others = np.array([x for x in p if x != p[pos]], dtype=np.int64)
        want_rows, _ = brute_nearest(t, others, t[p[pos]], m)
        assert got[pos, :len(want_rows)].tolist() == want_rows, f"pos {pos}"
        assert np.all(got[pos, len(want_rows):] == -1)
    if nu >= 2:
        # distances against the oracle on a few nodes
        oq_near = [oq.nearest_neighbors(t, p, t[p[pos]].tolist(), m, exclude=int(p[pos])) for pos in range(5)]
        for pos in range(5):
            d = exact_sq_dist(t, got[pos][got[pos] >= 0], t[p[pos]])
            assert [x for x, _ in oq_near[pos]] == d
    offsets, lists = kd.reverse_nearest(perm, nu, near)
    offsets, lists = offsets.cpu().numpy(), lists.cpu().numpy()
    want = oq.reverse_lists(p, [[int(r) for r in got[pos] if r >= 0] for pos in range(nu)])
    assert offsets[0] == 0 and offsets[-1] == sum(len(v) for v in want.values())
    for r in range(n):
        assert lists[offsets[r]:offsets[r + 1]].tolist() == want.get(r, []), f"row {r}"


def test_region_with_nan_coordinates(kd):
    # a NaN coordinate is never inside a box; subtree boxes holding a NaN are
    # walked, so the counts with and without bounds agree with a scan
    g = kdgen.rng(990)
    t = g.normal(size=(4000, 3)).astype(np.float32)
    t[g.integers(0, 4000, size=400), g.integers(0, 3, size=400)] = np.nan
    t[g.integers(0, 4000, size=200), g.integers(0, 3, size=200)] = -np.nan
    print("[gpu case] region with NaN coordinates", flush=True)
    dt, perm, nu = gpu_tree(kd, t)
    p = perm.cpu().numpy()
    nodes_h = t[p]
    lo, hi = boxes(g, t[~np.isnan(t).any(axis=1)], 100)
    dn = kd.gather_nodes(dt, perm, nu)
    bounds = kd.subtree_bounds(dn, nu)
    dlo, dhi = torch.from_numpy(lo).cuda(), torch.from_numpy(hi).cuda()
    c0 = kd.region_count(dt, perm, nu, dlo, dhi, nodes=dn).cpu().numpy()
    c1 = kd.region_count(dt, perm, nu, dlo, dhi, nodes=dn, bounds=bounds).cpu().numpy()
    assert np.array_equal(c0, c1)
    for q in range(lo.shape[0]):
        with np.errstate(invalid="ignore"):
            inside = np.all((nodes_h >= lo[q]) & (nodes_h <= hi[q]), axis=1)
        assert c1[q] == int(inside.sum()), f"box {q}"


def test_reverse_lists_with_a_hub_row(kd):
    # a neighbour table in which every node names the same row: that row's
    # reverse list holds every node (sorted at L log L, not L^2)
    n, m = 1 << 18, 4
    print(f"[gpu case] reverse lists with a hub row n={n}", flush=True)
    g = kdgen.rng(995)
    perm = torch.from_numpy(g.permutation(n).astype(np.int32)).cuda()
    near = torch.from_numpy(g.integers(0, n, size=(n, m)).astype(np.int32)).cuda()
    hub = 12345
    near[:, 0] = hub
    offsets, lists = kd.reverse_nearest(perm, n, near)
    o, l = offsets.cpu().numpy(), lists.cpu().numpy()
    got = l[o[hub]:o[hub + 1]]
    nr, pm = near.cpu().numpy(), perm.cpu().numpy()
    want = np.sort(np.repeat(pm, (nr == hub).sum(axis=1)))
    assert np.array_equal(got, want)
    for r in g.choice(n, size=50, replace=False):
        want_r = np.sort(np.repeat(pm, (nr == r).sum(axis=1)))
        assert np.array_equal(l[o[r]:o[r + 1]], want_r), f"row {r}"


def test_queries_maximum_count(kd):
    """The largest query batch accepted (KD_MAX_QUERIES = 2^28), nearest
    neighbour and box counts over a 2^16-row tree, queries drawn on the GPU
    from a seeded generator; a sample of them is checked by a scan."""
    g = kdgen.rng(970)
    n, k, nq = 1 << 16, 3, 1 << 28
    t = kdgen.uniform_int(n, k, -(1 << 20), 1 << 20, 0.01, 971)
    print(f"[gpu case] queries maximum count nq={nq} n={n}", flush=True)
    dt, perm, nu = gpu_tree(kd, t)
    p = perm.cpu().numpy()
    nodes = t[p]
    tg = torch.Generator(device="cuda")
    tg.manual_seed(972)
    pts = torch.randint(-(1 << 20), 1 << 20, (nq, k), dtype=torch.int32, device="cuda", generator=tg)
    got = kd.nearest(dt, perm, nu, pts, 1)
    half = torch.randint(0, 1 << 15, (nq, k), dtype=torch.int32, device="cuda", generator=tg)
    lo, hi = pts - half, pts + half
    del half
    counts = kd.region_count(dt, perm, nu, lo, hi)
    torch.cuda.synchronize()
    sample = g.choice(nq, size=40, replace=False)
    got_s = got[torch.from_numpy(sample).cuda()].cpu().numpy()
    pts_s = pts[torch.from_numpy(sample).cuda()].cpu().numpy()
    lo_s = lo[torch.from_numpy(sample).cuda()].cpu().numpy()
    hi_s = hi[torch.from_numpy(sample).cuda()].cpu().numpy()
    counts_s = counts[torch.from_numpy(sample).cuda()].cpu().numpy()
    for i in range(len(sample)):
        want_rows, _ = brute_nearest_fast(t, p, pts_s[i], 1)
        assert got_s[i].tolist() == want_rows, f"query {sample[i]}"
        inside = np.all((nodes >= lo_s[i]) & (nodes <= hi_s[i]), axis=1)
        assert counts_s[i] == int(inside.sum()), f"box {sample[i]}"
