"""GPU parity of the learned presort and its CDF model.

* the training objective and its gradient (kd_cdf_loss_grad) against the
  fp64 oracle in oracle/learned.py, whose gradient is pinned by finite
  differences;
* model evaluation (kd_cdf_eval): F and the bucket bit for bit against the
  oracle's single-precision evaluation of the same model;
* GPU training (kd_cdf_train) against the oracle's Adam on the same sample;
* learned builds against the tree oracle, bit for bit, with and without
  fallbacks, and against the plain GPU build at the full mixture size;
* what the trained model gains over the untrained (linear) map.
"""
import os

import numpy as np
import pytest

import kdgen
import oracle
from oracle import learned as L

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1410_5420_amd as kd

    return kd


def case(msg):
    print(f"[gpu case] {msg}", flush=True)


@pytest.mark.parametrize("is_float", [False, True])
def test_loss_grad_matches_oracle(kd, is_float):
    case(f"loss_grad float={is_float}")
    g = np.random.Generator(np.random.PCG64(11))
    if is_float:
        vals = kdgen.gaussian_mixture_f32(1 << 16, 1, 16, 5)[:, 0]
    else:
        vals = kdgen.clustered_int(1 << 16, 1, 32, 3000.0, 1 << 24, 0.05, 6)[:, 0]
    keys = np.sort(L.canonical(vals, is_float))
    vals_sorted = L.key_value(keys, is_float) if is_float else (keys ^ np.uint32(0x80000000)).view(np.int32)
    dm = L.Domain.of_sample(keys, is_float)
    if is_float:
        lo_raw = int(np.array([dm.lo], dtype=np.float32).view(np.uint32)[0])
        hi_raw = int(np.array([dm.hi], dtype=np.float32).view(np.uint32)[0])
    else:
        lo_raw = int(dm.kmin ^ np.uint32(0x80000000))
        hi_raw = int(dm.kmax ^ np.uint32(0x80000000))
    theta = g.normal(0, 2, size=L.K).astype(np.float32)
    t_vals = torch.from_numpy(np.ascontiguousarray(vals_sorted)).cuda()
    loss, grad = kd.cdf_loss_grad(t_vals, lo_raw, hi_raw, torch.from_numpy(theta).cuda())
    torch.cuda.synchronize()
    p = L.masses(dm, keys)
    want_loss, want_grad = L.loss_grad(theta.astype(np.float64), p)
    got = grad.cpu().numpy().astype(np.float64)
    assert float(loss.item()) == pytest.approx(want_loss, rel=1e-5, abs=1e-6)
    assert np.max(np.abs(got - want_grad)) <= 1e-7 + 1e-4 * np.max(np.abs(want_grad))


def model_bytes(c32, dm, theta):
    head = np.zeros(8, dtype=np.uint32)
    head[0] = np.float32(dm.lo).view(np.uint32)
    head[1] = np.float32(dm.hi).view(np.uint32)
    head[2] = np.float32(dm.scale).view(np.uint32)
    head[3] = dm.kmin
    head[4] = dm.kmax
    head[5] = 1 if dm.is_float else 0
    head[6] = L.K
    body = np.concatenate([c32.astype(np.float32).view(np.uint32), theta.astype(np.float32).view(np.uint32),
                           np.zeros(55, dtype=np.uint32)])
    out = np.concatenate([head, body])
    assert out.nbytes == 33024
    return out.view(np.uint8)


@pytest.mark.parametrize("is_float", [False, True])
def test_eval_bit_exact_against_oracle(kd, is_float):
    case(f"cdf_eval float={is_float}")
    g = np.random.Generator(np.random.PCG64(12))
    if is_float:
        vals = kdgen.gaussian_mixture_f32(200000, 1, 16, 8)[:, 0]
        vals[:10] = np.array([np.inf, -np.inf, np.nan, -0.0, 0.0, 1e-40, -1e-40, 3e38, -3e38, 7.0],
                             dtype=np.float32)
    else:
        vals = g.integers(-(2 ** 31), 2 ** 31, size=200000).astype(np.int32)
    keys = L.canonical(vals, is_float)
    dm = L.Domain.of_sample(np.sort(keys[10::3]), is_float)
    theta = g.normal(0, 3, size=L.K)
    c32 = L.levels(theta).astype(np.float32)
    model = torch.from_numpy(model_bytes(c32, dm, theta)).cuda()
    for nb in (1, 8, 14, 16):
        F, b = kd.cdf_eval(model, 0, torch.from_numpy(vals).cuda(), nb)
        torch.cuda.synchronize()
        wantF = L.forward_f32(c32, dm, keys)
        assert np.array_equal(F.cpu().numpy().view(np.uint32), wantF.view(np.uint32)), nb
        assert np.array_equal(b.cpu().numpy(), L.bucket(wantF, nb)), nb


def test_training_matches_oracle_adam(kd):
    case("cdf_train vs oracle")
    x = kdgen.gaussian_mixture_f32(1 << 18, 3, 64, kdgen.SEED_BASE + 5)
    S, steps, lr = 1 << 14, 300, 0.1
    models = kd.train_cdf(torch.from_numpy(x).cuda(), n_samples=S, steps=steps, lr=lr)
    torch.cuda.synchronize()
    sample = L.strided_sample(x, S)
    for d in range(3):
        rec = kd.model_record(models, d)
        sk = np.sort(L.canonical(sample[:, d], True))
        dm = L.Domain.of_column(L.canonical(x[:, d], True), True)
        assert rec["kmin"] == int(dm.kmin) and rec["kmax"] == int(dm.kmax)
        assert np.float32(rec["scale"]) == dm.scale
        p = L.masses(dm, sk)
        th = L.train_adam(p, steps, lr)
        assert np.max(np.abs(rec["c"].astype(np.float64) - L.levels(th, S))) < 2e-4, d
        assert rec["loss"] == pytest.approx(L.loss(th, p), rel=1e-3)


def oracle_tree(t):
    return oracle.build_tree(t, threads=8)


def assert_learned_same(kd, t, models=None, expect_learned=True):
    dt = torch.from_numpy(np.ascontiguousarray(t)).cuda()
    if models is None:
        models = kd.train_cdf(dt)
    perm, nu, fb, lo, hi = kd.build_learned(dt, models, children=True)
    torch.cuda.synchronize()
    want = oracle_tree(t)
    assert nu == want["n_unique"]
    assert np.array_equal(perm.cpu().numpy(), want["perm"])
    assert np.array_equal(lo.cpu().numpy(), want["lo"]) and np.array_equal(hi.cpu().numpy(), want["hi"])
    if expect_learned:
        assert fb.numpy().tolist() == [0] * t.shape[1], fb
    return fb


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("n", [1, 2, 7, 1000, 4097, 70001])
def test_learned_small(kd, k, n):
    case(f"learned n={n} k={k}")
    t = kdgen.uniform_int(n, k, -(1 << 20), 1 << 20, 0.1, 500 + n + k)
    assert_learned_same(kd, t)


@pytest.mark.parametrize("k", [2, 3, 6])
@pytest.mark.parametrize("n", [8191, 300001])
def test_learned_large_tiles(kd, k, n):
    """Every sort through the learned buckets, whose bucket passes then run
    on tiles of 8192 keys, as the bucket passes of the tuned C2 and C5 builds
    do."""
    case(f"learned sort_tile=8192 n={n} k={k}")
    t = kdgen.uniform_int(n, k, -(1 << 24), 1 << 24, 0.05, 960 + n + k)
    dt = torch.from_numpy(t).cuda()
    models = kd.train_cdf(dt)
    perm, nu, fb, lo, hi = kd.build_learned(dt, models, children=True, sort_tile=8192)
    torch.cuda.synchronize()
    want = oracle_tree(t)
    assert nu == want["n_unique"]
    assert np.array_equal(perm.cpu().numpy(), want["perm"])
    assert np.array_equal(lo.cpu().numpy(), want["lo"]) and np.array_equal(hi.cpu().numpy(), want["hi"])
    assert fb.numpy().tolist() == [0] * k, fb


@pytest.mark.parametrize("k", [3, 6])
def test_learned_deferred_partitioning(kd, k):
    """The learned presort followed by deferred partitioning (level form 3)."""
    case(f"learned deferred k={k}")
    t = kdgen.uniform_int(300001, k, -(1 << 24), 1 << 24, 0.05, 950 + k)
    dt = torch.from_numpy(t).cuda()
    models = kd.train_cdf(dt)
    b = kd.LearnedBuilder(t.shape[0], k, torch.int32, level=3)
    perm = torch.full((t.shape[0],), -1, dtype=torch.int32, device="cuda")
    b.build(dt, perm, models=models)
    torch.cuda.synchronize()
    want = oracle_tree(t)
    assert int(b.n_unique.item()) == want["n_unique"]
    assert np.array_equal(perm[: want["n_unique"]].cpu().numpy(), want["perm"])


@pytest.mark.parametrize("k", [1, 3, 8])
@pytest.mark.parametrize("n", [1000, 70001])
def test_learned_heavy_duplicates(kd, k, n):
    """100 distinct values per coordinate: long runs of equal keys may send a
    sort to the radix fallback; the tree is exact either way."""
    case(f"learned heavy duplicates n={n} k={k}")
    t = kdgen.uniform_int(n, k, -50, 50, 0.1, 900 + n + k)
    assert_learned_same(kd, t, expect_learned=False)


def test_learned_all_duplicates_fall_back(kd):
    """10000 copies of one row share one bucket, more than a workgroup holds:
    the first sort falls back to radix, and the tree is still exact."""
    case("learned all duplicates")
    t = np.tile(np.array([[5, -7, 9]], dtype=np.int32), (10000, 1))
    fb = assert_learned_same(kd, t, expect_learned=False)
    assert int(fb.numpy()[0]) & 1


def test_learned_float_specials(kd):
    case("learned float specials")
    g = np.random.Generator(np.random.PCG64(4))
    specials = np.array([0x80000000, 0x00000000, 0x7F800000, 0xFF800000, 0x7FC00000, 0xFFC00000,
                         0x00000001, 0x80000001, 0x3F800000, 0xBF800000], dtype=np.uint32).view(np.float32)
    t = g.normal(size=(60000, 3)).astype(np.float32)
    mask = g.random(size=t.shape) < 0.05
    t[mask] = g.choice(specials, size=int(mask.sum()))
    assert_learned_same(kd, np.ascontiguousarray(t), expect_learned=False)


@pytest.mark.parametrize("k", [2, 3, 6])
def test_learned_clustered(kd, k):
    """256 narrow clusters over a wide range: each cluster is much narrower
    than one model segment, so buckets can be lopsided and sorts may fall
    back; the tree is exact either way."""
    case(f"learned clustered k={k}")
    t = kdgen.clustered_int(1 << 18, k, 256, float(1 << 12), 1 << 30, 0.10, 1000 + k)
    fb = assert_learned_same(kd, t, expect_learned=False)
    print(f"fell_back {fb.numpy().tolist()}", flush=True)


def test_learned_mixture_and_c1(kd):
    case("learned mixture 2^20, C1")
    assert_learned_same(kd, kdgen.gaussian_mixture_f32(1 << 20, 3, 64, kdgen.SEED_BASE + 5))
    assert_learned_same(kd, kdgen.c1_small_uniform())


def test_untrained_model_falls_back_and_stays_exact(kd):
    """steps = 0 leaves the linear map, under which the mixture overflows
    buckets: the sorts fall back to radix and the tree is still exact."""
    case("learned untrained fallback")
    x = kdgen.gaussian_mixture_f32(1 << 21, 3, 64, kdgen.SEED_BASE + 5)
    dx = torch.from_numpy(x).cuda()
    fb = assert_learned_same(kd, x, models=kd.train_cdf(dx, steps=0), expect_learned=False)
    assert int(fb.numpy()[0]) & 1, fb


def test_trained_model_gain(kd):
    """On the mixture the trained model keeps every bucket within a few
    shares (no fallback); the untrained map overflows the on-chip capacity."""
    case("learned gain 2^22")
    x = kdgen.gaussian_mixture_f32(1 << 22, 3, 64, kdgen.SEED_BASE + 5)
    dx = torch.from_numpy(x).cuda()
    nb = 12  # buckets the build uses at 2^22 rows (about 1024 keys each)
    trained = kd.train_cdf(dx)
    untrained = kd.train_cdf(dx, steps=0)
    mean = x.shape[0] / (1 << nb)
    for d in range(3):
        col = dx[:, d].contiguous()
        _, bt = kd.cdf_eval(trained, d, col, nb)
        _, bu = kd.cdf_eval(untrained, d, col, nb)
        ct = torch.bincount(bt.long(), minlength=1 << nb).max().item()
        cu = torch.bincount(bu.long(), minlength=1 << nb).max().item()
        print(f"dim {d}: fullest bucket trained {ct} untrained {cu} (mean {mean:.0f})", flush=True)
        assert ct < 4 * mean
        assert cu > 8192
    b = kd.LearnedBuilder(x.shape[0], 3, torch.float32)
    perm = torch.empty(x.shape[0], dtype=torch.int32, device="cuda")
    b.build(dx, perm, models=trained)
    torch.cuda.synchronize()
    assert b.fell_back.cpu().numpy().tolist() == [0, 0, 0]


def test_learned_equals_plain_full_mixture(kd):
    """The learned-presort workload (k=3, n=2^26 float32 mixture): the learned
    build against the plain GPU build (itself checked bit for bit against
    the oracle at full size), every output compared."""
    case("learned vs plain 2^26")
    x = kdgen.c5_mixture()
    dx = torch.from_numpy(x).cuda()
    del x
    n = dx.shape[0]
    models = kd.train_cdf(dx)
    lb = kd.LearnedBuilder(n, 3, torch.float32)
    pl = torch.empty(n, dtype=torch.int32, device="cuda")
    lb.build(dx, pl, models=models)
    torch.cuda.synchronize()
    assert lb.fell_back.cpu().numpy().tolist() == [0, 0, 0]
    nu = int(lb.n_unique.item())
    del lb
    pb = kd.Builder(n, 3, torch.float32)
    pp = torch.empty(n, dtype=torch.int32, device="cuda")
    pb.build(dx, pp)
    torch.cuda.synchronize()
    assert int(pb.n_unique.item()) == nu
    assert torch.equal(pl[:nu], pp[:nu])
