"""GPU parity of the comparison builder (kdtree_build_select: every level
selects each subarray's median afresh by a radix-select and partitions the
subarray about it; no presort beyond the first array, no rank records).  Its
in-order layout must equal, bit for bit, the presort builder's and the
oracle's."""
import numpy as np
import pytest

import kdgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1410_5420_amd as kd

    return kd


def check(kd, t: np.ndarray, with_oracle: bool):
    print(f"[gpu case] select n={t.shape[0]} k={t.shape[1]} dtype={t.dtype}", flush=True)
    dt = torch.from_numpy(t).cuda()
    perm_s, nu_s = kd.build_select(dt)
    perm_p, nu_p = kd.build(dt)
    assert nu_s == nu_p
    assert torch.equal(perm_s, perm_p)
    if with_oracle:
        r = oracle.build_tree(t, threads=8)
        assert nu_s == r["n_unique"]
        assert np.array_equal(perm_s.cpu().numpy().astype(np.int64), r["perm"].astype(np.int64))


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_select_matches_oracle(kd, k):
    t = kdgen.uniform_int(5000, k, -2**31, 2**31, 0.05, 1000 + k)
    check(kd, t, True)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 7, 8, 9, 1023, 1024, 1025])
def test_select_small_and_ragged(kd, n):
    t = kdgen.uniform_int(max(n, 1), 3, -50, 50, 0.2, 1100 + n)[:n]
    check(kd, np.ascontiguousarray(t), n > 0)


def test_select_float_and_ties(kd):
    g = kdgen.rng(1200)
    t = g.normal(size=(20000, 3)).astype(np.float32)
    t[g.integers(0, 20000, size=500)] = t[g.integers(0, 20000, size=500)]
    t[:200, 0] = -0.0
    t[200:400, 0] = 0.0
    check(kd, t, True)
    # coordinates with many equal values: later words of the super keys decide
    t = g.integers(0, 4, size=(30000, 4)).astype(np.int32)
    check(kd, t, True)


@pytest.mark.parametrize("k", [2, 3, 6])
def test_select_large_clustered(kd, k):
    t = kdgen.clustered_int(1 << 20, k, 256, float(1 << 12), 1 << 30, 0.10, 1300 + k)
    check(kd, t, False)


@pytest.mark.parametrize("k", [2, 3, 5, 8])
@pytest.mark.parametrize("n", [2049, 4097, 70001, 600000])
def test_select_global_levels(kd, k, n):
    """Sizes with global levels (subarrays above 2048 rows) and ragged tails."""
    t = kdgen.uniform_int(n, k, -(1 << 30), 1 << 30, 0.05, 1400 + n + k)
    check(kd, t, True)


@pytest.mark.parametrize("k", [3, 6])
def test_select_heavy_ties(kd, k):
    """Few distinct first coordinates: the median's candidates are many (digit
    rounds over word p and later words in the candidate zone), and long tie
    runs in the on-chip sorts take the full multi-word sort."""
    t = kdgen.uniform_int(300000, k, -(1 << 30), 1 << 30, 0.0, 1500 + k)
    t[:, 0] = t[:, 0] % 7
    check(kd, t, True)
    t = kdgen.uniform_int(200000, k, -3, 3, 0.0, 1510 + k)
    check(kd, t, True)


def test_select_float_mixture(kd):
    t = kdgen.gaussian_mixture_f32(500000, 3, 16, 1600)
    t[:100] = np.array([[np.inf, -0.0, 0.0]] * 100, dtype=np.float32)
    check(kd, t, True)


def test_select_c2_full_size(kd):
    """The headline input (k=3, n=2^24) through the comparison builder."""
    check(kd, kdgen.c2_full_range(), False)


@pytest.mark.parametrize("k", [2, 8])
def test_select_c3_full_size(kd, k):
    check(kd, kdgen.c3_clustered(k), False)
