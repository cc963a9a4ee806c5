"""GPU parity of level form 4 (one multi-level split per level): the HIP
build through the C ABI against the CPU oracle, bit for bit, over every
output; the status word of every build must be clean (kd.build checks it)."""
import os

import numpy as np
import pytest

import kdgen
import oracle
from test_gpu_build import assert_same, run_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1410_5420_amd as kd

    return kd


@pytest.mark.parametrize("k", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("n", [1, 7, 1000, 1025, 4097, 70001, 600000])
def test_form4_small_and_ragged(kd, k, n):
    """Trees with no global level, with fewer global levels than k - 1 (the
    first splits start from the presorted layout) and with many."""
    t = kdgen.uniform_int(n, k, -(1 << 20), 1 << 20, 0.05, 700 + n + k)
    assert_same(kd, t, cutover=1024, level=4)


@pytest.mark.parametrize("k", [3, 6, 8])
@pytest.mark.parametrize("cutover", [1024, 2048, 4096])
def test_form4_duplicates_shrink_the_tree(kd, k, cutover):
    """Duplicate removal leaves far fewer distinct rows than rows, so the
    device's global levels end above the host's bound and its last splits
    differ from the host's plan; and runs of equal first coordinates."""
    r = {3: 6, 6: 3, 8: 2}[k]
    t = kdgen.uniform_int(200000, k, -r, r, 0.0, 91 + k + cutover)
    assert_same(kd, t, cutover=cutover, level=4)
    t = kdgen.uniform_int(150000, k, -(1 << 30), 1 << 30, 0.0, 92 + k)
    t[:, 0] = t[:, 0] % 7
    assert_same(kd, t, cutover=cutover, level=4)


@pytest.mark.parametrize("k", [2, 3, 4, 6, 8])
def test_form4_c3_full_size(kd, k):
    """The dimension sweep at its full size (n=2^22, 256 Gaussian clusters,
    10% copies), children included."""
    assert_same(kd, kdgen.c3_clustered(k), threads=os.cpu_count() or 8, level=4)


def test_form4_c2_bit_exact(kd):
    """The headline workload (k=3, n=2^24) through level form 4."""
    t = kdgen.c2_full_range()
    want = oracle.build_tree(t, threads=os.cpu_count() or 8, children=False)
    perm, nu = run_gpu(kd, t, children=False, level=4)
    assert nu == want["n_unique"]
    assert np.array_equal(perm, want["perm"])


def test_form4_float_specials_and_points(kd):
    t = kdgen.gaussian_mixture_f32(300000, 3, 16, 93)
    t[:50] = np.array([[np.inf, -0.0, 0.0]] * 50, dtype=np.float32)
    t[50:60] = np.array([[-np.inf, np.nan, 1e-45]] * 10, dtype=np.float32)
    assert_same(kd, t, cutover=1024, level=4)
    x, offsets = kdgen.c4_batched(trees=1, lo=65536, hi=65536, seed=94)
    assert_same(kd, x, cutover=2048, level=4)


def test_form4_presort_then_partition(kd):
    t = kdgen.uniform_int(123457, 3, 0, 1 << 18, 0.05, 95)
    want = oracle.build_tree(t, threads=8, children=False)
    print("[gpu case] presort + partition level=4", flush=True)
    b = kd.Builder(t.shape[0], 3, torch.int32, level=4)
    dt = torch.from_numpy(t).cuda()
    perm = torch.full((t.shape[0],), -1, dtype=torch.int32, device="cuda")
    b.presort(dt)
    b.partition(dt, perm)
    assert b.status() == 0
    assert int(b.n_unique.item()) == want["n_unique"]
    assert np.array_equal(perm[: want["n_unique"]].cpu().numpy(), want["perm"])


def test_form4_workspace_reuse_shrinking(kd):
    """One workspace, a large build then a smaller one: nothing from the
    first build leaks into the second."""
    b = kd.Builder(600000, 4, torch.int32, level=4)
    for n, seed in ((600000, 96), (70001, 97), (5000, 98)):
        t = kdgen.uniform_int(n, 4, -(1 << 24), 1 << 24, 0.02, seed)
        want = oracle.build_tree(t, threads=8, children=False)
        print(f"[gpu case] reuse level=4 n={n}", flush=True)
        perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        b.build(torch.from_numpy(t).cuda(), perm)
        assert b.status() == 0
        assert int(b.n_unique.item()) == want["n_unique"]
        assert np.array_equal(perm[: want["n_unique"]].cpu().numpy(), want["perm"])
