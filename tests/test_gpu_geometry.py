"""GPU parity of the radix geometries the autotuner sweeps: digit width 8 or
11 bits (four or three passes per key word) and tiles of 4096 or 8192 keys.
Every build is compared with the oracle bit for bit; the knobs change speed
only."""
import os

import numpy as np
import pytest

import kdgen
import oracle
from test_gpu_build import assert_same, assert_batched_same

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GEOMS = [(8, 8192), (11, 4096), (11, 8192)]


@pytest.fixture(scope="module")
def kd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1410_5420_amd as kd

    return kd


@pytest.mark.parametrize("bits,tile", GEOMS)
@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("n", [1, 4097, 70001, 600000])
def test_geometry_same_tree(kd, bits, tile, k, n):
    t = kdgen.uniform_int(n, k, -2**31, 2**31, 0.03, 1700 + n + k)
    assert_same(kd, t, digit_bits=bits, sort_tile=tile)


@pytest.mark.parametrize("bits,tile", GEOMS)
def test_geometry_long_runs_take_the_complete_sort(kd, bits, tile):
    """Runs of equal first words longer than the tie step takes: the gated
    complete sort of array 0 runs (word 0 at the chosen width, the other
    words at 8 bits) and must end in the same buffers."""
    for k in (2, 3, 4):
        t = kdgen.uniform_int(60000, k, -(1 << 20), 1 << 20, 0.02, 1800 + k)
        t[:, 0] = 5
        assert_same(kd, t, digit_bits=bits, sort_tile=tile)


@pytest.mark.parametrize("bits,tile", GEOMS)
def test_geometry_complete_sort_at_size(kd, bits, tile):
    """The gated complete sort over 1.2 M rows: more tiles than its
    workgroups (each walks several) and several groups of 64 tiles, whose
    scans the counts' last workgroups do, at every digit width (2048 digits
    per tile at 11 bits)."""
    t = kdgen.uniform_int(1_200_000, 3, -(1 << 20), 1 << 20, 0.02, 1850)
    t[:, 0] = 7
    print(f"[gpu case] complete sort n=1.2M bits={bits} tile={tile}", flush=True)
    assert_same(kd, t, digit_bits=bits, sort_tile=tile)


@pytest.mark.parametrize("bits,tile", GEOMS)
def test_geometry_floats_and_forest(kd, bits, tile):
    t = kdgen.gaussian_mixture_f32(200000, 3, 16, 1900)
    t[:30] = np.array([[np.inf, -0.0, np.nan]] * 30, dtype=np.float32)
    assert_same(kd, t, digit_bits=bits, sort_tile=tile)
    x, offsets = kdgen.c4_batched(trees=64, lo=64, hi=65536, seed=1901)
    assert_batched_same(kd, x, offsets, digit_bits=bits, sort_tile=tile)


def test_geometry_c2_full_size(kd):
    """The headline input with 11-bit digits and 8192-key tiles."""
    t = kdgen.c2_full_range()
    want = oracle.build_tree(t, threads=os.cpu_count() or 8, children=False)
    dt = torch.from_numpy(t).cuda()
    print("[gpu case] c2 bits=11 tile=8192", flush=True)
    perm, nu = kd.build(dt, digit_bits=11, sort_tile=8192)
    assert nu == want["n_unique"]
    assert np.array_equal(perm.cpu().numpy(), want["perm"])


@pytest.mark.parametrize("bits", [8, 11])
def test_geometry_learned(kd, bits):
    x = kdgen.gaussian_mixture_f32(300000, 3, 16, 2000)
    dx = torch.from_numpy(x).cuda()
    models = kd.train_cdf(dx)
    want = oracle.build_tree(x, threads=8, children=False)
    print(f"[gpu case] learned bits={bits}", flush=True)
    perm, nu, fb = kd.build_learned(dx, models, digit_bits=bits, sort_tile=8192)
    assert nu == want["n_unique"]
    assert np.array_equal(perm.cpu().numpy(), want["perm"])
