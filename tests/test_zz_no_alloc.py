"""kdtree_build_noalloc (the build for callers that cannot allocate device
memory; its workspace is a device array inside the library) against
kdtree_build with a caller workspace: every output equal, on two calls in a
row, the second with a smaller input (the array keeps the first call's
contents, which the second must not see)."""
import ctypes

import numpy as np
import pytest

import kdgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1410_5420_amd as kd

    return kd


def _noalloc(kd, t):
    from paper_1410_5420_amd import _lib

    n, k = t.shape
    code = _lib.KD_F32 if t.dtype == torch.float32 else _lib.KD_I32
    perm = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    lo = torch.full_like(perm, -2)
    hi = torch.full_like(perm, -2)
    nu = torch.zeros(1, dtype=torch.int64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    vp = ctypes.c_void_p
    rc = _lib.lib.kdtree_build_noalloc(vp(t.data_ptr()), n, k, code, vp(perm.data_ptr()),
                                       vp(lo.data_ptr()), vp(hi.data_ptr()), vp(nu.data_ptr()),
                                       None, stream)
    assert rc == 0, _lib.lib.kd_strerror(rc)
    torch.cuda.synchronize()
    u = int(nu.item())
    return perm[:u].cpu().numpy(), u, lo[:u].cpu().numpy(), hi[:u].cpu().numpy()


def _with_workspace(kd, t):
    perm, nu, lo, hi = kd.build(t, children=True)
    return perm.cpu().numpy(), nu, lo.cpu().numpy(), hi.cpu().numpy()


@pytest.mark.parametrize("first,second", [
    ((400000, 3, "i32"), (5000, 3, "i32")),
    ((100000, 5, "f32"), (4097, 2, "i32")),
])
def test_noalloc_equals_build_on_two_calls(kd, first, second):
    for n, k, dt in (first, second):
        print(f"[gpu case] noalloc n={n} k={k} {dt}", flush=True)
        if dt == "i32":
            x = kdgen.uniform_int(n, k, -(1 << 20), 1 << 20, 0.05, 31 * n + k)
        else:
            x = kdgen.gaussian_mixture_f32(n, k, 8, 31 * n + k)
        t = torch.from_numpy(x).cuda()
        got = _noalloc(kd, t)
        want = _with_workspace(kd, t)
        assert got[1] == want[1]
        for a, b in zip(got, want):
            assert np.array_equal(np.asarray(a), np.asarray(b))


def test_noalloc_refuses_inputs_beyond_its_array(kd):
    from paper_1410_5420_amd import _lib

    n = 4 << 20
    assert _lib.workspace_bytes(n, 3, 0) > _lib.KD_NOALLOC_WORKSPACE_BYTES
    vp = ctypes.c_void_p
    rc = _lib.lib.kdtree_build_noalloc(vp(1 << 20), n, 3, 0, vp(1 << 20), None, None, vp(1 << 20),
                                       None, None)
    assert rc == -2  # KD_ENOMEM, before anything touches the device
