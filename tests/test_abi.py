"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/kdtree.h declares, sizes workspaces, and rejects bad arguments on the
host before any HIP call (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kdtree.h")


@pytest.fixture(scope="module")
def L():
    from paper_1410_5420_amd import _lib

    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kd\w*)\s*\(", text)))


def test_header_declarations_are_exported(L):
    names = declared_functions()
    assert "kdtree_build" in names and len(names) >= 5
    for name in names:
        assert hasattr(L.lib, name), f"{name} declared in kdtree.h but not exported"
    assert sorted(L.EXPORTED) == names


def test_only_declared_functions_have_c_linkage(L):
    """The library's unmangled exports are exactly the header's functions:
    internal helpers are not exported with C linkage."""
    import shutil
    import subprocess

    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("no nm")
    out = subprocess.run([nm, "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = sorted({ln.split()[-1] for ln in out.splitlines()
                       if ln.split()[1:2] == ["T"] and not ln.split()[-1].startswith(("_Z", "_"))})
    assert exported == declared_functions()


def test_workspace_bytes(L):
    small = L.workspace_bytes(4096, 3, L.KD_I32)
    big = L.workspace_bytes(1 << 24, 3, L.KD_I32)
    assert 0 < small < big
    assert L.workspace_bytes(0, 3, L.KD_I32) > 0
    out = ctypes.c_size_t(0)
    assert L.lib.kdtree_workspace_bytes(-1, 3, 0, ctypes.byref(out)) == -1
    assert L.lib.kdtree_workspace_bytes(10, 9, 0, ctypes.byref(out)) == -4
    assert L.lib.kdtree_workspace_bytes(10, 3, 7, ctypes.byref(out)) == -1
    assert L.lib.kdtree_workspace_bytes(1 << 30, 3, 0, ctypes.byref(out)) == -4


FAKE = 0x7F0000000000  # never dereferenced: every call below fails validation first
FAKE8 = 1 << 20  # an 8-byte aligned stand-in address (never dereferenced)


def call_build(L, n=100, k=3, dtype=0, tuples=FAKE, perm=FAKE, lo=None, hi=None, nu=FAKE, ws=FAKE,
               ws_bytes=None, opts=None):
    if ws_bytes is None:
        ws_bytes = L.workspace_bytes(max(n, 0), max(min(k, 8), 1), 0) if 0 <= n < (1 << 30) else 0
    vp = ctypes.c_void_p
    return L.lib.kdtree_build(vp(tuples), n, k, dtype, vp(perm), vp(lo), vp(hi), vp(nu), vp(ws),
                              ws_bytes, opts, None)


def test_build_rejects_bad_arguments(L):
    assert call_build(L, k=0) == -1
    assert call_build(L, k=9) == -4
    assert call_build(L, n=-5) == -1
    assert call_build(L, n=1 << 30) == -4
    assert call_build(L, dtype=2) == -1
    assert call_build(L, tuples=0) == -1
    assert call_build(L, ws=0) == -1
    assert call_build(L, perm=0) == -1
    assert call_build(L, nu=0) == -1
    assert call_build(L, lo=FAKE) == -1          # lo without hi
    assert call_build(L, tuples=FAKE + 2) == -1  # misaligned
    assert call_build(L, ws_bytes=16) == -2
    o = L.kd_options()
    o.cutover = 3000
    assert call_build(L, opts=ctypes.byref(o)) == -1
    o.cutover = 2048
    o.leaf_blocks = 100  # below the accepted range
    assert call_build(L, opts=ctypes.byref(o)) == -1
    o.leaf_blocks = 20000  # above it
    assert call_build(L, opts=ctypes.byref(o)) == -1
    o.leaf_blocks = 0
    o.records = 3  # 0, 1 or 2
    assert call_build(L, opts=ctypes.byref(o)) == -1
    o.records = 0
    o.level = 5  # 0 .. 4
    assert call_build(L, opts=ctypes.byref(o)) == -1
    o.level = 0
    o.digit_bits = 10  # 8 or 11
    assert call_build(L, opts=ctypes.byref(o)) == -1
    o.digit_bits = 0
    o.sort_tile = 2048  # 4096 or 8192
    assert call_build(L, opts=ctypes.byref(o)) == -1
    o.sort_tile = 0
    o.reserved[0] = 1  # reserved words must be zero
    assert call_build(L, opts=ctypes.byref(o)) == -1


def test_learned_and_training_reject_bad_arguments(L):
    vp = ctypes.c_void_p
    out = ctypes.c_size_t(0)
    assert L.lib.kd_cdf_model_bytes(0, ctypes.byref(out)) == -1
    assert L.lib.kd_cdf_model_bytes(9, ctypes.byref(out)) == -4
    assert L.lib.kd_cdf_model_bytes(3, ctypes.byref(out)) == 0 and out.value == 3 * L.CDF_MODEL_BYTES
    assert L.lib.kd_cdf_train_workspace_bytes(3, 0, ctypes.byref(out)) == -1
    assert L.lib.kd_cdf_train_workspace_bytes(3, (1 << 20) + 1, ctypes.byref(out)) == -4
    ws = 1 << 30
    # n < 1, bad steps, non-positive learning rate, null model: rejected before any launch
    assert L.lib.kd_cdf_train(vp(FAKE), 0, 3, 0, 0, 1024, 10, 0.1, vp(FAKE), vp(FAKE), ws, None) == -1
    assert L.lib.kd_cdf_train(vp(FAKE), 100, 3, 0, 0, 1024, -1, 0.1, vp(FAKE), vp(FAKE), ws, None) == -1
    assert L.lib.kd_cdf_train(vp(FAKE), 100, 3, 0, 0, 1024, 10, 0.0, vp(FAKE), vp(FAKE), ws, None) == -1
    assert L.lib.kd_cdf_train(vp(FAKE), 100, 3, 0, 0, 1024, 10, 0.1, None, vp(FAKE), ws, None) == -1
    assert L.lib.kd_cdf_train(vp(FAKE), 100, 3, 0, 0, 1024, 10, 0.1, vp(FAKE), vp(FAKE), 8, None) == -2
    # model kinds: only the piecewise-linear model (0) is built; the MLP (1)
    # and unknown kinds are refused before any launch
    assert L.lib.kd_cdf_train(vp(FAKE), 100, 3, 0, L.KD_CDF_MLP, 1024, 10, 0.1, vp(FAKE), vp(FAKE), ws,
                              None) == L.KD_EUNSUPPORTED
    assert L.lib.kd_cdf_train(vp(FAKE), 100, 3, 0, 7, 1024, 10, 0.1, vp(FAKE), vp(FAKE), ws,
                              None) == L.KD_EUNSUPPORTED
    assert L.lib.kd_cdf_eval(vp(FAKE), vp(FAKE), 10, 17, vp(FAKE), vp(FAKE), None) == -1
    assert L.lib.kd_cdf_loss_grad(vp(FAKE), 0, 0, 0, 1, vp(FAKE), vp(FAKE), vp(FAKE), vp(FAKE), None) == -1
    assert L.lib.kdtree_workspace_bytes_learned(-1, 3, 0, ctypes.byref(out)) == -1
    assert L.lib.kdtree_workspace_bytes_learned(100, 3, 0, ctypes.byref(out)) == 0
    learned_ws = out.value
    assert L.lib.kdtree_workspace_bytes(100, 3, 0, ctypes.byref(out)) == 0
    assert learned_ws > out.value
    nu = FAKE
    # no models; too small a workspace
    assert L.lib.kdtree_build_learned(vp(FAKE), 100, 3, 0, None, vp(FAKE), None, None, vp(nu), None,
                                      vp(FAKE), learned_ws, None, None) == -1
    assert L.lib.kdtree_build_learned(vp(FAKE), 100, 3, 0, vp(FAKE), vp(FAKE), None, None, vp(nu),
                                      None, vp(FAKE), out.value, None, None) == -2


def test_strerror(L):
    for code in (0, -1, -2, -3, -4, -5):
        assert L.lib.kd_strerror(code) and L.lib.kd_strerror(code) != b"unknown status"
    assert L.lib.kd_strerror(-99) == b"unknown status"


def test_status_rejects_bad_arguments(L):
    """kd_status validates before it touches the stream or the device."""
    vp = ctypes.c_void_p
    bits = ctypes.c_uint32(0)
    assert L.lib.kd_status(None, 1024, ctypes.byref(bits), None) == -1
    assert L.lib.kd_status(vp(FAKE + 2), 1024, ctypes.byref(bits), None) == -1
    assert L.lib.kd_status(vp(FAKE), 1024, None, None) == -1
    assert L.lib.kd_status(vp(FAKE), 8, ctypes.byref(bits), None) == -2


def test_probe_rejects_bad_class(L):
    assert L.lib.kd_probe_start(0, 10) == -1
    assert L.lib.kd_probe_start(2, 0) == -1


def test_queries_reject_bad_arguments(L):
    """Tree searches: every bad size, dtype, alignment or null pointer is
    caught on the host (nothing reaches the device, so the fake pointers are
    never dereferenced)."""
    vp = ctypes.c_void_p
    F, F8 = vp(FAKE), vp(FAKE8)
    # gathering the node coordinates: bad k, dtype, n; null perm, count, output
    assert L.lib.kd_gather_nodes(F, 100, 0, 0, F, F8, F, None) == -1
    assert L.lib.kd_gather_nodes(F, 100, 9, 0, F, F8, F, None) == -4
    assert L.lib.kd_gather_nodes(F, 100, 3, 2, F, F8, F, None) == -1
    assert L.lib.kd_gather_nodes(F, -1, 3, 0, F, F8, F, None) == -1
    assert L.lib.kd_gather_nodes(F, 100, 3, 0, None, F8, F, None) == -1
    assert L.lib.kd_gather_nodes(F, 100, 3, 0, F, None, F, None) == -1
    assert L.lib.kd_gather_nodes(F, 100, 3, 0, F, F8, None, None) == -1
    assert L.lib.kd_gather_nodes(F, 100, 3, 0, F, vp(FAKE8 + 4), F, None) == -1
    assert L.lib.kd_gather_nodes(F, 0, 3, 0, F, F8, None, None) == 0  # no rows: nothing to do
    # region counts: bad k, dtype, n, nq; null and misaligned pointers
    assert L.lib.kd_region_count(F, None, 100, 0, 0, F8, F, F, 10, F, None, None) == -1
    assert L.lib.kd_region_count(F, None, 100, 9, 0, F8, F, F, 10, F, None, None) == -4
    assert L.lib.kd_region_count(F, None, 100, 3, 2, F8, F, F, 10, F, None, None) == -1
    assert L.lib.kd_region_count(F, None, -1, 3, 0, F8, F, F, 10, F, None, None) == -1
    assert L.lib.kd_region_count(F, None, 100, 3, 0, F8, F, F, -1, F, None, None) == -1
    assert L.lib.kd_region_count(F, None, 100, 3, 0, F8, F, F, (1 << 28) + 1, F, None, None) == -4
    assert L.lib.kd_region_count(None, None, 100, 3, 0, F8, F, F, 10, F, None, None) == -1
    assert L.lib.kd_region_count(F, None, 100, 3, 0, None, F, F, 10, F, None, None) == -1
    assert L.lib.kd_region_count(F, None, 100, 3, 0, F8, None, F, 10, F, None, None) == -1
    assert L.lib.kd_region_count(F, None, 100, 3, 0, F8, F, F, 10, None, None, None) == -1
    assert L.lib.kd_region_count(vp(FAKE + 2), None, 100, 3, 0, F8, F, F, 10, F, None, None) == -1
    assert L.lib.kd_region_count(F, None, 100, 3, 0, vp(FAKE8 + 4), F, F, 10, F, None, None) == -1
    assert L.lib.kd_region_count(F, None, 100, 3, 0, F8, F, F, 10, F, vp(FAKE8 + 4), None) == -1
    # no queries: nothing to do
    assert L.lib.kd_region_count(F, None, 100, 3, 0, F8, None, None, 0, None, None, None) == 0
    # region rows: null perm, negative capacity, null offsets, rows null with a capacity
    assert L.lib.kd_region_rows(F, None, 100, 3, 0, None, F8, F, F, 10, F8, F, 10, None, None) == -1
    assert L.lib.kd_region_rows(F, None, 100, 3, 0, F, F8, F, F, 10, F8, F, -1, None, None) == -1
    assert L.lib.kd_region_rows(F, None, 100, 3, 0, F, F8, F, F, 10, None, F, 10, None, None) == -1
    assert L.lib.kd_region_rows(F, None, 100, 3, 0, F, F8, F, F, 10, F8, None, 10, None, None) == -1
    assert L.lib.kd_region_rows(F, None, 100, 3, 0, F, F8, F, F, 10, vp(FAKE8 + 4), F, 10, None, None) == -1
    # nearest: null perm, m out of range, null points or rows
    assert L.lib.kd_nearest(F, 100, 3, 0, None, F8, F, 10, 4, F, None, None) == -1
    assert L.lib.kd_nearest(F, 100, 3, 0, F, F8, F, 10, 0, F, None, None) == -1
    assert L.lib.kd_nearest(F, 100, 3, 0, F, F8, F, 10, 65, F, None, None) == -1
    assert L.lib.kd_nearest(F, 100, 3, 0, F, F8, None, 10, 4, F, None, None) == -1
    assert L.lib.kd_nearest(F, 100, 3, 0, F, F8, F, 10, 4, None, None, None) == -1
    assert L.lib.kd_nearest(F, 100, 3, 1, F, F8, F, 0, 4, None, None, None) == 0
    # subtree bounds: null output, misaligned bounds given to a search
    assert L.lib.kd_subtree_bounds(F, 100, 3, 0, F8, None, None) == -1
    assert L.lib.kd_subtree_bounds(F, 100, 9, 0, F8, F, None) == -4
    assert L.lib.kd_subtree_bounds(F, 0, 3, 0, F8, None, None) == 0
    assert L.lib.kd_region_count(F, vp(FAKE + 2), 100, 3, 0, F8, F, F, 10, F, None, None) == -1
    assert L.lib.kd_probe_start(11, 10) == -1


def test_all_nearest_and_reverse_reject_bad_arguments(L):
    vp = ctypes.c_void_p
    F, F8 = vp(FAKE), vp(FAKE8)
    out = ctypes.c_size_t(0)
    assert L.lib.kd_all_nearest(F, 100, 3, 0, F, F8, 0, F, None, None) == -1
    assert L.lib.kd_all_nearest(F, 100, 3, 0, F, F8, 65, F, None, None) == -1
    assert L.lib.kd_all_nearest(F, 100, 3, 0, None, F8, 4, F, None, None) == -1
    assert L.lib.kd_all_nearest(F, 100, 3, 0, F, F8, 4, None, None, None) == -1
    assert L.lib.kd_all_nearest(F, 0, 3, 0, F, F8, 4, None, None, None) == 0
    assert L.lib.kd_reverse_workspace_bytes(-1, ctypes.byref(out)) == -1
    assert L.lib.kd_reverse_workspace_bytes(1 << 20, ctypes.byref(out)) == 0 and out.value >= 4 << 20
    need = out.value
    assert L.lib.kd_reverse_nearest(F, F8, 1 << 20, 0, F, F8, F, F8, need, None) == -1
    assert L.lib.kd_reverse_nearest(None, F8, 1 << 20, 4, F, F8, F, F8, need, None) == -1
    assert L.lib.kd_reverse_nearest(F, F8, 1 << 20, 4, F, vp(FAKE8 + 4), F, F8, need, None) == -1
    assert L.lib.kd_reverse_nearest(F, F8, 1 << 20, 4, F, F8, F, F8, need - 8, None) == -2
    assert L.lib.kd_reverse_nearest(F, F8, 0, 4, None, None, None, None, 0, None) == 0


def test_select_build_rejects_bad_arguments(L):
    vp = ctypes.c_void_p
    out = ctypes.c_size_t(0)
    assert L.lib.kdtree_workspace_bytes(100, 3, 0, ctypes.byref(out)) == 0
    ws = out.value
    nu = FAKE
    assert L.lib.kdtree_build_select(vp(FAKE), 100, 0, 0, vp(FAKE), vp(nu), vp(FAKE), ws, None, None) == -1
    assert L.lib.kdtree_build_select(vp(FAKE), 100, 9, 0, vp(FAKE), vp(nu), vp(FAKE), ws, None, None) == -4
    assert L.lib.kdtree_build_select(vp(FAKE), 100, 3, 2, vp(FAKE), vp(nu), vp(FAKE), ws, None, None) == -1
    assert L.lib.kdtree_build_select(vp(FAKE), 100, 3, 0, None, vp(nu), vp(FAKE), ws, None, None) == -1
    assert L.lib.kdtree_build_select(vp(FAKE), 100, 3, 0, vp(FAKE), vp(nu), vp(FAKE), ws - 8, None, None) == -2
