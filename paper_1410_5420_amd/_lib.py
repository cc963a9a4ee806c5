"""ctypes binding of libkdtree.so (the gfx950 HIP library).

Argument marshalling only: every step of a build runs in the library's
kernels.  If the library has not been built the import fails loudly; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkdtree.so")

KD_OK = 0
KD_EUNSUPPORTED = -4
KD_EINTERNAL = -5
KD_I32 = 0
KD_F32 = 1
KD_NOALLOC_WORKSPACE_BYTES = 64 << 20
KD_CDF_PWL = 0
KD_CDF_MLP = 1


class KdError(RuntimeError):
    pass


class kd_options(ctypes.Structure):
    _fields_ = [("cutover", ctypes.c_int32), ("leaf_blocks", ctypes.c_int32),
                ("records", ctypes.c_int32), ("learned_sorts", ctypes.c_int32),
                ("level", ctypes.c_int32), ("digit_bits", ctypes.c_int32),
                ("sort_tile", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: the HIP library has not been built "
            "(run `python -c 'import __graft_entry__ as g; g.build()'`)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    opt = ctypes.POINTER(kd_options)
    lib.kd_strerror.argtypes = [ctypes.c_int]
    lib.kd_strerror.restype = ctypes.c_char_p
    lib.kd_status.argtypes = [vp, sz, ctypes.POINTER(ctypes.c_uint32), vp]
    lib.kd_status.restype = ctypes.c_int
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.kd_level_plan.argtypes = [i32, i32, u32p, u32p]
    lib.kd_level_plan.restype = ctypes.c_int
    lib.kd_level_masks.argtypes = [i32, i32, i32, ctypes.POINTER(ctypes.c_uint64),
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.kd_level_masks.restype = ctypes.c_int
    lib.kdtree_workspace_bytes.argtypes = [i64, i32, i32, ctypes.POINTER(sz)]
    lib.kdtree_workspace_bytes.restype = ctypes.c_int
    lib.kdtree_build.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp, vp, sz, opt, vp]
    lib.kdtree_build.restype = ctypes.c_int
    lib.kdtree_build_noalloc.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp, opt, vp]
    lib.kdtree_build_noalloc.restype = ctypes.c_int
    lib.kdtree_presort.argtypes = [vp, i64, i32, i32, vp, vp, sz, opt, vp]
    lib.kdtree_presort.restype = ctypes.c_int
    lib.kdtree_partition.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp, vp, sz, opt, vp]
    lib.kdtree_partition.restype = ctypes.c_int
    lib.kdtree_build_select.argtypes = [vp, i64, i32, i32, vp, vp, vp, sz, opt, vp]
    lib.kdtree_build_select.restype = ctypes.c_int
    lib.kdtree_workspace_bytes_batched.argtypes = [i64, i32, i32, i32, ctypes.POINTER(sz)]
    lib.kdtree_workspace_bytes_batched.restype = ctypes.c_int
    lib.kdtree_build_batched.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, sz, opt, vp]
    lib.kdtree_build_batched.restype = ctypes.c_int
    u32, fp = ctypes.c_uint32, ctypes.c_float
    lib.kd_cdf_model_bytes.argtypes = [i32, ctypes.POINTER(sz)]
    lib.kd_cdf_model_bytes.restype = ctypes.c_int
    lib.kd_cdf_train_workspace_bytes.argtypes = [i32, i32, ctypes.POINTER(sz)]
    lib.kd_cdf_train_workspace_bytes.restype = ctypes.c_int
    lib.kd_cdf_train.argtypes = [vp, i64, i32, i32, i32, i32, i32, fp, vp, vp, sz, vp]
    lib.kd_cdf_train.restype = ctypes.c_int
    lib.kd_cdf_loss_grad.argtypes = [vp, i32, i32, u32, u32, vp, vp, vp, vp, vp]
    lib.kd_cdf_loss_grad.restype = ctypes.c_int
    lib.kd_cdf_eval.argtypes = [vp, vp, i32, i32, vp, vp, vp]
    lib.kd_cdf_eval.restype = ctypes.c_int
    lib.kdtree_workspace_bytes_learned.argtypes = [i64, i32, i32, ctypes.POINTER(sz)]
    lib.kdtree_workspace_bytes_learned.restype = ctypes.c_int
    lib.kdtree_build_learned.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp, vp, vp, vp, sz, opt, vp]
    lib.kdtree_build_learned.restype = ctypes.c_int
    lib.kdtree_presort_learned.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp, sz, opt, vp]
    lib.kdtree_presort_learned.restype = ctypes.c_int
    lib.kd_gather_nodes.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp]
    lib.kd_gather_nodes.restype = ctypes.c_int
    lib.kd_subtree_bounds.argtypes = [vp, i64, i32, i32, vp, vp, vp]
    lib.kd_subtree_bounds.restype = ctypes.c_int
    lib.kd_region_count.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp, i64, vp, vp, vp]
    lib.kd_region_count.restype = ctypes.c_int
    lib.kd_region_rows.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp, vp, i64, vp, vp, i64, vp, vp]
    lib.kd_region_rows.restype = ctypes.c_int
    lib.kd_nearest.argtypes = [vp, i64, i32, i32, vp, vp, vp, i64, i32, vp, vp, vp]
    lib.kd_nearest.restype = ctypes.c_int
    lib.kd_all_nearest.argtypes = [vp, i64, i32, i32, vp, vp, i32, vp, vp, vp]
    lib.kd_all_nearest.restype = ctypes.c_int
    lib.kd_reverse_workspace_bytes.argtypes = [i64, ctypes.POINTER(sz)]
    lib.kd_reverse_workspace_bytes.restype = ctypes.c_int
    lib.kd_reverse_nearest.argtypes = [vp, vp, i64, i32, vp, vp, vp, vp, sz, vp]
    lib.kd_reverse_nearest.restype = ctypes.c_int
    lib.kd_probe_start.argtypes = [i32, i32]
    lib.kd_probe_start.restype = ctypes.c_int
    lib.kd_probe_stop.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32)]
    lib.kd_probe_stop.restype = ctypes.c_int
    return lib


lib = _load()

# Every symbol include/kdtree.h declares (the tests check the library exports them).
EXPORTED = ["kd_strerror", "kd_status", "kd_level_plan", "kd_level_masks", "kdtree_workspace_bytes", "kdtree_build",
            "kdtree_build_noalloc", "kdtree_presort",
            "kdtree_partition", "kdtree_build_select", "kdtree_workspace_bytes_batched",
            "kdtree_build_batched",
            "kd_cdf_model_bytes", "kd_cdf_train_workspace_bytes", "kd_cdf_train",
            "kd_cdf_loss_grad", "kd_cdf_eval", "kdtree_workspace_bytes_learned",
            "kdtree_build_learned", "kdtree_presort_learned", "kd_gather_nodes", "kd_subtree_bounds",
            "kd_region_count",
            "kd_region_rows", "kd_nearest", "kd_all_nearest", "kd_reverse_workspace_bytes",
            "kd_reverse_nearest", "kd_probe_start", "kd_probe_stop"]

KERNEL_CLASSES = {"onesweep": 1, "level": 2, "leaf": 3, "dedup": 4, "hist": 5, "canon": 6,
                  "records": 7, "bucket": 8, "ties": 9, "query": 10}

MAX_NEIGHBORS = 64

CDF_SEGMENTS = 4096
CDF_MODEL_BYTES = 33024


def probe_start(kernel: str, capacity: int) -> None:
    check(lib.kd_probe_start(KERNEL_CLASSES[kernel], capacity), "kd_probe_start")


def probe_stop(capacity: int):
    buf = (ctypes.c_float * capacity)()
    cnt = ctypes.c_int32(0)
    check(lib.kd_probe_stop(buf, ctypes.byref(cnt)), "kd_probe_stop")
    return [float(buf[i]) for i in range(cnt.value)]


def status(workspace_ptr, workspace_bytes: int, stream_ptr) -> int:
    """The status bits of the last build enqueued with a workspace
    (kd_status: waits for the stream); raises KdError when one is set."""
    bits = ctypes.c_uint32(0)
    rc = lib.kd_status(workspace_ptr, workspace_bytes, ctypes.byref(bits), stream_ptr)
    if rc != KD_OK:
        raise KdError(f"kd_status: {lib.kd_strerror(rc).decode()} ({rc}), bits {bits.value:#x}")
    return int(bits.value)


def level_plan(k: int, levels: int):
    """(level masks, final masks) of level form 4 (kd_level_plan, host only)."""
    lm = (ctypes.c_uint32 * max(levels, 1))()
    fm = (ctypes.c_uint32 * k)()
    check(lib.kd_level_plan(k, levels, lm, fm), "kd_level_plan")
    return [int(lm[i]) for i in range(levels)], [int(fm[j]) for j in range(k)]


def level_masks(k: int, levels: int, defer: int):
    """(write masks per level, moves per (depth, array)) of level forms 1 and
    3 (kd_level_masks, host only)."""
    wm = (ctypes.c_uint64 * max(levels, 1))()
    mv = (ctypes.c_int32 * ((levels + 1) * k))()
    check(lib.kd_level_masks(k, levels, defer, wm, mv), "kd_level_masks")
    return ([int(wm[i]) for i in range(levels)],
            [[int(mv[d * k + j]) for j in range(k)] for d in range(levels + 1)])


def check(rc: int, what: str) -> None:
    if rc != KD_OK:
        raise KdError(f"{what}: {lib.kd_strerror(rc).decode()} ({rc})")


def workspace_bytes(n: int, k: int, dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check(lib.kdtree_workspace_bytes(n, k, dtype, ctypes.byref(out)), "kdtree_workspace_bytes")
    return int(out.value)


def workspace_bytes_batched(total: int, trees: int, k: int, dtype: int) -> int:
    out = ctypes.c_size_t(0)
    check(lib.kdtree_workspace_bytes_batched(total, trees, k, dtype, ctypes.byref(out)),
          "kdtree_workspace_bytes_batched")
    return int(out.value)


def options(cutover: int | None, leaf_blocks: int | None = None, records: int | None = None,
            learned_sorts: int | None = None, level: int | None = None,
            digit_bits: int | None = None, sort_tile: int | None = None):
    vals = (cutover, leaf_blocks, records, learned_sorts, level, digit_bits, sort_tile)
    if all(v is None for v in vals):
        return None
    o = kd_options()
    o.cutover = int(cutover or 0)
    o.leaf_blocks = int(leaf_blocks or 0)
    o.records = int(records or 0)
    o.learned_sorts = int(learned_sorts or 0)
    o.level = int(level or 0)
    o.digit_bits = int(digit_bits or 0)
    o.sort_tile = int(sort_tile or 0)
    return ctypes.byref(o)


def _size(fn, *args) -> int:
    out = ctypes.c_size_t(0)
    check(getattr(lib, fn)(*args, ctypes.byref(out)), fn)
    return int(out.value)


def workspace_bytes_learned(n: int, k: int, dtype: int) -> int:
    return _size("kdtree_workspace_bytes_learned", n, k, dtype)


def cdf_model_bytes(k: int) -> int:
    return _size("kd_cdf_model_bytes", k)


def cdf_train_workspace_bytes(k: int, n_samples: int) -> int:
    return _size("kd_cdf_train_workspace_bytes", k, n_samples)
