"""CPU oracle for the presorting balanced k-d tree build (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the
oracle never imports the GPU library: the two share nothing but the seeded
input generators in ``kdgen``.

The arithmetic lives in ``kd_oracle.cpp`` (plain C++17, compiled with g++ by
:func:`build`); this module only marshals numpy arrays through ctypes, plus
the tree queries in :mod:`oracle.queries`.

Output convention (the in-order layout): ``perm[pos]`` is the input row of the
node stored at position ``pos``; the node of a subarray ``[s, e]`` sits at its
lower median ``s + (e - s) // 2`` (Sec. 2.1, with the two-element rule of
Sec. 3.1 fixing the even case).  ``lo``/``hi`` give the child positions or -1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kd_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "libkdoracle.so")
_lib = None

DT_I32 = 0
DT_F32 = 1


def build() -> str:
    """Compile the oracle with g++ (no GPU, no HIP)."""
    cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread", "-o", _LIB_PATH + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.kdo_presort.argtypes = [vp, i64, i32, i32, i32, vp, vp]
    lib.kdo_presort.restype = ctypes.c_int
    lib.kdo_build.argtypes = [vp, i64, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
    lib.kdo_build.restype = ctypes.c_int
    _lib = lib
    return lib


def _dtype_code(t: np.ndarray) -> int:
    if t.dtype == np.int32:
        return DT_I32
    if t.dtype == np.float32:
        return DT_F32
    raise TypeError(f"tuples must be int32 or float32, got {t.dtype}")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def presort(tuples: np.ndarray, threads: int = 1):
    """Sec. 2.1 presort and duplicate removal.

    Returns ``(arrays, n_unique)`` where ``arrays[d, :n_unique]`` is the index
    array sorted by the super key that starts at dimension ``d``.
    """
    t = np.ascontiguousarray(tuples)
    n, k = t.shape
    out = np.zeros((k, max(n, 1)), dtype=np.int32)
    nu = np.zeros(1, dtype=np.int64)
    rc = _load().kdo_presort(_ptr(t), n, k, _dtype_code(t), threads, _ptr(out), _ptr(nu))
    if rc != 0:
        raise RuntimeError(f"kdo_presort failed ({rc})")
    return out[:, : int(nu[0])].copy(), int(nu[0])


def build_tree(tuples: np.ndarray, threads: int = 1, max_depth: int = -1, children: bool = True,
               arrays: bool = False):
    """Sec. 2.1 build (parent/child threads of Sec. 2.2 when ``threads`` > 1).

    Returns a dict with ``perm`` (int32[n_unique]), ``n_unique``, ``lo``/``hi``
    (int32[n_unique], when ``children``), ``arrays`` (int32[k, n], the index
    arrays after ``max_depth`` levels, when ``arrays``) and ``times``
    (presort seconds, build seconds).
    """
    t = np.ascontiguousarray(tuples)
    n, k = t.shape
    perm = np.full(max(n, 1), -1, dtype=np.int32)
    lo = np.full(max(n, 1), -1, dtype=np.int32) if children else None
    hi = np.full(max(n, 1), -1, dtype=np.int32) if children else None
    arr = np.zeros((k, max(n, 1)), dtype=np.int32) if arrays else None
    nu = np.zeros(1, dtype=np.int64)
    times = np.zeros(2, dtype=np.float64)
    rc = _load().kdo_build(_ptr(t), n, k, _dtype_code(t), threads, max_depth, _ptr(perm), _ptr(lo),
                           _ptr(hi), _ptr(nu), _ptr(arr), _ptr(times))
    if rc != 0:
        raise RuntimeError(f"kdo_build failed ({rc})")
    u = int(nu[0])
    res = {"perm": perm[:u].copy(), "n_unique": u, "times": (float(times[0]), float(times[1]))}
    if children:
        res["lo"] = lo[:u].copy()
        res["hi"] = hi[:u].copy()
    if arrays:
        res["arrays"] = arr[:, :n].copy()
    return res
