"""MI355X (gfx950) presorting balanced k-d tree builder.

Python face of ``libkdtree.so`` (C ABI in ``include/kdtree.h``).  PyTorch is
used only to hold device memory and to name the current HIP stream; every
step of the build runs in the library's hand-written kernels.

Output is the in-order layout of the balanced tree: ``perm[pos]`` is the input
row of the node at position ``pos`` (pos < n_unique); the node of a subarray
``[s, e]`` is at ``s + (e - s) // 2`` and splits on dimension ``depth mod k``.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import KD_F32, KD_I32, KdError  # noqa: F401

__all__ = ["Builder", "BatchedBuilder", "build", "build_batched", "KdError"]


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.int32:
        return KD_I32
    if t.dtype == torch.float32:
        return KD_F32
    raise TypeError(f"tuples must be int32 or float32, got {t.dtype}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Builder:
    """Holds a device workspace for builds of up to ``n`` rows in ``k``
    dimensions, so repeated builds allocate nothing."""

    def __init__(self, n: int, k: int, dtype=torch.int32, device="cuda", cutover: int | None = None):
        self.n, self.k = int(n), int(k)
        self.code = _dtype_code(torch.empty(0, dtype=dtype))
        self.device = torch.device(device)
        self.cutover = cutover
        nbytes = _lib.workspace_bytes(self.n, self.k, self.code)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.n_unique = torch.zeros(1, dtype=torch.int64, device=self.device)

    def _check_input(self, tuples: torch.Tensor):
        if tuples.dim() != 2 or tuples.shape[1] != self.k or tuples.shape[0] > self.n:
            raise ValueError(f"tuples must be (<= {self.n}, {self.k}); got {tuple(tuples.shape)}")
        if not tuples.is_cuda or not tuples.is_contiguous():
            raise ValueError("tuples must be a contiguous device tensor")
        if _dtype_code(tuples) != self.code:
            raise TypeError("tuples dtype differs from the builder's")

    def build(self, tuples: torch.Tensor, perm: torch.Tensor, lo=None, hi=None, stream=None):
        """Enqueue a whole build; perm (and lo/hi) are int32 device tensors of >= n rows."""
        self._check_input(tuples)
        n = tuples.shape[0]
        rc = _lib.lib.kdtree_build(_ptr(tuples), n, self.k, self.code, _ptr(perm), _ptr(lo), _ptr(hi),
                                   _ptr(self.n_unique), _ptr(self.workspace), self.workspace.numel(),
                                   _lib.options(self.cutover), _stream(stream))
        _lib.check(rc, "kdtree_build")

    def presort(self, tuples: torch.Tensor, stream=None):
        self._check_input(tuples)
        rc = _lib.lib.kdtree_presort(_ptr(tuples), tuples.shape[0], self.k, self.code, _ptr(self.n_unique),
                                     _ptr(self.workspace), self.workspace.numel(),
                                     _lib.options(self.cutover), _stream(stream))
        _lib.check(rc, "kdtree_presort")

    def partition(self, tuples: torch.Tensor, perm: torch.Tensor, lo=None, hi=None, stream=None):
        self._check_input(tuples)
        rc = _lib.lib.kdtree_partition(_ptr(tuples), tuples.shape[0], self.k, self.code, _ptr(perm),
                                       _ptr(lo), _ptr(hi), _ptr(self.n_unique), _ptr(self.workspace),
                                       self.workspace.numel(), _lib.options(self.cutover),
                                       _stream(stream))
        _lib.check(rc, "kdtree_partition")


class BatchedBuilder:
    """Builds many independent trees with one sequence of launches.

    ``offsets`` (host sequence or int64 tensor of B+1 values) splits the rows of
    ``tuples`` into trees; the workspace is sized for exactly that split."""

    def __init__(self, offsets, k: int, dtype=torch.int32, device="cuda", cutover: int | None = None):
        import numpy as np

        off = np.asarray(offsets.cpu() if isinstance(offsets, torch.Tensor) else offsets, dtype=np.int64)
        self.h_offsets = np.ascontiguousarray(off)
        self.trees = int(off.shape[0] - 1)
        self.total = int(off[-1])
        self.k = int(k)
        self.code = _dtype_code(torch.empty(0, dtype=dtype))
        self.device = torch.device(device)
        self.cutover = cutover
        self.d_offsets = torch.from_numpy(self.h_offsets).to(self.device)
        nbytes = _lib.workspace_bytes_batched(self.total, self.trees, self.k, self.code)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.n_unique = torch.zeros(self.trees, dtype=torch.int64, device=self.device)

    def build(self, tuples: torch.Tensor, perm: torch.Tensor, stream=None):
        if tuples.dim() != 2 or tuples.shape[0] != self.total or tuples.shape[1] != self.k:
            raise ValueError(f"tuples must be ({self.total}, {self.k})")
        if not tuples.is_cuda or not tuples.is_contiguous() or _dtype_code(tuples) != self.code:
            raise ValueError("tuples must be a contiguous device tensor of the builder's dtype")
        rc = _lib.lib.kdtree_build_batched(
            _ptr(tuples), _ptr(self.d_offsets), self.h_offsets.ctypes.data_as(ctypes.c_void_p),
            self.trees, self.k, self.code, _ptr(perm), _ptr(self.n_unique), _ptr(self.workspace),
            self.workspace.numel(), _lib.options(self.cutover), _stream(stream))
        _lib.check(rc, "kdtree_build_batched")


def build_batched(tuples: torch.Tensor, offsets, cutover: int | None = None, stream=None):
    """Build one tree per row range ``offsets[b] .. offsets[b+1]-1``.

    Returns ``(perm, n_unique)``: perm (int32, length offsets[-1]) holds tree
    b's in-order layout at positions offsets[b] .. offsets[b]+n_unique[b]-1,
    as row indices local to the tree.
    """
    b = BatchedBuilder(offsets, tuples.shape[1], tuples.dtype, tuples.device, cutover)
    perm = torch.full((max(b.total, 1),), -1, dtype=torch.int32, device=tuples.device)
    b.build(tuples.contiguous(), perm, stream)
    return perm[: b.total], b.n_unique


def build(tuples: torch.Tensor, children: bool = False, cutover: int | None = None, stream=None):
    """Build the tree of ``tuples`` ((n, k) int32/float32 device tensor).

    Returns ``(perm, n_unique)`` or ``(perm, n_unique, lo, hi)`` with device
    tensors trimmed to ``n_unique`` (this synchronises to read the count).
    """
    n, k = tuples.shape
    b = Builder(max(n, 1), k, tuples.dtype, tuples.device, cutover)
    perm = torch.full((max(n, 1),), -1, dtype=torch.int32, device=tuples.device)
    lo = hi = None
    if children:
        lo = torch.full_like(perm, -2)
        hi = torch.full_like(perm, -2)
    b.build(tuples.contiguous(), perm, lo, hi, stream)
    nu = int(b.n_unique.item())
    if children:
        return perm[:nu], nu, lo[:nu], hi[:nu]
    return perm[:nu], nu
