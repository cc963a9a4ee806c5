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

__all__ = ["Builder", "BatchedBuilder", "LearnedBuilder", "build", "build_batched", "build_learned",
           "train_cdf", "cdf_loss_grad", "cdf_eval", "gather_nodes", "subtree_bounds", "region_count",
           "region_rows",
           "nearest", "all_nearest", "reverse_nearest", "build_select", "SelectBuilder", "KdError"]


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

    def __init__(self, n: int, k: int, dtype=torch.int32, device="cuda", cutover: int | None = None,
                 leaf_blocks: int | None = None, records: int | None = None, level: int | None = None,
                 digit_bits: int | None = None, sort_tile: int | None = None):
        self.n, self.k = int(n), int(k)
        self.code = _dtype_code(torch.empty(0, dtype=dtype))
        self.device = torch.device(device)
        self.cutover = cutover
        self.leaf_blocks = leaf_blocks
        self.records = records
        self.level = level
        self.digit_bits = digit_bits
        self.sort_tile = sort_tile
        nbytes = _lib.workspace_bytes(self.n, self.k, self.code)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.n_unique = torch.zeros(1, dtype=torch.int64, device=self.device)

    def status(self, stream=None) -> int:
        """Waits for the stream and checks the last build's device status
        word (kd_status): raises KdError if a kernel found inconsistent
        counts, else returns 0."""
        return _lib.status(_ptr(self.workspace), self.workspace.numel(), _stream(stream))

    def _opts(self):
        return _lib.options(self.cutover, getattr(self, "leaf_blocks", None),
                            getattr(self, "records", None), getattr(self, "learned_sorts", None),
                            getattr(self, "level", None), getattr(self, "digit_bits", None),
                            getattr(self, "sort_tile", None))

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
                                   self._opts(), _stream(stream))
        _lib.check(rc, "kdtree_build")

    def presort(self, tuples: torch.Tensor, stream=None):
        self._check_input(tuples)
        rc = _lib.lib.kdtree_presort(_ptr(tuples), tuples.shape[0], self.k, self.code, _ptr(self.n_unique),
                                     _ptr(self.workspace), self.workspace.numel(),
                                     self._opts(), _stream(stream))
        _lib.check(rc, "kdtree_presort")

    def partition(self, tuples: torch.Tensor, perm: torch.Tensor, lo=None, hi=None, stream=None):
        self._check_input(tuples)
        rc = _lib.lib.kdtree_partition(_ptr(tuples), tuples.shape[0], self.k, self.code, _ptr(perm),
                                       _ptr(lo), _ptr(hi), _ptr(self.n_unique), _ptr(self.workspace),
                                       self.workspace.numel(), self._opts(),
                                       _stream(stream))
        _lib.check(rc, "kdtree_partition")


class BatchedBuilder:
    """Builds many independent trees with one sequence of launches.

    ``offsets`` (host sequence or int64 tensor of B+1 values) splits the rows of
    ``tuples`` into trees; the workspace is sized for exactly that split."""

    def __init__(self, offsets, k: int, dtype=torch.int32, device="cuda", cutover: int | None = None,
                 leaf_blocks: int | None = None, records: int | None = None, level: int | None = None,
                 digit_bits: int | None = None, sort_tile: int | None = None):
        import numpy as np

        self.leaf_blocks = leaf_blocks
        self.records = records
        self.level = level
        self.digit_bits = digit_bits
        self.sort_tile = sort_tile
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
            self.workspace.numel(), _lib.options(self.cutover, self.leaf_blocks, self.records,
                                                 level=self.level, digit_bits=self.digit_bits,
                                                 sort_tile=self.sort_tile),
            _stream(stream))
        _lib.check(rc, "kdtree_build_batched")

    def status(self, stream=None) -> int:
        """As :meth:`Builder.status`."""
        return _lib.status(_ptr(self.workspace), self.workspace.numel(), _stream(stream))


def build_batched(tuples: torch.Tensor, offsets, cutover: int | None = None, stream=None,
                  level: int | None = None, **knobs):
    """Build one tree per row range ``offsets[b] .. offsets[b+1]-1``.

    Returns ``(perm, n_unique)``: perm (int32, length offsets[-1]) holds tree
    b's in-order layout at positions offsets[b] .. offsets[b]+n_unique[b]-1,
    as row indices local to the tree.
    """
    b = BatchedBuilder(offsets, tuples.shape[1], tuples.dtype, tuples.device, cutover, level=level,
                       **knobs)
    perm = torch.full((max(b.total, 1),), -1, dtype=torch.int32, device=tuples.device)
    b.build(tuples.contiguous(), perm, stream)
    b.status(stream)
    return perm[: b.total], b.n_unique


def build(tuples: torch.Tensor, children: bool = False, cutover: int | None = None, stream=None,
          records: int | None = None, level: int | None = None, digit_bits: int | None = None,
          sort_tile: int | None = None):
    """Build the tree of ``tuples`` ((n, k) int32/float32 device tensor).

    Returns ``(perm, n_unique)`` or ``(perm, n_unique, lo, hi)`` with device
    tensors trimmed to ``n_unique`` (this synchronises to read the count).
    """
    n, k = tuples.shape
    b = Builder(max(n, 1), k, tuples.dtype, tuples.device, cutover, records=records, level=level,
                digit_bits=digit_bits, sort_tile=sort_tile)
    perm = torch.full((max(n, 1),), -1, dtype=torch.int32, device=tuples.device)
    lo = hi = None
    if children:
        lo = torch.full_like(perm, -2)
        hi = torch.full_like(perm, -2)
    b.build(tuples.contiguous(), perm, lo, hi, stream)
    b.status(stream)
    nu = int(b.n_unique.item())
    if children:
        return perm[:nu], nu, lo[:nu], hi[:nu]
    return perm[:nu], nu


# ---- searches over a built tree ---------------------------------------------------

def _query_args(tuples: torch.Tensor, perm: torch.Tensor, n_nodes, queries: torch.Tensor):
    n, k = tuples.shape
    if perm.dtype != torch.int32:
        raise TypeError("perm must be int32")
    if queries.dtype != tuples.dtype or queries.dim() != 2 or queries.shape[1] != k:
        raise ValueError("queries must be (nq, k) of the tuples' dtype")
    if not torch.is_tensor(n_nodes):
        n_nodes = torch.tensor([int(n_nodes)], dtype=torch.int64, device=tuples.device)
    return n, k, _dtype_code(tuples), n_nodes.reshape(1).to(torch.int64).contiguous()


def gather_nodes(tuples: torch.Tensor, perm: torch.Tensor, n_nodes, stream=None) -> torch.Tensor:
    """The tree's node coordinates in tree-position order (kd_gather_nodes):
    row pos of the result is ``tuples[perm[pos]]``.  The searches read these;
    gather once per tree and pass them as ``nodes=``."""
    n, k, code, nn = _query_args(tuples, perm, n_nodes, tuples[:0])
    nodes = torch.empty_like(tuples)
    _lib.check(_lib.lib.kd_gather_nodes(_ptr(tuples.contiguous()), n, k, code, _ptr(perm), _ptr(nn),
                                        _ptr(nodes), _stream(stream)), "kd_gather_nodes")
    return nodes


def subtree_bounds(nodes: torch.Tensor, n_nodes, stream=None) -> torch.Tensor:
    """Bounding box of every subtree at its node's position
    (kd_subtree_bounds): an (n, 2k) tensor, the k smallest then the k
    largest coordinates.  Optional ``bounds=`` of the box queries."""
    n, k = nodes.shape
    if not torch.is_tensor(n_nodes):
        n_nodes = torch.tensor([int(n_nodes)], dtype=torch.int64, device=nodes.device)
    nn = n_nodes.reshape(1).to(torch.int64).contiguous()
    bounds = torch.empty((n, 2 * k), dtype=nodes.dtype, device=nodes.device)
    _lib.check(_lib.lib.kd_subtree_bounds(_ptr(nodes), n, k, _dtype_code(nodes), _ptr(nn),
                                          _ptr(bounds), _stream(stream)), "kd_subtree_bounds")
    return bounds


def region_count(tuples: torch.Tensor, perm: torch.Tensor, n_nodes, lower: torch.Tensor,
                 upper: torch.Tensor, visits: torch.Tensor | None = None, nodes=None, bounds=None,
                 stream=None):
    """Number of tree nodes inside every box (kd_region_count).

    ``perm``: the in-order layout of ``tuples``' tree; ``n_nodes``: its node
    count (int or device int64 tensor); ``lower``/``upper``: (nq, k) box
    corners, inclusive.  ``visits``: optional uint64 device counter;
    ``nodes``: ``gather_nodes``' result, gathered here when not given;
    ``bounds``: ``subtree_bounds``' result, or None (same counts, more visits).
    """
    n, k, code, nn = _query_args(tuples, perm, n_nodes, lower)
    if nodes is None:
        nodes = gather_nodes(tuples, perm, nn, stream)
    lower, upper = lower.contiguous(), upper.contiguous()
    if upper.shape != lower.shape or upper.dtype != lower.dtype:
        raise ValueError("lower and upper must match")
    nq = lower.shape[0]
    counts = torch.empty(nq, dtype=torch.int32, device=tuples.device)
    _lib.check(_lib.lib.kd_region_count(_ptr(nodes), _ptr(bounds), n, k, code, _ptr(nn), _ptr(lower),
                                        _ptr(upper), nq, _ptr(counts), _ptr(visits),
                                        _stream(stream)), "kd_region_count")
    return counts


def region_rows(tuples: torch.Tensor, perm: torch.Tensor, n_nodes, lower: torch.Tensor,
                upper: torch.Tensor, nodes=None, bounds=None, stream=None):
    """Rows of the tree nodes inside every box, as ``(rows, offsets)``: the
    rows of box q are ``rows[offsets[q]:offsets[q + 1]]`` in increasing tree
    position.  Counts first (kd_region_count), then rows (kd_region_rows);
    this synchronises once to size the output."""
    n, k, code, nn = _query_args(tuples, perm, n_nodes, lower)
    if nodes is None:
        nodes = gather_nodes(tuples, perm, nn, stream)
    counts = region_count(tuples, perm, nn, lower, upper, nodes=nodes, bounds=bounds, stream=stream)
    nq = lower.shape[0]
    offsets = torch.zeros(nq + 1, dtype=torch.int64, device=tuples.device)
    torch.cumsum(counts.to(torch.int64), 0, out=offsets[1:])
    total = int(offsets[-1].item())
    rows = torch.empty(max(total, 1), dtype=torch.int32, device=tuples.device)
    _lib.check(_lib.lib.kd_region_rows(_ptr(nodes), _ptr(bounds), n, k, code, _ptr(perm), _ptr(nn),
                                       _ptr(lower.contiguous()), _ptr(upper.contiguous()), nq,
                                       _ptr(offsets), _ptr(rows), total, None, _stream(stream)),
               "kd_region_rows")
    return rows[:total], offsets


def nearest(tuples: torch.Tensor, perm: torch.Tensor, n_nodes, points: torch.Tensor, m: int,
            visits: torch.Tensor | None = None, nodes=None, stream=None):
    """The m nearest tree nodes of every query point (kd_nearest): an (nq, m)
    int32 tensor of rows in increasing (squared distance, row), -1 past the
    node count."""
    n, k, code, nn = _query_args(tuples, perm, n_nodes, points)
    if nodes is None:
        nodes = gather_nodes(tuples, perm, nn, stream)
    points = points.contiguous()
    nq = points.shape[0]
    rows = torch.empty((nq, m), dtype=torch.int32, device=tuples.device)
    _lib.check(_lib.lib.kd_nearest(_ptr(nodes), n, k, code, _ptr(perm), _ptr(nn), _ptr(points), nq,
                                   int(m), _ptr(rows), _ptr(visits), _stream(stream)), "kd_nearest")
    return rows


def all_nearest(tuples: torch.Tensor, perm: torch.Tensor, n_nodes, m: int,
                visits: torch.Tensor | None = None, nodes=None, stream=None):
    """Every tree node's m nearest other nodes (kd_all_nearest): an (n, m)
    int32 tensor whose row pos (a tree position) lists rows in increasing
    (squared distance, row); -1 past the node count, rows past it unset."""
    n, k, code, nn = _query_args(tuples, perm, n_nodes, tuples[:0])
    if nodes is None:
        nodes = gather_nodes(tuples, perm, nn, stream)
    rows = torch.full((n, m), -1, dtype=torch.int32, device=tuples.device)
    _lib.check(_lib.lib.kd_all_nearest(_ptr(nodes), n, k, code, _ptr(perm), _ptr(nn), int(m),
                                       _ptr(rows), _ptr(visits), _stream(stream)), "kd_all_nearest")
    return rows


def reverse_nearest(perm: torch.Tensor, n_nodes, near_rows: torch.Tensor, stream=None):
    """Reverse nearest-neighbour lists from ``all_nearest``'s output
    (kd_reverse_nearest): ``(offsets, lists)`` with the list of row r in
    ``lists[offsets[r]:offsets[r + 1]]``, ascending."""
    n, m = near_rows.shape
    if not torch.is_tensor(n_nodes):
        n_nodes = torch.tensor([int(n_nodes)], dtype=torch.int64, device=near_rows.device)
    nn = n_nodes.reshape(1).to(torch.int64).contiguous()
    ws = torch.empty(_lib._size("kd_reverse_workspace_bytes", n), dtype=torch.uint8,
                     device=near_rows.device)
    offsets = torch.empty(n + 1, dtype=torch.int64, device=near_rows.device)
    lists = torch.empty(max(n * m, 1), dtype=torch.int32, device=near_rows.device)
    _lib.check(_lib.lib.kd_reverse_nearest(_ptr(perm), _ptr(nn), n, int(m),
                                           _ptr(near_rows.contiguous()), _ptr(offsets), _ptr(lists),
                                           _ptr(ws), ws.numel(), _stream(stream)),
               "kd_reverse_nearest")
    return offsets, lists


def build_select(tuples: torch.Tensor, stream=None, digit_bits: int | None = None,
                 sort_tile: int | None = None):
    """The same tree by the comparison method (kdtree_build_select): every
    subarray's median selected afresh at each level (an MSD radix-select and
    a three-way partition) instead of k presorts and partitions.  Returns
    ``(perm, n_unique)`` like ``build``."""
    n, k = tuples.shape
    code = _dtype_code(tuples)
    nbytes = _lib.workspace_bytes(max(n, 1), k, code)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=tuples.device)
    nu = torch.zeros(1, dtype=torch.int64, device=tuples.device)
    perm = torch.full((max(n, 1),), -1, dtype=torch.int32, device=tuples.device)
    _lib.check(_lib.lib.kdtree_build_select(_ptr(tuples.contiguous()), n, k, code, _ptr(perm),
                                            _ptr(nu), _ptr(ws), nbytes,
                                            _lib.options(None, digit_bits=digit_bits,
                                                         sort_tile=sort_tile),
                                            _stream(stream)),
               "kdtree_build_select")
    _lib.status(_ptr(ws), nbytes, _stream(stream))
    u = int(nu.item())
    return perm[:u], u


class SelectBuilder:
    """Reusable workspace for ``build_select`` (no allocation per build)."""

    def __init__(self, n: int, k: int, dtype=torch.int32, device="cuda"):
        self.n, self.k = int(n), int(k)
        self.code = _dtype_code(torch.empty(0, dtype=dtype))
        nbytes = _lib.workspace_bytes(self.n, self.k, self.code)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.n_unique = torch.zeros(1, dtype=torch.int64, device=device)

    def build(self, tuples: torch.Tensor, perm: torch.Tensor, stream=None):
        n, k = tuples.shape
        _lib.check(_lib.lib.kdtree_build_select(_ptr(tuples), n, k, self.code, _ptr(perm),
                                                _ptr(self.n_unique), _ptr(self.workspace),
                                                self.workspace.numel(), None, _stream(stream)),
                   "kdtree_build_select")

    def status(self, stream=None) -> int:
        """As :meth:`Builder.status`."""
        return _lib.status(_ptr(self.workspace), self.workspace.numel(), _stream(stream))


# ---- learned presort ------------------------------------------------------------

def train_cdf(tuples: torch.Tensor, n_samples: int = 1 << 18, steps: int = 300, lr: float = 0.1,
              stream=None, kind: int = _lib.KD_CDF_PWL) -> torch.Tensor:
    """Train one CDF model per dimension on the GPU (kd_cdf_train).

    ``kind`` is the model family: only the piecewise-linear model (0) is
    built; any other kind raises KdError (KD_EUNSUPPORTED).
    Returns the model buffer (uint8 device tensor of k * 33024 bytes)."""
    if tuples.dim() != 2 or not tuples.is_cuda or not tuples.is_contiguous():
        raise ValueError("tuples must be a contiguous (n, k) device tensor")
    n, k = tuples.shape
    code = _dtype_code(tuples)
    models = torch.zeros(_lib.cdf_model_bytes(k), dtype=torch.uint8, device=tuples.device)
    ws = torch.empty(_lib.cdf_train_workspace_bytes(k, n_samples), dtype=torch.uint8,
                     device=tuples.device)
    rc = _lib.lib.kd_cdf_train(_ptr(tuples), n, k, code, int(kind), n_samples, steps, float(lr),
                               _ptr(models), _ptr(ws), ws.numel(), _stream(stream))
    _lib.check(rc, "kd_cdf_train")
    return models


def model_record(models: torch.Tensor, d: int) -> dict:
    """Fields of dimension d's model record (copies to the host)."""
    import numpy as np

    raw = models.view(-1)[d * _lib.CDF_MODEL_BYTES:(d + 1) * _lib.CDF_MODEL_BYTES].cpu().numpy()
    f = raw.view(np.float32)
    u = raw.view(np.uint32)
    i = raw.view(np.int32)
    K = _lib.CDF_SEGMENTS
    return {"lo": float(f[0]), "hi": float(f[1]), "scale": float(f[2]), "kmin": int(u[3]),
            "kmax": int(u[4]), "is_float": int(i[5]), "segments": int(i[6]), "loss": float(f[7]),
            "c": f[8:8 + K + 1].copy(), "theta": f[8 + K + 1:8 + 2 * K + 1].copy()}


def cdf_loss_grad(values_sorted: torch.Tensor, lo_bits: int, hi_bits: int, theta: torch.Tensor,
                  stream=None):
    """Training objective and its gradient for logits ``theta`` (kd_cdf_loss_grad)."""
    m = values_sorted.numel()
    code = _dtype_code(values_sorted)
    dev = values_sorted.device
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    grad = torch.zeros(_lib.CDF_SEGMENTS, dtype=torch.float32, device=dev)
    scratch = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    rc = _lib.lib.kd_cdf_loss_grad(_ptr(values_sorted.contiguous()), m, code, lo_bits & 0xFFFFFFFF,
                                   hi_bits & 0xFFFFFFFF, _ptr(theta.contiguous()), _ptr(loss),
                                   _ptr(grad), _ptr(scratch), _stream(stream))
    _lib.check(rc, "kd_cdf_loss_grad")
    return loss, grad


def cdf_eval(models: torch.Tensor, d: int, values: torch.Tensor, nb_bits: int, stream=None):
    """(F, bucket) of ``values`` under dimension d's model (kd_cdf_eval)."""
    m = values.numel()
    F = torch.zeros(max(m, 1), dtype=torch.float32, device=values.device)
    bucket = torch.zeros(max(m, 1), dtype=torch.int32, device=values.device)
    rec = ctypes.c_void_p(models.data_ptr() + d * _lib.CDF_MODEL_BYTES)
    rc = _lib.lib.kd_cdf_eval(rec, _ptr(values.contiguous()), m, nb_bits, _ptr(F), _ptr(bucket),
                              _stream(stream))
    _lib.check(rc, "kd_cdf_eval")
    return F[:m], bucket[:m]


class LearnedBuilder(Builder):
    """Builder whose presort goes through learned CDF buckets (same output as
    :class:`Builder`).  ``fell_back`` (int32[k] device) reports, per sort,
    whether it had to fall back to the radix passes.  ``learned_sorts``
    (bit d: the sort for super key d uses the learned buckets; default all)
    is a speed knob."""

    def __init__(self, n: int, k: int, dtype=torch.int32, device="cuda", cutover: int | None = None,
                 leaf_blocks: int | None = None, records: int | None = None,
                 learned_sorts: int | None = None, level: int | None = None,
                 digit_bits: int | None = None, sort_tile: int | None = None):
        self.n, self.k = int(n), int(k)
        self.digit_bits = digit_bits
        self.sort_tile = sort_tile
        self.code = _dtype_code(torch.empty(0, dtype=dtype))
        self.device = torch.device(device)
        self.cutover = cutover
        self.leaf_blocks = leaf_blocks
        self.records = records
        self.learned_sorts = learned_sorts
        self.level = level
        nbytes = _lib.workspace_bytes_learned(self.n, self.k, self.code)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.n_unique = torch.zeros(1, dtype=torch.int64, device=self.device)
        self.fell_back = torch.zeros(self.k, dtype=torch.int32, device=self.device)

    def build(self, tuples: torch.Tensor, perm: torch.Tensor, lo=None, hi=None, stream=None,
              models: torch.Tensor | None = None):
        self._check_input(tuples)
        if models is None:
            raise ValueError("a learned build needs the models from train_cdf()")
        rc = _lib.lib.kdtree_build_learned(_ptr(tuples), tuples.shape[0], self.k, self.code, _ptr(models),
                                           _ptr(perm), _ptr(lo), _ptr(hi), _ptr(self.n_unique),
                                           _ptr(self.fell_back), _ptr(self.workspace),
                                           self.workspace.numel(), self._opts(),
                                           _stream(stream))
        _lib.check(rc, "kdtree_build_learned")

    def presort(self, tuples: torch.Tensor, stream=None, models: torch.Tensor | None = None):
        self._check_input(tuples)
        if models is None:
            raise ValueError("a learned presort needs the models from train_cdf()")
        rc = _lib.lib.kdtree_presort_learned(_ptr(tuples), tuples.shape[0], self.k, self.code,
                                             _ptr(models), _ptr(self.n_unique), _ptr(self.fell_back),
                                             _ptr(self.workspace), self.workspace.numel(),
                                             self._opts(), _stream(stream))
        _lib.check(rc, "kdtree_presort_learned")


def build_learned(tuples: torch.Tensor, models: torch.Tensor, children: bool = False,
                  cutover: int | None = None, stream=None, **knobs):
    """Like :func:`build`, through the learned presort.  Returns ``(perm,
    n_unique, fell_back)`` or ``(perm, n_unique, fell_back, lo, hi)``."""
    n, k = tuples.shape
    b = LearnedBuilder(max(n, 1), k, tuples.dtype, tuples.device, cutover, **knobs)
    perm = torch.full((max(n, 1),), -1, dtype=torch.int32, device=tuples.device)
    lo = hi = None
    if children:
        lo = torch.full_like(perm, -2)
        hi = torch.full_like(perm, -2)
    b.build(tuples.contiguous(), perm, lo, hi, stream, models=models)
    b.status(stream)
    nu = int(b.n_unique.item())
    fb = b.fell_back.cpu()
    if children:
        return perm[:nu], nu, fb, lo[:nu], hi[:nu]
    return perm[:nu], nu, fb
