"""Oracle of the learned CDF model behind the learned presort.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
leg may import it; the GPU library never does, and nothing here calls it.

The model is not in the paper.  It only guesses where a key lands in the
sorted order; the presort it serves must return exactly what the radix presort
returns, so the model changes speed, never results.

Definition.  K segments split a finite value range [lo, hi] evenly (the
trained model uses the column's finite range).  Logits theta[0..K-1] give segment masses q = softmax(theta); the
exported model floors every mass at 1/(4S) for a sample of S keys and
renormalises (q' = (q + 1/(4S)) / (1 + K/(4S))), and its cumulative levels
are c_0 = 0, c_i = q'_0 + ... + q'_{i-1}, c_K = 1.  For a key
strictly between the keys of lo and hi, with value v:

    t = (v - lo) * scale,   scale = K / (hi - lo)
    i = min(floor(t), K - 1),  f = clamp(t - i, 0, 1)
    F = min(c_i + f (c_{i+1} - c_i), c_{i+1})

F = 0 at or below lo's key and 1 at or above hi's key (keys in the
order-preserving 32-bit form).  The bucket of a key among 2^b buckets is
min(floor(F 2^b), 2^b - 1).

Training objective: the sample's segment masses p_j (the fraction of sample
keys in segment j; keys at or below lo count in segment 0, at or above hi in
segment K-1) against q: L = -sum_j p_j log q_j, whose gradient is q - p.

Precision.  The segment index, and F itself where it decides a bucket, are
integer decisions taken from floating point; the GPU takes them in single
precision, so :func:`segments_f32` and :func:`forward_f32` take them in
single precision too, step by step (numpy float32 arithmetic rounds every
operation to nearest, as the kernels' explicitly rounded operations do).
The losses, gradients and training run in fp64.
"""
from __future__ import annotations

import numpy as np

K = 4096


# ---- keys ----------------------------------------------------------------------

def canonical(vals: np.ndarray, is_float: bool) -> np.ndarray:
    """Order-preserving uint32 key: int32 with its sign bit flipped; float32
    under IEEE totalOrder (negative encodings complemented, others with the
    sign bit set)."""
    if not is_float:
        return (np.asarray(vals, dtype=np.int32).view(np.uint32) ^ np.uint32(0x80000000)).astype(np.uint32)
    b = np.asarray(vals, dtype=np.float32).view(np.uint32)
    return np.where(b >> np.uint32(31) == 1, ~b, b ^ np.uint32(0x80000000)).astype(np.uint32)


def key_value(keys: np.ndarray, is_float: bool) -> np.ndarray:
    """float32 coordinate value of canonical keys."""
    keys = np.asarray(keys, dtype=np.uint32)
    if not is_float:
        return (keys ^ np.uint32(0x80000000)).view(np.int32).astype(np.float32)
    neg = (keys & np.uint32(0x80000000)) == 0
    bits = np.where(neg, ~keys, keys ^ np.uint32(0x80000000)).astype(np.uint32)
    return bits.view(np.float32)


def finite(keys: np.ndarray, is_float: bool) -> np.ndarray:
    if not is_float:
        return np.ones(len(keys), dtype=bool)
    return np.isfinite(key_value(keys, True))


# ---- domain and segments ---------------------------------------------------------

class Domain:
    """Finite value range of a sorted sample of canonical keys."""

    def __init__(self, kmin: int, kmax: int, is_float: bool):
        self.kmin = np.uint32(kmin)
        self.kmax = np.uint32(kmax)
        self.is_float = is_float
        self.lo = key_value(np.array([kmin], dtype=np.uint32), is_float)[0]
        self.hi = key_value(np.array([kmax], dtype=np.uint32), is_float)[0]
        if self.hi > self.lo:
            self.scale = np.float32(K / (np.float64(self.hi) - np.float64(self.lo)))
        else:
            self.scale = np.float32(0.0)

    @staticmethod
    def of_sample(sorted_keys: np.ndarray, is_float: bool) -> "Domain":
        fin = np.nonzero(finite(sorted_keys, is_float))[0]
        if len(fin) == 0:
            return Domain(0x80000000, 0x80000000, is_float)
        return Domain(int(sorted_keys[fin[0]]), int(sorted_keys[fin[-1]]), is_float)

    @staticmethod
    def of_column(keys: np.ndarray, is_float: bool) -> "Domain":
        """The finite range of a whole column (the trained model's domain)."""
        keys = np.asarray(keys, dtype=np.uint32)
        fk = keys[finite(keys, is_float)]
        if len(fk) == 0:
            return Domain(0x80000000, 0x80000000, is_float)
        return Domain(int(fk.min()), int(fk.max()), is_float)


def segments_f32(dm: Domain, keys: np.ndarray):
    """(inside mask, segment index, fraction) of keys, the index and fraction
    taken in single precision."""
    keys = np.asarray(keys, dtype=np.uint32)
    inside = (keys > dm.kmin) & (keys < dm.kmax)
    v = key_value(keys, dm.is_float)
    with np.errstate(over="ignore", invalid="ignore"):
        t = np.float32(v - dm.lo) * dm.scale  # float32 subtract, then float32 multiply
        t = t.astype(np.float32)
        i = np.where(t < np.float32(K), np.trunc(np.where(np.isfinite(t), t, 0)), K - 1)
    i = np.clip(i, 0, K - 1).astype(np.int64)
    with np.errstate(invalid="ignore"):
        f = (t - i.astype(np.float32)).astype(np.float32)
    f = np.where(f < 0, np.float32(0), np.where(f > 1, np.float32(1), f)).astype(np.float32)
    return inside, i, f


def sample_segments(dm: Domain, keys: np.ndarray) -> np.ndarray:
    """Segment of every sample key for the training masses."""
    keys = np.asarray(keys, dtype=np.uint32)
    inside, i, _ = segments_f32(dm, keys)
    return np.where(keys <= dm.kmin, 0, np.where(keys >= dm.kmax, K - 1, i))


# ---- objective ----------------------------------------------------------------------

def masses(dm: Domain, keys: np.ndarray) -> np.ndarray:
    """p_j: fraction of the sample in segment j (fp64)."""
    if len(keys) == 0:
        return np.zeros(K)
    return np.bincount(sample_segments(dm, keys), minlength=K).astype(np.float64) / len(keys)


def softmax(theta: np.ndarray) -> np.ndarray:
    th = np.asarray(theta, dtype=np.float64)
    e = np.exp(th - th.max())
    return e / e.sum()


def loss(theta: np.ndarray, p: np.ndarray) -> float:
    q = softmax(theta)
    nz = p > 0
    return float(-np.sum(p[nz] * np.log(q[nz])))


def loss_grad(theta: np.ndarray, p: np.ndarray):
    """(L, dL/dtheta) with dL/dtheta_i = sum_j p_j (q_i - [i = j]) = q_i - p_i."""
    q = softmax(theta)
    return loss(theta, p), q * p.sum() - p


def train_adam(p: np.ndarray, steps: int, lr: float, b1=0.9, b2=0.999, eps=1e-8) -> np.ndarray:
    """Adam (Kingma and Ba, 2015: exponential moving averages of the gradient
    and of its square, each divided by its bias correction 1 - beta^t, and a
    step of lr * m_hat / (sqrt(v_hat) + eps)) from theta = 0 on the
    objective above (fp64)."""
    th = np.zeros(K)
    m = np.zeros(K)
    s = np.zeros(K)
    for t in range(1, steps + 1):
        _, g = loss_grad(th, p)
        m = b1 * m + (1 - b1) * g
        s = b2 * s + (1 - b2) * g * g
        th = th - lr * (m / (1 - b1 ** t)) / (np.sqrt(s / (1 - b2 ** t)) + eps)
    return th


def running_levels(theta: np.ndarray, S: int = 0) -> np.ndarray:
    """c_0 .. c_K (fp64) exactly as summed: c_i = q'_0 + ... + q'_{i-1}.
    With a sample size S, every mass first gets a floor of 1/(4S) and the
    masses are renormalised (the exported model; segments the sample missed
    still cover some range).  c_K is 1 up to rounding when the masses are
    normalised correctly."""
    q = softmax(theta)
    if S > 0:
        fl = 0.25 / S
        q = (q + fl) / (1.0 + len(q) * fl)
    return np.concatenate([[0.0], np.cumsum(q)])


def levels(theta: np.ndarray, S: int = 0) -> np.ndarray:
    """The exported levels: :func:`running_levels` with c_K set to exactly 1
    (the model's definition), after checking that the sum reached 1."""
    c = running_levels(theta, S)
    if abs(c[-1] - 1.0) > 1e-9:
        raise ValueError(f"segment masses sum to {c[-1]!r}, not 1")
    c[-1] = 1.0
    return np.minimum(c, 1.0)


# ---- evaluation -------------------------------------------------------------------

def forward(c: np.ndarray, dm: Domain, keys: np.ndarray) -> np.ndarray:
    """F of canonical keys in fp64 arithmetic (segment decisions in fp32)."""
    c = np.asarray(c, dtype=np.float64)
    keys = np.asarray(keys, dtype=np.uint32)
    inside, i, f = segments_f32(dm, keys)
    a, b = c[i], c[i + 1]
    F = np.minimum(a + f.astype(np.float64) * (b - a), b)
    return np.where(keys <= dm.kmin, 0.0, np.where(keys >= dm.kmax, 1.0, F))


def forward_f32(c32: np.ndarray, dm: Domain, keys: np.ndarray) -> np.ndarray:
    """F in single precision, every step rounded: the value a bucket is cut from."""
    c32 = np.asarray(c32, dtype=np.float32)
    keys = np.asarray(keys, dtype=np.uint32)
    inside, i, f = segments_f32(dm, keys)
    a, b = c32[i], c32[i + 1]
    F = np.minimum((a + (f * (b - a)).astype(np.float32)).astype(np.float32), b)
    return np.where(keys <= dm.kmin, np.float32(0), np.where(keys >= dm.kmax, np.float32(1), F)).astype(np.float32)


def bucket(F32: np.ndarray, nb_bits: int) -> np.ndarray:
    nb = 1 << nb_bits
    b = np.floor((np.asarray(F32, dtype=np.float32) * np.float32(nb)).astype(np.float32)).astype(np.int64)
    return np.minimum(b, nb - 1)


def strided_sample(tuples: np.ndarray, S: int) -> np.ndarray:
    """Rows floor(s * n / S), s = 0 .. S-1 (the training sample)."""
    n = tuples.shape[0]
    rows = (np.arange(S, dtype=np.int64) * n) // S
    return tuples[rows]
