"""Pins of the learned-CDF oracle (oracle/learned.py) against facts that do
not come from it: finite differences of its own loss, the closed-form
minimiser of the cross-entropy, the linear map of the untrained model, a
library histogram, and monotonicity."""
import numpy as np
import pytest

import kdgen
from oracle import learned as L


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_gradient_matches_central_differences():
    g = rng(1)
    theta = g.normal(0, 2, size=L.K)
    p = g.dirichlet(np.full(L.K, 0.3))
    _, grad = L.loss_grad(theta, p)
    h = 1e-5
    idx = g.choice(L.K, size=64, replace=False)
    for i in idx:
        e = np.zeros(L.K)
        e[i] = h
        fd = (L.loss(theta + e, p) - L.loss(theta - e, p)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 + 1e-5 * abs(grad[i]), i


def test_minimiser_is_log_mass():
    """The cross-entropy is minimised by q = p, i.e. theta = log p, where it
    equals the entropy of p."""
    g = rng(2)
    p = g.dirichlet(np.ones(L.K))
    theta = np.log(p)
    val, grad = L.loss_grad(theta, p)
    assert np.max(np.abs(grad)) < 1e-12
    assert val == pytest.approx(-np.sum(p * np.log(p)), rel=1e-12)


def test_adam_reaches_the_minimum():
    g = rng(3)
    p = g.dirichlet(np.full(L.K, 2.0))
    th = L.train_adam(p, steps=300, lr=0.1)
    kl = L.loss(th, p) + np.sum(p * np.log(p))
    assert kl < 1e-3


def test_untrained_model_is_the_linear_map():
    g = rng(4)
    vals = np.sort(g.integers(-(1 << 20), 1 << 20, size=5000).astype(np.int32))
    keys = L.canonical(vals, False)
    dm = L.Domain.of_sample(keys, False)
    F = L.forward(L.levels(np.zeros(L.K)), dm, keys)
    lin = (vals.astype(np.float64) - dm.lo) / (float(dm.hi) - float(dm.lo))
    assert np.max(np.abs(F - lin)) < 1e-5


def test_masses_equal_library_histogram():
    """Integer values with (hi - lo) = 8 K: every segment is exactly 8 values
    wide, so the masses are np.histogram's."""
    g = rng(5)
    vals = np.sort(g.integers(0, 8 * L.K + 1, size=20000)).astype(np.int32)
    vals[0], vals[-1] = 0, 8 * L.K
    keys = L.canonical(vals, False)
    dm = L.Domain.of_sample(keys, False)
    h, _ = np.histogram(vals, bins=L.K, range=(0, 8 * L.K))
    assert np.array_equal(np.rint(L.masses(dm, keys) * len(vals)).astype(np.int64), h)


def test_canonical_keys_follow_total_order():
    vals = np.array([-np.inf, -3.5, -1e-30, -0.0, 0.0, 1e-45, 2.0, np.inf], dtype=np.float32)
    keys = L.canonical(vals, True)
    assert np.all(np.diff(keys.astype(np.int64)) > 0)
    assert np.array_equal(L.key_value(keys, True).view(np.uint32), vals.view(np.uint32))
    ints = np.array([-(2 ** 31), -1, 0, 1, 2 ** 31 - 1], dtype=np.int32)
    ik = L.canonical(ints, False)
    assert np.all(np.diff(ik.astype(np.int64)) > 0)
    assert np.array_equal(L.key_value(ik, False), ints.astype(np.float32))


@pytest.mark.parametrize("is_float", [False, True])
def test_forward_and_buckets_are_monotone(is_float):
    g = rng(6)
    if is_float:
        vals = kdgen.gaussian_mixture_f32(20000, 1, 8, 7)[:, 0]
        vals[:20] = np.array([np.inf, -np.inf, np.nan, -0.0, 0.0] * 4, dtype=np.float32)
    else:
        vals = g.integers(-(2 ** 31), 2 ** 31, size=20000).astype(np.int32)
    keys = np.sort(L.canonical(vals, is_float))
    dm = L.Domain.of_sample(keys[::7], is_float)
    c32 = L.levels(g.normal(0, 3, size=L.K)).astype(np.float32)
    F = L.forward_f32(c32, dm, keys)
    assert np.all(np.diff(F.astype(np.float64)) >= 0)
    assert F.min() >= 0 and F.max() <= 1
    b = L.bucket(F, 12)
    assert np.all(np.diff(b) >= 0) and b.min() >= 0 and b.max() < 4096


def test_trained_model_balances_mixture_buckets():
    """What training buys on the heavy-tailed mixture: with the untrained
    (linear) map the fullest of 2^10 buckets holds far more than its share;
    after training it holds a few shares at most."""
    x = kdgen.gaussian_mixture_f32(1 << 20, 3, 64, kdgen.SEED_BASE + 5)
    sample = L.strided_sample(x, 1 << 16)
    nb = 10
    for d in range(3):
        sk = np.sort(L.canonical(sample[:, d], True))
        keys = L.canonical(x[:, d], True)
        dm = L.Domain.of_column(keys, True)
        untrained = np.bincount(L.bucket(L.forward_f32(L.levels(np.zeros(L.K)).astype(np.float32),
                                                       dm, keys), nb), minlength=1 << nb)
        th = L.train_adam(L.masses(dm, sk), steps=300, lr=0.1)
        trained = np.bincount(L.bucket(L.forward_f32(L.levels(th, 1 << 16).astype(np.float32), dm, keys), nb),
                              minlength=1 << nb)
        mean = len(keys) / (1 << nb)
        assert trained.max() < 4 * mean, d
        assert untrained.max() > 2 * trained.max(), d


def test_mass_floor_keeps_levels_increasing():
    """With the export floor every segment spans some CDF range, even where
    the trained mass is negligible."""
    th = np.full(L.K, -50.0)
    th[10] = 0.0
    c = L.levels(th, 1 << 16)
    assert c[0] == 0.0 and c[-1] == 1.0
    assert np.all(np.diff(c) > 0.2 / (1 << 16))


# ---- training and export pinned to outside facts ------------------------------------

def _p_with_edge_cases(seed):
    """Segment masses with zeros and one entry of exactly 1/K (gradient 0 at
    theta = 0), the rest Dirichlet."""
    g = rng(seed)
    p = g.dirichlet(np.full(L.K, 0.5))
    p[:100] = 0.0
    p[100] = 1.0 / L.K
    rest = np.ones(L.K, dtype=bool)
    rest[:101] = False
    p[rest] *= (1.0 - p[100]) / p[rest].sum()
    return p


def _adam_pins_hold(train):
    """True when `train` (signature of L.train_adam) satisfies both pins:
    the first step's closed form and agreement with torch.optim.Adam."""
    import torch

    lr = 0.05
    for seed in (11, 12):
        p = _p_with_edge_cases(seed)
        # Step 1 from theta = 0: the moment estimates after bias correction
        # are g and g^2 exactly, so the step is -lr * g / (|g| + eps) with the
        # gradient at theta = 0 (about 1/K - p; the gradient itself is pinned
        # by finite differences above).
        g = L.loss_grad(np.zeros(L.K), p)[1]
        assert np.max(np.abs(g - (1.0 / L.K - p))) < 1e-15
        want1 = -lr * g / (np.abs(g) + 1e-8)
        if not np.allclose(train(p, 1, lr), want1, rtol=1e-12, atol=1e-15):
            return False
        # Many steps: torch's Adam (the same published rule, a library
        # implementation) fed the oracle's own gradient of the objective.
        th = torch.zeros(L.K, dtype=torch.float64, requires_grad=True)
        opt = torch.optim.Adam([th], lr=lr, betas=(0.9, 0.999), eps=1e-8)
        for _ in range(40):
            _, gr = L.loss_grad(th.detach().numpy(), p)
            th.grad = torch.from_numpy(gr.copy())
            opt.step()
        if not np.allclose(train(p, 40, lr), th.detach().numpy(), rtol=1e-9, atol=1e-12):
            return False
    return True


def test_adam_matches_first_step_and_torch_optim():
    assert _adam_pins_hold(L.train_adam)


def _adam_variant(bias_correct=True, eps_inside=False, b2=0.999):
    """A copy of the oracle's Adam with one planted mistake (CPU only), to
    show the pins above catch it."""
    def train(p, steps, lr, b1=0.9, eps=1e-8):
        th = np.zeros(L.K)
        m = np.zeros(L.K)
        s = np.zeros(L.K)
        for t in range(1, steps + 1):
            _, g = L.loss_grad(th, p)
            m = b1 * m + (1 - b1) * g
            s = b2 * s + (1 - b2) * g * g
            mh = m / (1 - b1 ** t) if bias_correct else m
            sh = s / (1 - b2 ** t) if bias_correct else s
            den = np.sqrt(sh + eps) if eps_inside else np.sqrt(sh) + eps
            th = th - lr * mh / den
        return th
    return train


@pytest.mark.parametrize("mistake", [dict(bias_correct=False), dict(eps_inside=True), dict(b2=0.99)])
def test_adam_pins_catch_planted_mistakes(mistake):
    assert _adam_pins_hold(_adam_variant())  # the variant without a mistake passes
    assert not _adam_pins_hold(_adam_variant(**mistake))


@pytest.mark.parametrize("S", [0, 1 << 16])
def test_levels_of_uniform_logits_are_equal_steps(S):
    """Equal logits give equal masses 1/K; the floor adds the same amount to
    each and the renormalisation divides it back out, so c_i = i/K."""
    c = L.running_levels(np.zeros(L.K), S)
    assert np.max(np.abs(c - np.arange(L.K + 1) / L.K)) < 1e-12


@pytest.mark.parametrize("S", [0, 1 << 10, 1 << 16])
def test_levels_of_two_valued_logits_by_hand(S):
    """theta = log 2 on the first half of the segments, 0 on the second:
    softmax gives 4/(3K) and 2/(3K); with the floor f = 1/(4S) (0 without
    a sample size) every mass becomes (q + f) / (1 + K f).  Hence
    c_{K/4} = (1/3 + K f/4) / (1 + K f), c_{K/2} = (2/3 + K f/2) / (1 + K f)
    and c_K = 1, checked before anything is set to 1."""
    th = np.zeros(L.K)
    th[: L.K // 2] = np.log(2.0)
    c = L.running_levels(th, S)
    f = 0.25 / S if S else 0.0
    K = L.K
    assert abs(c[K // 4] - (1 / 3 + K * f / 4) / (1 + K * f)) < 1e-12
    assert abs(c[K // 2] - (2 / 3 + K * f / 2) / (1 + K * f)) < 1e-12
    assert abs(c[K] - 1.0) < 1e-12
    assert abs(c[3 * K // 4] - (2 / 3 + 3 * K * f / 4 + 1 / 6) / (1 + K * f)) < 1e-12
    assert np.array_equal(L.levels(th, S)[:-1], np.minimum(c[:-1], 1.0))


def test_levels_refuse_masses_that_do_not_sum_to_one():
    """A wrong normaliser (planted in a copy of the export on the CPU) is
    seen at c_K instead of being hidden by setting c_K to 1."""
    th = np.zeros(L.K)
    q = L.softmax(th)
    fl = 0.25 / 1024
    wrong = (q + fl) / (1.0 + (L.K - 1) * fl)  # normaliser off by one segment's floor
    c = np.concatenate([[0.0], np.cumsum(wrong)])
    assert abs(c[-1] - 1.0) > 1e-6
    assert abs(L.running_levels(th, 1024)[-1] - 1.0) < 1e-12
