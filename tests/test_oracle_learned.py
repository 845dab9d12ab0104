"""Pins of the oracle's learned-splitter part (fp64) against facts fixed
outside it: published generator outputs, finite differences, closed forms of
special cases, optimizer invariants, the bisection postcondition and numpy."""
import math
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs(oracle_mod):
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert [oracle_mod.splitmix64_at(0, k) for k in range(3)] == vals


def test_sample_indices_range_and_uniformity(oracle_mod):
    n = 1000
    idx = oracle_mod.sample_indices(12345, n, 200000)
    assert idx.min() >= 0 and idx.max() < n
    counts = np.bincount(idx, minlength=n)
    chi2 = ((counts - 200.0) ** 2 / 200.0).sum()
    assert 800 < chi2 < 1200  # 999 degrees of freedom


def _tiny_params(entries):
    p = np.zeros(oracle_mod_nparam(), dtype=np.float64)
    for k, v in entries.items():
        p[k] = v
    return p


def oracle_mod_nparam():
    return 1153


H = 32
W1, B1, W2, B2, W3, B3 = 0, 32, 64, 64 + 1024, 64 + 1024 + 32, 64 + 1024 + 64


def test_forward_special_cases(oracle_mod):
    z = np.linspace(-3, 3, 13)
    # all zero: sigmoid(0)
    assert np.allclose(oracle_mod.mlp_forward(np.zeros(1153), z), 0.5, atol=0, rtol=0)
    # one path through unit 5 of layer 1 and unit 3 of layer 2 (row = output unit)
    a, b1, c, b2, w, b3 = 0.7, -0.2, 1.3, 0.1, -2.0, 0.25
    p = _tiny_params({W1 + 5: a, B1 + 5: b1, W2 + 3 * H + 5: c, B2 + 3: b2, W3 + 3: w, B3: b3})
    expect = [1 / (1 + math.exp(-(w * math.tanh(c * math.tanh(a * t + b1) + b2) + b3))) for t in z]
    got = oracle_mod.mlp_forward(p, z)
    # other hidden units are tanh(0 * z + 0) = 0 or tanh(b2 only) and carry weight 0
    assert np.allclose(got, expect, rtol=1e-14, atol=1e-15)


def test_gradient_matches_finite_differences(oracle_mod):
    g = workloads.rng(3)
    p = oracle_mod.mlp_init(11) + g.normal(0, 0.05, 1153)
    z = g.normal(0, 1.2, 64)
    y = np.clip(0.5 + 0.3 * z + g.normal(0, 0.05, 64), 0.01, 0.99)
    _, grad = oracle_mod.mlp_loss_grad(p, z, y)
    h = 1e-6
    worst = 0.0
    for i in list(range(0, 1153, 7)) + [B3, W1, W2 + 1023]:
        e = np.zeros(1153)
        e[i] = h
        lp, _ = oracle_mod.mlp_loss_grad(p + e, z, y)
        lm, _ = oracle_mod.mlp_loss_grad(p - e, z, y)
        fd = (lp - lm) / (2 * h)
        worst = max(worst, abs(fd - grad[i]) / max(1e-7, abs(fd) + abs(grad[i])))
    assert worst < 1e-6


def test_adam_first_steps_closed_form(oracle_mod):
    """With zero moments and a gradient held fixed, bias correction makes the
    corrected moments equal g and g^2 at every step, so each step moves a
    parameter by lr * g / (|g| + eps)."""
    g = workloads.rng(4)
    p = g.normal(0, 1, 1153)
    grad = g.normal(0, 1e-3, 1153)
    mom = np.zeros(1153)
    vel = np.zeros(1153)
    lr = 1e-2
    q = p.copy()
    for t in (1, 2, 3):
        oracle_mod.adam_step(q, mom, vel, grad, t, lr)
        expect = p - t * lr * grad / (np.abs(grad) + 1e-8)
        assert np.allclose(q, expect, rtol=1e-10, atol=1e-12)


def test_init_is_xavier_uniform(oracle_mod):
    p = oracle_mod.mlp_init(99)
    a1, a2, a3 = math.sqrt(6 / 33), math.sqrt(6 / 64), math.sqrt(6 / 33)
    assert np.all(np.abs(p[W1:W1 + H]) <= a1) and np.all(np.abs(p[W2:W2 + 1024]) <= a2)
    assert np.all(np.abs(p[W3:W3 + H]) <= a3)
    assert np.all(p[B1:B1 + H] == 0) and np.all(p[B2:B2 + H] == 0) and p[B3] == 0
    assert abs(np.var(p[W2:W2 + 1024]) - a2 * a2 / 3) < 0.15 * a2 * a2 / 3
    assert not np.array_equal(p, oracle_mod.mlp_init(100))


def test_feature_stats_match_numpy(oracle_mod):
    x = workloads.f64(5000, "lognormal", seed=6)
    for sc in (1.0, 0.01, 3.5):
        mu, sd = oracle_mod.feature_stats(x, sc)
        f = np.arcsinh(x / sc)
        assert abs(mu - f.mean()) < 1e-12 * max(1.0, abs(f.mean())) and abs(sd - f.std()) < 1e-12 * f.std()
    # a quotient beyond the largest double is clamped (asinh stays finite)
    big = np.array([1e308, -1e308, 1.0])
    mu, sd = oracle_mod.feature_stats(big, 1e-10)
    assert np.isfinite(mu) and np.isfinite(sd)


def test_feature_scale_branches(oracle_mod):
    """The scale rule on its three branches: a positive sample spanning more
    than three decades takes its 1% order statistic, a negative one minus its
    99% order statistic, anything else its standard deviation."""
    m = 1 << 14
    x = np.sort(workloads.f64(m, "lognormal", seed=3))
    assert oracle_mod.feature_scale(x) == x[int(0.01 * m)]
    neg = np.sort(-x)
    assert oracle_mod.feature_scale(neg) == -neg[int(0.99 * m)]
    for dist in ("normal", "uniform", "mixture"):
        y = np.sort(workloads.f64(m, dist, seed=4))
        assert abs(oracle_mod.feature_scale(y) - y.std()) <= 1e-12 * y.std()
    # positive, but within three decades: the standard deviation
    u = np.sort(1.0 + workloads.f64(m, "uniform", seed=5))
    assert abs(oracle_mod.feature_scale(u) - u.std()) <= 1e-12 * u.std()
    assert oracle_mod.feature_scale(np.full(100, 7.0)) == 1.0  # no spread: 1


def test_training_points(oracle_mod):
    """min(4096, m) evenly spaced ranks of the sorted sample."""
    for m in (1024, 4096, 1 << 16, 100000):
        r = oracle_mod.training_points(m)
        nt = min(4096, m)
        assert r.size == nt and r[0] >= 0 and r[-1] < m
        assert np.all(np.diff(r) >= m // nt) and np.all(np.diff(r) <= -(-m // nt))
    assert np.array_equal(oracle_mod.training_points(1 << 16), np.arange(4096) * 16 + 8)


def _cdf_data(oracle_mod, dist, m=4096, seed=8):
    x = np.sort(workloads.f64(m, dist, seed=seed))
    sc = oracle_mod.feature_scale(x)
    mu, sd = oracle_mod.feature_stats(x, sc)
    z = (np.arcsinh(x / sc) - mu) / sd
    y = (np.arange(m) + 0.5) / m
    return x, z, y, sc, mu, sd


@pytest.mark.parametrize("dist", ["lognormal", "mixture"])
def test_training_lowers_the_loss(oracle_mod, dist):
    x, z, y, sc, mu, sd = _cdf_data(oracle_mod, dist)
    p, losses = oracle_mod.mlp_train(5, z, y, 150, 1e-2)
    assert losses[-1] < 0.2 * losses[0]
    assert np.all(np.isfinite(p))


def _key_to_z(oracle_mod, keys, sc, mu, sd):
    bits = np.where(keys >> np.uint64(63) == 1, keys & np.uint64((1 << 63) - 1), ~keys)
    x = bits.view(np.float64)
    return (np.arcsinh(x / sc) - mu) / sd


def test_inversion_bisection_postcondition(oracle_mod):
    x, z, y, sc, mu, sd = _cdf_data(oracle_mod, "lognormal")
    p, _ = oracle_mod.mlp_train(5, z, y, 100, 1e-2)
    keys = oracle_mod.f64_order_keys(x)  # x is sorted
    nb = 64
    s = oracle_mod.invert_f64(p, sc, mu, sd, keys, nb)
    assert np.all(np.diff(s.astype(np.float64)) >= 0)  # running maximum applied
    assert np.all(np.isin(s, keys))  # every splitter is a sample key
    # every raw bisection result meets the invariant
    # (F(t_i) >= q or i == m - 1) and (i == 0 or F(t_{i-1}) < q)
    F = oracle_mod.mlp_forward(p, _key_to_z(oracle_mod, keys, sc, mu, sd))
    for j in range(1, nb):
        q = j / nb
        i = oracle_mod.invert_one_f64(p, sc, mu, sd, keys, q)
        assert (F[i] >= q or i == keys.size - 1) and (i == 0 or F[i - 1] < q), j
    # a trained model's median splitter sits near the sample median
    i = oracle_mod.invert_one_f64(p, sc, mu, sd, keys, 0.5)
    assert 0.3 < i / keys.size < 0.7
    # on a monotone stretch the bisection gives the first rank reaching q
    # (brute force over the ranks)
    mono = np.all(np.diff(F) >= 0)
    if mono:
        for j in range(1, nb):
            assert s[j - 1] == keys[np.argmax(F >= j / nb)] or not np.any(F >= j / nb)


def test_bucket_histogram_matches_numpy(oracle_mod):
    g = workloads.rng(9)
    keys = g.integers(0, 1000, 50000).astype(np.uint64)
    s = np.sort(g.integers(0, 1000, 40)).astype(np.uint64)
    d = oracle_mod.dedupe(s)
    assert np.array_equal(d, np.unique(s))
    counts = oracle_mod.bucket_hist(keys, d)
    r = np.searchsorted(d, keys, side="left")
    eq = (r < d.size) & (d[np.minimum(r, d.size - 1)] == keys)
    expect = np.bincount(np.where(eq, 2 * r + 1, 2 * r), minlength=2 * d.size + 1)
    assert np.array_equal(counts, expect)
    assert counts.sum() == keys.size
    # every key of an equality bucket equals its splitter
    for i in range(d.size):
        assert counts[2 * i + 1] == np.count_nonzero(keys == d[i])
