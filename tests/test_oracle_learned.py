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
    mu, sd = oracle_mod.feature_stats(x)
    assert abs(mu - np.arcsinh(x).mean()) < 1e-12 and abs(sd - np.arcsinh(x).std()) < 1e-12


def _cdf_data(oracle_mod, dist, m=4096, seed=8):
    x = np.sort(workloads.f64(m, dist, seed=seed))
    mu, sd = oracle_mod.feature_stats(x)
    z = (np.arcsinh(x) - mu) / sd
    y = (np.arange(m) + 0.5) / m
    return x, z, y, mu, sd


@pytest.mark.parametrize("dist", ["lognormal", "mixture"])
def test_training_lowers_the_loss(oracle_mod, dist):
    x, z, y, mu, sd = _cdf_data(oracle_mod, dist)
    p, losses = oracle_mod.mlp_train(5, z, y, 150, 1e-2)
    assert losses[-1] < 0.2 * losses[0]
    assert np.all(np.isfinite(p))


def _key_to_z(oracle_mod, keys, mu, sd):
    bits = np.where(keys >> np.uint64(63) == 1, keys & np.uint64((1 << 63) - 1), ~keys)
    x = bits.view(np.float64)
    return (np.arcsinh(x) - mu) / sd


def test_inversion_bisection_postcondition(oracle_mod):
    x, z, y, mu, sd = _cdf_data(oracle_mod, "lognormal")
    p, _ = oracle_mod.mlp_train(5, z, y, 100, 1e-2)
    keys = oracle_mod.f64_order_keys(x)
    kmin, kmax = int(keys.min()), int(keys.max())
    nb = 64
    s = oracle_mod.invert_f64(p, mu, sd, kmin, kmax, nb)
    assert np.all(np.diff(s.astype(np.float64)) >= 0)  # running maximum applied
    # recompute the raw bisection result for a few targets and check the
    # invariant (F(K) >= q or K == kmax) and (K == kmin or F(K-1) < q)
    raw = oracle_mod.invert_f64(p, mu, sd, kmin, kmax, 2)[0]  # q = 1/2, single splitter
    f = oracle_mod.mlp_forward(p, _key_to_z(oracle_mod, np.array([raw, raw - 1], dtype=np.uint64), mu, sd))
    assert (f[0] >= 0.5 or raw == kmax) and (raw == kmin or f[1] < 0.5)
    # a trained model's median splitter sits near the sample median
    med = float(np.uint64(raw).view(np.uint64))
    rank = np.searchsorted(keys.astype(np.float64), med) / keys.size
    assert 0.3 < rank < 0.7


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
