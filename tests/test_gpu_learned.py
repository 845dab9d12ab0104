"""Learned splitters on the GPU, through the C ABI, against the fp64 oracle.

* the model's forward pass and gradient (fp32 kernels) against the oracle's
  fp64 forward pass and gradient on the same fp32 weights and inputs;
* training: the loss falls, and follows the oracle's trajectory;
* the multiway pass: exact bucket-size parity with the oracle's bucket
  histogram for the same splitters, every key in its bucket, a permutation;
* the learned sort: bit-exact against the oracle's sort, with the model
  chosen, forced, or replaced by the sample's order statistics;
* what the trained network gains over the method without it (fewer bytes
  moved than the plain method, and lower imbalance than an untrained net).
"""
import numpy as np
import pytest

import workloads
from helpers import kv_index_check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# layout of the 1153 parameters: name -> slice
PARTS = {"W1": slice(0, 32), "b1": slice(32, 64), "W2": slice(64, 1088), "b2": slice(1088, 1120),
         "w3": slice(1120, 1152), "b3": slice(1152, 1153)}


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hsort


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _features(oracle_mod, x):
    """Inputs and targets of the model for a sample x (the oracle's reading)."""
    xs = np.sort(x)
    sc = oracle_mod.feature_scale(xs)
    mu, sd = oracle_mod.feature_stats(xs, sc)
    z = (np.arcsinh(xs / sc) - mu) / sd
    y = (np.arange(xs.size) + 0.5) / xs.size
    return z.astype(np.float32), y.astype(np.float32)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("m", [1000, 1 << 16])
def test_mlp_forward_matches_oracle(hs, oracle_mod, m):
    rng = np.random.default_rng(m)
    p32 = oracle_mod.mlp_init(5).astype(np.float32)
    p32[32:64] = rng.normal(0, 0.3, 32).astype(np.float32)  # non-zero biases too
    z = rng.normal(0, 1.5, m).astype(np.float32)
    got = hs.mlp_forward(_gpu(p32), _gpu(z)).cpu().numpy().astype(np.float64)
    want = oracle_mod.mlp_forward(p32.astype(np.float64), z.astype(np.float64))
    assert np.max(np.abs(got - want)) <= 1e-5


@pytest.mark.parametrize("m,dist", [(1000, "lognormal"), (1 << 16, "lognormal"), (1 << 16, "mixture"),
                                    (3 * 256 + 17, "normal")])
def test_mlp_grad_matches_oracle(hs, oracle_mod, m, dist):
    """Per-tensor relative L2 error of the fp32 gradient <= 1e-3."""
    x = workloads.f64(m, dist, seed=11)
    z, y = _features(oracle_mod, x)
    for p in (oracle_mod.mlp_init(3), oracle_mod.mlp_train(3, z.astype(np.float64), y.astype(np.float64), 30,
                                                            1e-2)[0]):
        p32 = p.astype(np.float32)
        g = hs.mlp_grad(_gpu(p32), _gpu(z), _gpu(y)).cpu().numpy().astype(np.float64)
        _, want = oracle_mod.mlp_loss_grad(p32.astype(np.float64), z.astype(np.float64), y.astype(np.float64))
        for name, sl in PARTS.items():
            assert _rel_l2(g[sl], want[sl]) <= 1e-3, (name, _rel_l2(g[sl], want[sl]))
        g2 = hs.mlp_grad(_gpu(p32), _gpu(z), _gpu(y)).cpu().numpy()
        assert np.array_equal(g.astype(np.float32), g2), "the gradient reduction is not deterministic"


def test_mlp_train_loss_falls_and_tracks_oracle(hs, oracle_mod):
    m, steps, lr, seed = 1 << 12, 200, 1e-2, 7
    x = workloads.f64(m, "lognormal", seed=12)
    z, y = _features(oracle_mod, x)
    p, loss = hs.mlp_train(_gpu(z), _gpu(y), steps, lr, seed)
    loss = loss.cpu().numpy().astype(np.float64)
    po, lo = oracle_mod.mlp_train(seed, z.astype(np.float64), y.astype(np.float64), steps, lr)
    # same initialisation: the first loss agrees to fp32 accuracy
    assert abs(loss[0] - lo[0]) <= 1e-5 * lo[0] + 1e-7
    assert loss[-1] < 0.2 * loss[0]
    assert np.all(np.isfinite(loss))
    # the trajectories stay close (fp32 against fp64 Adam)
    assert loss[-1] <= 1.5 * lo[-1] + 1e-5
    f_gpu = oracle_mod.mlp_forward(p.cpu().numpy().astype(np.float64), z.astype(np.float64))
    f_ora = oracle_mod.mlp_forward(po, z.astype(np.float64))
    assert np.max(np.abs(f_gpu - f_ora)) <= 0.05


def _bucket_of(keys_u64, d):
    r = np.searchsorted(d, keys_u64, side="left")
    eq = (r < d.size) & (d[np.minimum(r, max(d.size - 1, 0))] == keys_u64) if d.size else np.zeros(keys_u64.size,
                                                                                                     bool)
    return np.where(eq, 2 * r + 1, 2 * r)


@pytest.mark.parametrize("n,dist,k", [((1 << 20) + 333, "lognormal", 255), (100003, "zipf", 200),
                                      (5000, "normal", 1), (70000, "uniform", 0), (1 << 18, "mixture", 37)])
def test_multiway_bucket_parity(hs, oracle_mod, n, dist, k):
    x = workloads.f64(n, dist, seed=13)
    keys = oracle_mod.f64_order_keys(x)
    # splitters: distinct keys of the input (so equality buckets are used)
    rng = np.random.default_rng(14)
    d = np.unique(keys[rng.integers(0, n, 4 * k + 1)])[:k] if k else np.zeros(0, np.uint64)
    if d.size > 1:
        d = np.unique(d[np.linspace(0, d.size - 1, min(k, d.size)).astype(np.int64)])
    counts = oracle_mod.bucket_hist(keys, d)
    t = _gpu(x)
    starts = hs.multiway_partition_(t, _gpu(d.view(np.int64))).cpu().numpy().view(np.uint32).astype(np.int64)
    assert starts.size == 2 * d.size + 2
    assert np.array_equal(starts, np.concatenate([[0], np.cumsum(counts)])), "bucket starts differ"
    out = t.cpu().numpy()
    ok = oracle_mod.f64_order_keys(out)
    b = _bucket_of(ok, d)
    want_b = np.repeat(np.arange(2 * d.size + 1), counts)
    assert np.array_equal(b, want_b), "a key is outside its bucket"
    assert np.array_equal(np.sort(ok), np.sort(keys)), "not a permutation"


def test_multiway_empty(hs):
    t = torch.empty(0, dtype=torch.float64, device="cuda")
    d = torch.tensor([5, 9], dtype=torch.int64, device="cuda")
    starts = hs.multiway_partition_(t, d).cpu().numpy()
    assert np.array_equal(starts, np.zeros(6, np.int32))


def _sort_learned(hs, x, **kw):
    t = _gpu(x)
    st = hs.sort_(t, opts=hs.learned_opts(**kw), stats=True)
    torch.cuda.synchronize()
    return t.cpu().numpy(), st


@pytest.mark.parametrize("dist", ["lognormal", "zipf", "mixture", "uniform", "sorted"])
def test_learned_sort_f64_bit_exact(hs, oracle_mod, dist):
    n = (1 << 20) + 777
    x = workloads.f64(n, dist, seed=21)
    got, st = _sort_learned(hs, x, seed=3)
    want = oracle_mod.sort_f64(x)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    assert 1 <= st["splitters"] <= 255
    assert st["learn_ms"] > 0 and st["multiway_ms"] > 0
    assert st["model_imbalance"] > 0 and st["sample_imbalance"] > 0
    chose_model = st["model_imbalance"] <= 1.25 * st["sample_imbalance"] * (1 + 1e-6)
    assert st["fallback_used"] == (0 if chose_model else 1)
    assert np.isfinite(st["final_loss"]) and st["final_loss"] < 0.05


@pytest.mark.parametrize("flags", ["model", "sample"])
def test_learned_forced_choice_bit_exact(hs, oracle_mod, flags):
    n = 1 << 19
    x = workloads.f64(n, "mixture", seed=22)
    f = hs.LEARN_FORCE_MODEL if flags == "model" else hs.LEARN_FORCE_SAMPLE
    got, st = _sort_learned(hs, x, flags=f)
    assert np.array_equal(got.view(np.uint64), oracle_mod.sort_f64(x).view(np.uint64))
    assert st["fallback_used"] == (0 if flags == "model" else 1)
    if flags == "sample":
        assert st["model_imbalance"] == -1.0


def test_learned_f64_specials(hs, oracle_mod):
    x = np.concatenate([workloads.f64_specials(), workloads.f64(200000, "normal", seed=23),
                        workloads.f64_specials()])
    got, _ = _sort_learned(hs, x)
    assert np.array_equal(got.view(np.uint64), oracle_mod.sort_f64(x).view(np.uint64))


def test_learned_i32_and_kv(hs, oracle_mod):
    a = workloads.uniform_i32((1 << 20) + 5, seed=24)
    t = _gpu(a)
    st = hs.sort_(t, opts=hs.learned_opts(), stats=True)
    assert np.array_equal(t.cpu().numpy(), oracle_mod.sort_i32(a))
    assert st["splitters"] > 0
    keys, vals = workloads.kv_dup_i32((1 << 20) + 9, seed=25, ndistinct=1 << 12)
    kt, vt = _gpu(keys), _gpu(vals)
    hs.sort_kv_(kt, vt, opts=hs.learned_opts())
    ko, vo = kt.cpu().numpy(), vt.cpu().numpy()
    ok, _ = oracle_mod.sort_kv_i32(keys, vals)
    assert np.array_equal(ko, ok)
    kv_index_check(keys, ko, vo)


def test_learned_deterministic(hs):
    x = workloads.f64(1 << 19, "lognormal", seed=26)
    _, s1 = _sort_learned(hs, x, seed=9)
    _, s2 = _sort_learned(hs, x, seed=9)
    for k in ("splitters", "model_imbalance", "sample_imbalance", "final_loss", "bytes_alg", "fallback_used"):
        assert s1[k] == s2[k], k


def test_learned_small_inputs_run_plain(hs, oracle_mod):
    for n in (2, 100, 8192):
        x = workloads.f64(n, "lognormal", seed=27)
        got, st = _sort_learned(hs, x)
        assert np.array_equal(got.view(np.uint64), oracle_mod.sort_f64(x).view(np.uint64))
        assert st["splitters"] == 0


def test_trained_network_gain(hs):
    """What the trained network gains over the method without it, on the
    lognormal(0, 2) workload: the judge keeps the model (its held-out bucket
    imbalance is within 1.25 times that of the sample's order statistics),
    the learned sort moves fewer bytes than the plain method (one multiway
    pass instead of about eight partition levels), and training lowers the
    imbalance against a one-step network."""
    n = 1 << 22
    x = workloads.f64(n, "lognormal", seed=6)
    plain = hs.sort_(_gpu(x), stats=True)
    learned = _sort_learned(hs, x, seed=100)[1]
    untrained = _sort_learned(hs, x, seed=100, flags=hs.LEARN_FORCE_MODEL, steps=1)[1]
    print(f"\nlognormal 2^22: model imbalance {learned['model_imbalance']:.3f}, sample order statistics "
          f"{learned['sample_imbalance']:.3f}, one-step model {untrained['model_imbalance']:.3f}; bytes/key plain "
          f"{plain['bytes_alg'] / n:.1f}, learned {learned['bytes_alg'] / n:.1f}", flush=True)
    assert learned["fallback_used"] == 0, "the judge fell back to the order statistics"
    assert learned["model_imbalance"] <= 1.25 * learned["sample_imbalance"] * (1 + 1e-6)
    assert learned["bytes_alg"] < 0.75 * plain["bytes_alg"], (learned["bytes_alg"], plain["bytes_alg"])
    assert learned["model_imbalance"] < untrained["model_imbalance"]
