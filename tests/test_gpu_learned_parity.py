"""The learned front end, step by step, against the oracle (hs_learn_debug_f64).

Every intermediate the GPU produces before the multiway pass is recomputed
by the oracle from the same input:
* the training and held-out samples are the keys at the oracle's splitmix64
  sample indices (the training sample sorted by the oracle);
* the order statistics (the sampled-pivot fallback) are the oracle's ranks of
  that sorted sample, the feature's scale and normalisation the oracle's;
* the judge: its held-out bucket counts for both splitter sets equal the
  oracle's bucket histogram of the held-out keys over the oracle's running
  maximum and de-duplication of the same splitters; the imbalances and the
  decision follow from those counts in the judge's fp32 arithmetic;
* the model's splitters: each is a key of the sorted sample, of rank i with
  F(t_i) >= j/256 and F(t_{i-1}) < j/256 under the oracle's fp64 forward
  pass on the GPU's fp32 weights (within the fp32 forward tolerance), and
  within 16 ranks of the oracle's bisection on the same model, unless the
  model is not monotone there and both are crossings of j/256.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NB_MAX = 511
NB = 256
FWD_TOL = 2e-5     # fp32 forward pass against the fp64 oracle (measured error <= 1e-5)
RANK_TOL = 16      # sample ranks between the GPU's and the oracle's splitter


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hsort


def _key_value(k):
    """float64 value of totalOrder order words (uint64 array)."""
    k = np.asarray(k, dtype=np.uint64)
    bits = np.where(k >> np.uint64(63), k & np.uint64((1 << 63) - 1), ~k)
    return bits.view(np.float64)


def _model_at(oracle_mod, p, sc, mu, sd, words):
    z = (np.arcsinh(np.clip(_key_value(words) / sc, -1.7976931348623157e308, 1.7976931348623157e308)) - mu) / sd
    return oracle_mod.mlp_forward(p, z.astype(np.float32).astype(np.float64))


CASES = [((1 << 20) + 77, "lognormal", 21, 0), ((1 << 20) + 5, "zipf", 22, 0), (1 << 20, "mixture", 23, 0),
         (300001, "uniform", 24, 0), (1 << 19, "normal", 25, 1), (100000, "lognormal", 26, 2),
         (1 << 22, "lognormal", 6, 0), (1 << 22, "zipf", 7, 0), (1 << 22, "mixture", 8, 0)]


@pytest.mark.parametrize("n,dist,seed,flags", CASES)
def test_front_end_matches_oracle(hs, oracle_mod, n, dist, seed, flags):
    x = workloads.f64(n, dist, seed=seed)
    opts = hs.learned_opts(seed=1000 + seed, flags=flags)
    print(f"learn_debug n={n} dist={dist} seed={seed} flags={flags}", flush=True)
    xd = torch.from_numpy(x).to("cuda")
    out = hs.learn_debug(xd, opts)
    assert np.array_equal(xd.cpu().numpy().view(np.uint64), x.view(np.uint64)), "the keys were changed"
    m, h = out["m"], out["h"]
    assert (m, h) == (1 << 16, 1 << 14)

    # samples at the oracle's indices
    ti = oracle_mod.sample_indices(opts.seed, n, m)
    hi = oracle_mod.sample_indices(opts.seed + 1, n, h)
    train = out["train_sorted"].cpu().numpy()
    assert np.array_equal(train.view(np.uint64), oracle_mod.sort_f64(x[ti]).view(np.uint64))
    hold = out["holdout"].cpu().numpy().view(np.uint64)
    assert np.array_equal(hold, oracle_mod.f64_order_keys(x[hi]))

    # order statistics, extremes, feature statistics
    tk = oracle_mod.f64_order_keys(train)
    ss = out["sample_split"].cpu().numpy().view(np.uint64)
    assert np.array_equal(ss, tk[(np.arange(1, NB, dtype=np.int64) * m) // NB])
    assert out["smin"] == int(tk[0]) and out["smax"] == int(tk[-1])
    sc = oracle_mod.feature_scale(train)
    assert abs(out["scale"] - sc) <= 1e-12 * sc
    mu, sd = oracle_mod.feature_stats(train, out["scale"])
    assert abs(out["mu"] - mu) <= 1e-12 * max(1.0, abs(mu))
    assert abs(out["sd"] - sd) <= 1e-12 * max(1.0, abs(sd))

    # the judge: counts, imbalances, decision
    counts = out["counts"].cpu().numpy().astype(np.int64)
    ideal = np.float32(h) / np.float32(NB)
    ds = oracle_mod.dedupe(ss)
    cs = oracle_mod.bucket_hist(hold, ds)
    assert np.array_equal(counts[NB_MAX:NB_MAX + cs.size], cs), "order-statistic bucket counts differ"
    assert counts[NB_MAX + cs.size:].sum() == 0
    imb_s = np.float32(cs[0::2].max()) / ideal
    assert np.float32(out["sample_imbalance"]) == imb_s
    chosen = out["chosen"].cpu().numpy().view(np.uint64)
    if flags == 2:
        assert out["use_model"] == 0 and out["model_imbalance"] == -1.0
        assert out["k"] == ds.size and np.array_equal(chosen[:ds.size], ds)
        return
    ms = out["model_split"].cpu().numpy().view(np.uint64)
    dm = oracle_mod.dedupe(np.maximum.accumulate(ms))
    cm = oracle_mod.bucket_hist(hold, dm)
    assert np.array_equal(counts[:cm.size], cm), "model bucket counts differ"
    assert counts[cm.size:NB_MAX].sum() == 0
    imb_m = np.float32(cm[0::2].max()) / ideal
    assert np.float32(out["model_imbalance"]) == imb_m
    use = flags == 1 or bool(imb_m <= np.float32(1.25) * imb_s)
    assert bool(out["use_model"]) == use
    want = dm if use else ds
    assert out["k"] == want.size and np.array_equal(chosen[:want.size], want)

    # the model's splitters: sample keys meeting the search's postcondition
    # under the oracle's forward pass
    p = out["params"].cpu().numpy().astype(np.float64)
    q = np.arange(1, NB, dtype=np.float64) / NB
    assert np.all(np.isin(ms, tk)), "a model splitter is not a sample key"
    i_gpu = np.searchsorted(tk, ms, side="left")
    Fs = _model_at(oracle_mod, p, out["scale"], out["mu"], out["sd"], tk)
    ok_at = (i_gpu == m - 1) | (Fs[i_gpu] >= q - FWD_TOL)
    ok_below = (i_gpu == 0) | (Fs[np.maximum(i_gpu - 1, 0)] < q + FWD_TOL)
    assert ok_at.all(), np.flatnonzero(~ok_at)[:8]
    assert ok_below.all(), np.flatnonzero(~ok_below)[:8]
    # ... and close to the oracle's bisection of the same model: where the
    # two are far apart, both must be crossings of j/256 (the model is not
    # monotone there, and either is a valid answer of the search)
    i_ora = np.array([oracle_mod.invert_one_f64(p, out["scale"], out["mu"], out["sd"], tk, qq) for qq in q])
    assert np.array_equal(np.maximum.accumulate(tk[i_ora]),
                          oracle_mod.invert_f64(p, out["scale"], out["mu"], out["sd"], tk))
    far = np.abs(i_gpu - i_ora) > RANK_TOL
    crossing = (((i_ora == m - 1) | (Fs[i_ora] >= q - FWD_TOL)) &
                ((i_ora == 0) | (Fs[np.maximum(i_ora - 1, 0)] < q + FWD_TOL)))
    assert crossing[far].all(), np.flatnonzero(far & ~crossing)[:8]
    print(f"  {int(far.sum())} splitters at another crossing than the oracle's; model imbalance {imb_m:.3f}, "
          f"order statistics {imb_s:.3f}, use_model {int(use)}, final loss {out['final_loss']:.3g}", flush=True)
