"""Pins of the CPU oracle against facts fixed outside the oracle itself.

Each test checks the oracle against something the paper or mathematics fixes:
the paper's worked example and printed networks (golden fixtures), brute
force on tiny inputs, library sorts as special cases, closed forms and
invariants.  None of these re-types the oracle's own code.
"""
import itertools
import os

import numpy as np
import pytest

import workloads
from helpers import insertion_sort, is_sorted, kv_index_check, pair_multiset_equal

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


# ---------------------------------------------------------------- worked example

def test_fig1_example_hybrid(oracle_mod):
    rows = dict(r.split(":", 1) for r in _golden("fig1_quicksort_example.txt"))
    inp = np.array(rows["input"].split(), dtype=np.int32)
    out = np.array(rows["output"].split(), dtype=np.int32)
    for leaf in (1, 2, 256):
        assert np.array_equal(oracle_mod.sort_i32(inp, leaf=leaf), out)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("leaf", [1, 2, 3, 256])
def test_bruteforce_all_small_arrays(oracle_mod, leaf):
    """Every array of length 0..8 over {0,1,2} (9,841 arrays) against insertion sort."""
    for n in range(0, 9):
        for t in itertools.product((0, 1, 2), repeat=n):
            a = np.array(t, dtype=np.int32)
            got = oracle_mod.sort_i32(a, leaf=leaf)
            assert got.tolist() == insertion_sort(t), (t, leaf)


def test_bruteforce_random_small(oracle_mod):
    g = workloads.rng(11)
    for trial in range(400):
        n = int(g.integers(0, 65))
        a = g.integers(-5, 6, n).astype(np.int32) if trial % 2 else \
            g.integers(-(2 ** 31), 2 ** 31, n, dtype=np.int32)
        leaf = int(g.choice([1, 2, 4, 16, 256]))
        assert oracle_mod.sort_i32(a, leaf=leaf).tolist() == insertion_sort(a.tolist())


# ---------------------------------------------------------------- library special cases

@pytest.mark.parametrize("leaf", [1, 16, 256])
def test_i32_matches_numpy_sort(oracle_mod, leaf):
    for n in (1000, 4097, 65536):
        a = workloads.uniform_i32(n, seed=n + leaf)
        assert np.array_equal(oracle_mod.sort_i32(a, leaf=leaf), np.sort(a))
    a = workloads.rng(3).integers(-3, 4, 30000).astype(np.int32)  # heavy duplicates
    assert np.array_equal(oracle_mod.sort_i32(a, leaf=leaf), np.sort(a))


def test_i32_extremes(oracle_mod):
    a = np.array([2 ** 31 - 1, -(2 ** 31), 0, -1, 1, 2 ** 31 - 1, -(2 ** 31)] * 100, dtype=np.int32)
    for leaf in (1, 256):
        assert np.array_equal(oracle_mod.sort_i32(a, leaf=leaf), np.sort(a))


@pytest.mark.parametrize("dist", ["uniform", "normal", "sorted", "reverse", "lognormal", "mixture"])
def test_f64_matches_numpy_sort(oracle_mod, dist):
    """Without NaNs and zeros, totalOrder is the numeric order: numpy decides."""
    a = workloads.f64(50000, dist, seed=5)
    a = a[a != 0.0]
    got = oracle_mod.sort_f64(a)
    assert np.array_equal(got.view(np.uint64), np.sort(a).view(np.uint64))


def test_f64_total_order_specials(oracle_mod):
    """The IEEE 754-2008 totalOrder table (golden) fixes the order of NaNs,
    infinities, signed zeros and denormals."""
    expect = np.array([int(r.split()[0], 16) for r in _golden("ieee754_total_order.txt")],
                      dtype=np.uint64)
    g = workloads.rng(7)
    reps = np.repeat(expect, 5)
    shuffled = reps[g.permutation(reps.size)]
    got = oracle_mod.sort_f64(shuffled.view(np.float64)).view(np.uint64)
    assert np.array_equal(got, reps)
    # the key map is order-preserving and invertible on the same table
    keys = [oracle_mod.key_f64(int(b)) for b in expect]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    assert all(oracle_mod.unkey_f64(k) == int(b) for k, b in zip(keys, expect))


def test_f64_key_random_pairs(oracle_mod):
    """On random non-NaN pairs the key order agrees with the float '<'."""
    g = workloads.rng(8)
    x = np.concatenate([g.standard_normal(2000) * 10.0 ** g.integers(-300, 300, 2000),
                        workloads.f64_specials()[4:]])
    bits = x.view(np.uint64)
    k = np.array([oracle_mod.key_f64(int(b)) for b in bits], dtype=np.uint64)
    i, j = g.integers(0, x.size, (2, 20000))
    lt = x[i] < x[j]
    assert np.all(k[i][lt] < k[j][lt])
    nz = ~((x[i] == 0) & (x[j] == 0))
    eq = (x[i] == x[j]) & nz
    assert np.all(k[i][eq] == k[j][eq])


# ---------------------------------------------------------------- key/value

def test_kv_exact_index_check(oracle_mod):
    keys, vals = workloads.kv_dup_i32(200000, seed=4, ndistinct=1 << 10, force_extremes=True)
    k, v = oracle_mod.sort_kv_i32(keys, vals)
    assert np.array_equal(k, np.sort(keys))
    kv_index_check(keys, k, v)


def test_kv_bruteforce_ties(oracle_mod):
    """Small kv arrays with many ties: keys sorted, pairs preserved."""
    g = workloads.rng(13)
    for _ in range(300):
        n = int(g.integers(0, 600))
        k0 = g.integers(0, 4, n).astype(np.int32)
        if n:
            k0[g.integers(0, n, max(1, n // 10))] = 2 ** 31 - 1  # real keys equal to the pad key
        v0 = g.integers(-1000, 1000, n).astype(np.int32)
        leaf = int(g.choice([1, 8, 256]))
        k, v = oracle_mod.sort_kv_i32(k0, v0, leaf=leaf)
        assert k.tolist() == insertion_sort(k0.tolist())
        assert pair_multiset_equal(k0, v0, k, v)


# ---------------------------------------------------------------- partition

def test_partition_contract(oracle_mod):
    """Algorithm 3's contract: keys <= pivot land left, the result is their
    count (closed form), and the keys are permuted."""
    g = workloads.rng(21)
    for trial in range(1200):
        n = int(g.integers(0, 3000))
        a = g.integers(-50, 50, n).astype(np.int32) if trial % 3 else \
            g.integers(-(2 ** 31), 2 ** 31, n, dtype=np.int32)
        pivot = int(a[g.integers(0, n)]) if n and trial % 4 else int(g.integers(-60, 60))
        expect_k = int(np.count_nonzero(a <= pivot))
        out, k = oracle_mod.partition_le_i32(a, pivot)
        assert k == expect_k
        assert np.all(out[:k] <= pivot) and np.all(out[k:] > pivot)
        assert np.array_equal(np.sort(out), np.sort(a))


# ---------------------------------------------------------------- networks

def _paper_layers(rows):
    """Comparator pairs of a printed layer: the list is highest lane first, so
    lane i's partner is list[::-1][i]; the masked lane takes the maximum."""
    layers = []
    for r in rows:
        perm_s, mask_s = r.split("|")
        perm = [int(x) for x in perm_s.split(":")[1].split()][::-1]
        mask = int(mask_s.split(":")[1], 16)
        pairs = []
        for i, p in enumerate(perm):
            assert perm[p] == i, "not an involution"
            if i < p:
                takes_max_i = (mask >> i) & 1
                takes_max_p = (mask >> p) & 1
                assert takes_max_i != takes_max_p, "both lanes take the same side"
                lo, hi = (i, p) if not takes_max_i else (p, i)
                pairs.append((lo, hi))
        layers.append(pairs)
    return layers


def _apply_layers(keys, vals, layers):
    k = list(keys)
    v = list(vals)
    for pairs in layers:
        for lo, hi in pairs:
            if k[lo] > k[hi]:
                k[lo], k[hi] = k[hi], k[lo]
                v[lo], v[hi] = v[hi], v[lo]
    return k, v


def test_alg1_network_is_oracle_network(oracle_mod):
    """Algorithm 1's printed lists and the listing's masks give the oracle's
    8-line network comparator for comparator: on every 0-1 key input with
    distinct values (so that any difference in which pair is compared shows in
    where the values end up) both produce the same keys AND values."""
    layers = _paper_layers(_golden("alg1_bitonic_one_vector.txt"))
    for lo_hi in layers:
        for lo, hi in lo_hi:
            assert lo < hi, "the minimum goes to the lower lane"
    vals = list(range(8))
    for m in range(256):
        keys = [(m >> i) & 1 for i in range(8)]
        pk, pv = _apply_layers(keys, vals, layers)
        ok, ov = oracle_mod.bitonic_apply(np.array(keys, dtype=np.uint64),
                                          np.array(vals, dtype=np.int32))
        assert pk == sorted(keys)
        assert pk == ok.tolist() and pv == ov.tolist(), m


def test_alg1_lane0_first_reading_is_invalid(oracle_mod):
    """Negative control: reading the lists lowest lane first pairs lanes of
    equal mask parity, which is not a compare-exchange."""
    rows = _golden("alg1_bitonic_one_vector.txt")
    bad = []
    for r in rows:
        perm_s, mask_s = r.split("|")
        bad.append("perm: " + " ".join(perm_s.split(":")[1].split()[::-1]) + " |" + mask_s)
    with pytest.raises(AssertionError):
        _paper_layers(bad)


def test_alg2_network_is_oracle_network(oracle_mod):
    rows = _golden("alg2_bitonic_two_vectors.txt")
    one = _paper_layers(_golden("alg1_bitonic_one_vector.txt"))
    layers = [[(lo, hi) for lo, hi in p] + [(lo + 8, hi + 8) for lo, hi in p] for p in one]
    cross = [int(x) for x in rows[0].split(":")[1].split()][::-1]
    layers.append([(i, 8 + cross[i]) for i in range(8)])
    for r in rows[1:]:
        perm = [int(x) for x in r.split(":")[1].split()][::-1]
        pairs = [(i, p) for i, p in enumerate(perm) if i < p]
        layers.append(pairs + [(lo + 8, hi + 8) for lo, hi in pairs])
    vals = list(range(16))
    for m in range(1 << 16):
        keys = [(m >> i) & 1 for i in range(16)]
        pk, pv = _apply_layers(keys, vals, layers)
        if m % 97 == 0 or m in (0, 0xFFFF, 0x00FF, 0xFF00):
            ok, ov = oracle_mod.bitonic_apply(np.array(keys, dtype=np.uint64),
                                              np.array(vals, dtype=np.int32))
            assert pk == ok.tolist() and pv == ov.tolist(), m
        assert pk == sorted(keys)


@pytest.mark.parametrize("logn", [0, 1, 2, 3, 4])
def test_network_zero_one_exhaustive(oracle_mod, logn):
    assert oracle_mod.bitonic_exhaustive_failures(logn) == 0


@pytest.mark.parametrize("logn", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_merger_zero_one(oracle_mod, logn):
    """The last stage merges any two sorted halves (all (N/2+1)^2 0-1 cases)."""
    assert oracle_mod.bitonic_merger_failures(logn) == 0


def test_network_pads_never_move_kv(oracle_mod):
    """With the strict swap, pads (greatest key) placed at the top never leave
    their slots, even when real keys equal the pad key."""
    g = workloads.rng(17)
    for _ in range(200):
        logn = int(g.integers(1, 9))
        n = 1 << logn
        m = int(g.integers(1, n + 1))
        keys = g.integers(0, 3, n).astype(np.uint64)
        keys[g.random(n) < 0.3] = np.uint64(2 ** 64 - 1)
        keys[m:] = np.uint64(2 ** 64 - 1)
        vals = np.arange(n, dtype=np.int32)
        k, v = oracle_mod.bitonic_apply(keys, vals)
        assert is_sorted(k)
        assert np.array_equal(v[m:], np.arange(m, n)), "a pad moved"


# ---------------------------------------------------------------- segmented

def test_segmented_matches_per_segment_numpy(oracle_mod):
    off = workloads.segment_offsets(300, 1, 3000, seed=5)
    off = np.concatenate([[0], off[1:], [off[-1]]])  # one empty segment at the end
    keys = workloads.uniform_i32(int(off[-1]), seed=9)
    got = oracle_mod.sort_segmented_i32(keys, off)
    for s in range(off.size - 1):
        b, e = off[s], off[s + 1]
        assert np.array_equal(got[b:e], np.sort(keys[b:e]))


def test_depth_reported(oracle_mod):
    a = workloads.uniform_i32(1 << 16, seed=1)
    _, d0 = oracle_mod.sort_i32_depth(a[:200])
    assert d0 == 0
    _, d = oracle_mod.sort_i32_depth(a)
    assert 8 <= d <= 2 * 16
