"""The bitonic networks on the GPU under the 0-1 principle (Sec. III-A).

A comparator network sorts every input iff it sorts every 0-1 input.  The
GPU's networks (the same-direction network of Alg. 1/2 generalised to
64 * KPL keys per wave, and the packed 16- and 32-lane forms that sort
four or two small arrays per wave) are run on:
* all 2^16 0-1 inputs of 16 keys, through the packed quarter-wave path and
  through the one-array-per-wave path;
* for every network size N and every stage s, inputs whose blocks of 2^s
  keys are two sorted 0-1 halves, with every (zeros in the first half,
  zeros in the second half) combination: the earlier stages leave such
  blocks unchanged (each comparator they apply sees a sorted pair), so
  stage s merges them, and the last stage's inputs are exactly the merger
  inputs of the 0-1 principle; plus 4096 random 0-1 arrays per size.
Word sizes: 4 bytes (int32 keys, batched calls: the one-wave tasks of up to
1024 keys), 8 bytes (float64 keys, batched calls up to 512 keys, and whole
arrays of 1024 keys, one call each) and 16 bytes (float64 key / int32 value
pairs with all values 0, whole arrays of up to 512 pairs, one call each).
The sorted form of a 0-1 array is fixed by its number of zeros; every output
is compared element by element with it, and a sample of the batched inputs
with the oracle's sort.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hs():
    import paper_1704_08579_amd as hsort
    hsort.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return hsort


def exhaustive01(n):
    """All 2^n 0-1 arrays of n keys, one per row (uint8)."""
    i = np.arange(1 << n, dtype=np.int64)[:, None]
    return ((i >> np.arange(n)[None, :]) & 1).astype(np.uint8)


def sorted_halves01(N, s):
    """Arrays of N keys made of blocks of 2^s keys, each two sorted 0-1
    halves; together they hold every (a, b) combination of zeros in the two
    halves (the last array is completed with all-zero blocks)."""
    B = 1 << s
    H = B // 2
    a, b = np.meshgrid(np.arange(H + 1), np.arange(H + 1), indexing="ij")
    a, b = a.ravel(), b.ravel()
    per = N // B
    tot = -(-a.size // per) * per
    a = np.concatenate([a, np.full(tot - a.size, H)])
    b = np.concatenate([b, np.full(tot - b.size, H)])
    j = np.arange(H)[None, :]
    blocks = np.concatenate([(j >= a[:, None]), (j >= b[:, None])], axis=1).astype(np.uint8)
    return blocks.reshape(-1, N)


def all_stage_inputs(N, nrandom=4096):
    """Every stage's sorted-halves inputs, and random 0-1 arrays (each with
    its own density), which also exercise comparators that sorted blocks
    leave idle."""
    rng = np.random.default_rng(N)
    dens = rng.random((nrandom, 1))
    rand = (rng.random((nrandom, N)) < dens).astype(np.uint8)
    return np.concatenate([sorted_halves01(N, s) for s in range(1, N.bit_length())] + [rand], axis=0)


def expected01(rows):
    """Sorted form of each 0-1 row: its zeros, then its ones."""
    zeros = rows.shape[1] - rows.sum(axis=1, dtype=np.int64)
    return (np.arange(rows.shape[1])[None, :] >= zeros[:, None]).astype(np.uint8)


def _check_batched(hs, oracle_mod, rows, dtype, seed):
    """Sort every row as one segment of a batched call; compare."""
    nrow, N = rows.shape
    keys = rows.reshape(-1).astype(dtype)
    off = torch.arange(0, (nrow + 1) * N, N, dtype=torch.int64, device="cuda")
    t = torch.from_numpy(keys).to("cuda")
    hs.sort_segmented_(t, off)
    got = t.cpu().numpy().reshape(nrow, N)
    assert np.array_equal(got, expected01(rows).astype(dtype)), "a 0-1 input came out unsorted"
    rng = np.random.default_rng(seed)
    pick = rng.choice(nrow, size=min(nrow, 512), replace=False)
    sub = rows[pick].reshape(-1).astype(dtype)
    suboff = np.arange(0, (pick.size + 1) * N, N, dtype=np.int64)
    want = oracle_mod.sort_segmented_i32(sub, suboff) if dtype == np.int32 else \
        oracle_mod.sort_segmented_f64(sub, suboff)
    assert np.array_equal(got[pick].reshape(-1).view(np.uint8), want.view(np.uint8))


@pytest.mark.parametrize("dtype", [np.int32, np.float64])
def test_all_01_inputs_of_16_keys(hs, oracle_mod, dtype):
    rows = exhaustive01(16)
    print(f"16-key exhaustive, {np.dtype(dtype).name}, packed path", flush=True)
    _check_batched(hs, oracle_mod, rows, dtype, 1)
    # fewer than four tasks per wave: each wave sorts one array on its own
    print(f"16-key exhaustive, {np.dtype(dtype).name}, one array per wave", flush=True)
    for c in range(0, rows.shape[0], 4096):
        _check_batched(hs, oracle_mod, rows[c:c + 4096], dtype, 2 + c)


@pytest.mark.parametrize("dtype,N", [(np.int32, 32), (np.int32, 64), (np.int32, 128), (np.int32, 256),
                                     (np.int32, 512), (np.int32, 1024),
                                     (np.float64, 32), (np.float64, 64), (np.float64, 128),
                                     (np.float64, 256), (np.float64, 512)])
def test_sorted_halves_batched(hs, oracle_mod, dtype, N):
    rows = all_stage_inputs(N)
    if N == 32:
        rows = np.tile(rows, (-(-40000 // rows.shape[0]), 1))  # enough arrays for the packed half-wave path
    print(f"sorted halves, {np.dtype(dtype).name}, N={N}, {rows.shape[0]} arrays", flush=True)
    _check_batched(hs, oracle_mod, rows, dtype, N)


def _check_whole(hs, rows, kind):
    """One whole-array sort per row (the one-wave path), called through the C
    ABI on consecutive slices of one device buffer; compare."""
    nrow, N = rows.shape
    keys = torch.from_numpy(rows.reshape(-1).astype(np.float64)).to("cuda")
    vals = torch.zeros(nrow * N, dtype=torch.int32, device="cuda") if kind == "kv" else None
    L = hs.lib()
    stream = torch.cuda.current_stream().cuda_stream
    kp = keys.data_ptr()
    for r in range(nrow):
        if vals is None:
            rc = L.hs_sort_f64(kp + 8 * r * N, N, None, None, stream)
        else:
            rc = L.hs_sort_kv_f64(kp + 8 * r * N, vals.data_ptr() + 4 * r * N, N, None, None, stream)
        assert rc == 0, (r, L.hs_last_error())
    got = keys.cpu().numpy().reshape(nrow, N)
    assert np.array_equal(got, expected01(rows).astype(np.float64)), "a 0-1 input came out unsorted"
    if vals is not None:
        assert int(torch.count_nonzero(vals).item()) == 0


def test_sorted_halves_whole_f64_1024(hs):
    """The 1024-key network of 8-byte words runs only for whole arrays."""
    rows = all_stage_inputs(1024)
    print(f"sorted halves, float64 whole arrays, N=1024, {rows.shape[0]} calls", flush=True)
    _check_whole(hs, rows, "keys")


@pytest.mark.parametrize("N", [64, 128, 256, 512])
def test_sorted_halves_whole_kv_f64(hs, N):
    """16-byte words (float64 key, int32 value 0): whole arrays of N pairs."""
    rows = all_stage_inputs(N)
    print(f"sorted halves, float64 key/value whole arrays, N={N}, {rows.shape[0]} calls", flush=True)
    _check_whole(hs, rows, "kv")
