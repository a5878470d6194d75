"""The library's own device primitives against numpy (needs a GPU).

The stable LSD radix sorts (u64 keys by their low end_bit bits, u32 keys, with int32
values) must give exactly numpy's stable argsort order of the masked keys, including keys
above end_bit carried unchanged, runs of equal keys in input order, empty and one-key
inputs and ragged last tiles.  The exclusive scans (int32 or int64 in, int64 out) must
equal numpy's cumulative sums shifted by one, also across the scan's recursion levels.
These are the sorts behind duplicate-edge removal and the node order (Methods,
"Remove Multi-Edges", "Node Order") and the prefix sums behind every compaction.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TILE = 4096     # keys per sort tile and elements per scan tile


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_03211_amd as lf
    lf.load_library()
    h = lf.Handle(0)
    yield torch, h
    h.close()


def _keys(rng, n, kind):
    if kind == "full":
        return rng.integers(0, 2 ** 63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
    if kind == "few":          # many equal keys: stability decides the order
        return rng.integers(0, 7, n, dtype=np.uint64) << np.uint64(rng.integers(0, 50))
    if kind == "sorted":
        return np.sort(rng.integers(0, 2 ** 40, n, dtype=np.uint64))
    if kind == "reversed":
        return np.sort(rng.integers(0, 2 ** 40, n, dtype=np.uint64))[::-1].copy()
    raise KeyError(kind)


SIZES = [0, 1, 2, 63, 64, 65, TILE - 1, TILE, TILE + 1, 3 * TILE + 17, 100_003, (1 << 20) + 5]


@pytest.mark.parametrize("end_bit", [64, 62, 44, 13, 8, 7, 1, 0])
def test_sort_pairs_u64_matches_stable_argsort(env, end_bit):
    torch, h = env
    rng = np.random.default_rng(end_bit + 100)
    for n in SIZES:
        for kind in ("full", "few", "sorted", "reversed"):
            say("sort_u64", end_bit, n, kind)
            k = _keys(rng, n, kind)
            v = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
            mask = np.uint64((1 << end_bit) - 1) if end_bit < 64 else np.uint64(~np.uint64(0))
            order = np.argsort(k & mask, kind="stable")
            kd = torch.from_numpy(k.view(np.int64).copy()).cuda()
            vd = torch.from_numpy(v.copy()).cuda()
            h.lf_debug_sort_pairs(kd, vd, end_bit)
            gk = kd.cpu().numpy().view(np.uint64)
            gv = vd.cpu().numpy()
            assert np.array_equal(gk, k[order]), (n, kind)
            assert np.array_equal(gv, v[order]), (n, kind)


def test_sort_keys_only_u64(env):
    torch, h = env
    rng = np.random.default_rng(5)
    for n in (0, 1, 5000, 250_001):
        say("sort_keys", n)
        k = rng.integers(0, 2 ** 44, n, dtype=np.uint64)
        kd = torch.from_numpy(k.view(np.int64).copy()).cuda()
        h.lf_debug_sort_pairs(kd, None, 44)
        assert np.array_equal(kd.cpu().numpy().view(np.uint64), np.sort(k))


def test_sort_pairs_u32_matches_stable_argsort(env):
    torch, h = env
    rng = np.random.default_rng(9)
    for n in SIZES:
        for hi in (2 ** 32, 5, 2 ** 12):
            say("sort_u32", n, hi)
            k = rng.integers(0, hi, n, dtype=np.uint64).astype(np.uint32)
            v = np.arange(n, dtype=np.int32)
            order = np.argsort(k, kind="stable")
            kd = torch.from_numpy(k.view(np.int32).copy()).cuda()
            vd = torch.from_numpy(v.copy()).cuda()
            h.lf_debug_sort_pairs_u32(kd, vd)
            assert np.array_equal(kd.cpu().numpy().view(np.uint32), k[order])
            assert np.array_equal(vd.cpu().numpy(), v[order])


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_exclusive_scan_matches_cumsum(env, dtype):
    torch, h = env
    rng = np.random.default_rng(7)
    # the last two sizes need two and three levels of tile sums
    for n in [0, 1, 2, 255, 256, TILE - 1, TILE, TILE + 1, 1_000_003, TILE * TILE + 9, 17_000_001]:
        say("scan", np.dtype(dtype).name, n)
        if dtype == np.int32:
            x = rng.integers(-1000, 100_000, n).astype(np.int32)
        else:
            x = rng.integers(-2 ** 40, 2 ** 40, n).astype(np.int64)
        want = np.zeros(n, np.int64)
        if n > 1:
            want[1:] = np.cumsum(x.astype(np.int64))[:-1]
        xd = torch.from_numpy(x).cuda()
        od = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
        h.lf_debug_exclusive_scan(xd, od[:n] if n else od[:0])
        assert np.array_equal(od[:n].cpu().numpy(), want)


def test_exclusive_scan_in_place(env):
    torch, h = env
    rng = np.random.default_rng(8)
    x = rng.integers(0, 50, 3 * TILE + 5).astype(np.int64)
    want = np.concatenate([[0], np.cumsum(x)[:-1]])
    xd = torch.from_numpy(x.copy()).cuda()
    say("scan_in_place", x.size)
    h.lf_debug_exclusive_scan(xd, xd)
    assert np.array_equal(xd.cpu().numpy(), want)


def test_primitive_argument_errors(env):
    torch, h = env
    import paper_2210_03211_amd as lf
    kd = torch.zeros(4, dtype=torch.int64, device="cuda")
    with pytest.raises(lf.LazyFoxError):
        h.lf_debug_sort_pairs(kd, None, 65)
    with pytest.raises(lf.LazyFoxError):
        h.lf_debug_sort_pairs(kd, None, -1)
