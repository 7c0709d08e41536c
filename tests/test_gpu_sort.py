"""The library's stable radix sort of (u32 key, u32 value) pairs (needs an
MI355X), through msgs_debug_sort_pairs, against numpy's stable argsort of the
masked key bits.  Bit-exact: keys and values both.

Sizes cover the single-pass look-back path (fewer than 512 tiles), the
reduce-then-scan path (512 tiles and more, with 2048- and 4096-key tiles),
tile boundaries, ragged tails, heavy key duplication (stability), partial bit
ranges, 511 tiles (the longest look-back chains) and both sides of the switch
between the pass kinds, and device-side counts smaller than the arrays or
larger than them (clamped to the arrays).
"""
import numpy as np
import pytest
import torch

from paper_2311_17089_amd import msgs as M

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0)
    yield c
    torch.cuda.synchronize()


def _ref(keys, begin, end, n):
    k = keys[:n].astype(np.uint64)
    width = end - begin
    masked = (k >> begin) & ((1 << width) - 1)
    perm = np.argsort(masked, kind="stable")
    return keys[:n][perm], perm.astype(np.uint32)


@pytest.mark.parametrize("n,begin,end,distinct", [
    (1, 0, 32, 0),
    (1000, 0, 32, 0),
    (2048, 0, 13, 64),
    (2049, 0, 32, 1000),
    (4097, 8, 24, 0),
    (131_071, 0, 32, 0),                # 64 tiles of 2048: look-back
    (1_046_527, 0, 32, 0),              # 511 tiles: the longest look-back chains
    (1_046_527, 0, 13, 6700),           # 511 tiles, tile-key shape with duplicates
    (1_046_528, 0, 32, 0),              # exactly 511 full tiles
    ((1 << 20) - 1, 0, 32, 0),          # 512 tiles of 2048: reduce-then-scan
    (3_000_001, 0, 13, 6700),           # tile-key shape, many duplicates
    (5_000_003, 0, 32, 0),              # 4096-key tiles
    (5_000_003, 3, 17, 300),
])
def test_sort_matches_stable_argsort(ctx, n, begin, end, distinct):
    _say(f"  sort n={n} bits [{begin},{end}) distinct={distinct}")
    rng = np.random.default_rng(n + begin)
    if distinct:
        keys = rng.integers(0, distinct, size=n, dtype=np.uint64).astype(np.uint32)
        keys = (keys << np.uint32(begin)) | rng.integers(0, 2, size=n).astype(np.uint32)
    else:
        keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int32).copy()).cuda()
    vt = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    M.debug_sort_pairs(ctx, kt, vt, begin, end)
    gk = kt.cpu().numpy().view(np.uint32)
    gv = vt.cpu().numpy().view(np.uint32)
    rk, rv = _ref(keys, begin, end, n)
    np.testing.assert_array_equal(gk, rk)
    np.testing.assert_array_equal(gv, rv)


@pytest.mark.parametrize("nmax,n", [(3_000_000, 2_500_001), (3_000_000, 0), (100_000, 99_999),
                                     (1_040_000, 1_000_001),   # look-back side of the switch
                                     (1_060_000, 1_000_001),   # reduce-then-scan side
                                     (100_000, 150_000),       # count above nmax: clamped
                                     (2_000_000, 4_000_000)])
def test_sort_device_count(ctx, nmax, n):
    _say(f"  sort nmax={nmax} device count {n}")
    rng = np.random.default_rng(nmax + n)
    keys = rng.integers(0, 1 << 32, size=nmax, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(nmax, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int32).copy()).cuda()
    vt = torch.from_numpy(vals.view(np.int32).copy()).cuda()
    dn = torch.tensor([n], dtype=torch.int32, device="cuda")
    M.debug_sort_pairs(ctx, kt, vt, 0, 32, d_n=dn)
    n = min(n, nmax)  # a device count above the arrays sorts all of them
    gk = kt.cpu().numpy().view(np.uint32)[:n]
    gv = vt.cpu().numpy().view(np.uint32)[:n]
    rk, rv = _ref(keys, 0, 32, n)
    np.testing.assert_array_equal(gk, rk)
    np.testing.assert_array_equal(gv, rv)


def test_sort_rejects_bad_arguments(ctx):
    kt = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(M.MsgsError):
        M.debug_sort_pairs(ctx, kt, kt.clone(), 0, 33)
    with pytest.raises(M.MsgsError):
        M.debug_sort_pairs(ctx, kt, kt.clone(), 9, 8)
