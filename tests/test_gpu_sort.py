"""The library's stable radix sort (the depth order and the (tile, depth, id)
order of the tile lists, Sec. 3.3) through the C ABI, against NumPy's stable
argsort of the same key bits: bit-exact keys and values at sizes from empty
to the full-size workloads' list lengths, with ragged last tiles, heavy
duplication, float depth keys and partial bit ranges."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_19202_amd as nvgs
    ctx = nvgs.Context(0)
    yield nvgs, torch, ctx
    ctx.close()


def _keys(kind, n, rng):
    if kind == "uniform":
        return rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    if kind == "few":  # seven distinct keys: long runs of equal digits
        return rng.integers(0, 7, n).astype(np.uint32) * np.uint32(0x01010101)
    if kind == "depth":  # bit patterns of positive FP32 depths over three decades
        return (10.0 ** rng.uniform(-1.0, 2.0, n)).astype(np.float32).view(np.uint32)
    if kind == "equal":
        return np.full(n, 0xdeadbeef, np.uint32)
    if kind == "descending":
        return np.sort(rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32))[::-1].copy()
    raise ValueError(kind)


def _check(env, keys, begin, end, seed):
    nvgs, torch, ctx = env
    n = len(keys)
    vals = np.random.default_rng(seed + 1).permutation(n).astype(np.uint32)  # distinct: checks the value moves
    kd = torch.from_numpy(keys.view(np.int32).copy()).to("cuda")
    vd = torch.from_numpy(vals.view(np.int32).copy()).to("cuda")
    ctx.sort_pairs(kd, vd, begin, end)
    gk = kd.cpu().numpy().view(np.uint32)
    gv = vd.cpu().numpy().view(np.uint32)
    width = end - begin
    mask = np.uint64((1 << width) - 1)
    digit = (keys.astype(np.uint64) >> np.uint64(begin)) & mask
    order = np.argsort(digit, kind="stable")
    assert np.array_equal(gk, keys[order]), "keys differ from the stable order"
    assert np.array_equal(gv, vals[order]), "values differ from the stable order"


SIZES = [1, 5, 2047, 2048, 2049, 3 * 2048 + 17, 100_003, (1 << 20) + 12_345]


@pytest.mark.parametrize("kind", ["uniform", "few", "depth", "equal", "descending"])
@pytest.mark.parametrize("n", SIZES)
def test_sort_pairs_matches_stable_argsort(env, kind, n):
    log(f"[sort] kind={kind} n={n}")
    rng = np.random.default_rng(n * 31 + len(kind))
    _check(env, _keys(kind, n, rng), 0, 32, n)


@pytest.mark.parametrize("begin,end", [(0, 5), (0, 15), (3, 19), (8, 16), (24, 32), (0, 1)])
def test_sort_pairs_bit_ranges(env, begin, end):
    log(f"[sort] bits [{begin}, {end})")
    rng = np.random.default_rng(begin * 100 + end)
    _check(env, _keys("uniform", 300_001, rng), begin, end, begin + end)


@pytest.mark.parametrize("n,kind,bits", [(6_400_000, "depth", 32), (14_100_000, "few", 15)])
def test_sort_pairs_full_size(env, n, kind, bits):
    """The composed 1080p frame's list lengths: ~6.4M splats by depth, ~14.1M
    (tile, splat) entries by a 15-bit tile key."""
    log(f"[sort] full size n={n} kind={kind} bits={bits}")
    rng = np.random.default_rng(n)
    keys = _keys(kind, n, rng)
    if bits < 32:
        keys = (keys ^ rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)) & np.uint32((1 << bits) - 1)
    _check(env, keys, 0, bits, n)


@pytest.mark.parametrize("n,kind,bits", [((24 << 20) - 1, "depth", 32), ((24 << 20) + 4097, "depth", 32),
                                         ((24 << 20) + 4097, "few", 18)])
def test_sort_pairs_block_size_switch(env, n, kind, bits):
    """From 24Mi keys on the sort uses 4,096-key blocks instead of 2,048:
    just below and just above the switch, with a ragged last block."""
    log(f"[sort] block switch n={n} kind={kind} bits={bits}")
    rng = np.random.default_rng(n + bits)
    keys = _keys(kind, n, rng)
    if bits < 32:
        keys = (keys ^ rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)) & np.uint32((1 << bits) - 1)
    _check(env, keys, 0, bits, n)


def test_sort_pairs_empty_and_invalid(env):
    nvgs, torch, ctx = env
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    ctx.sort_pairs(e, e, 0, 32)  # nothing to do
    k = torch.zeros(4, dtype=torch.int32, device="cuda")
    v = torch.arange(4, dtype=torch.int32, device="cuda")
    ctx.sort_pairs(k, v, 7, 7)  # empty bit range: unchanged
    assert v.cpu().tolist() == [0, 1, 2, 3]
    for b, en in [(-1, 8), (0, 33), (9, 8)]:
        with pytest.raises(nvgs.NvgsError):
            ctx.sort_pairs(k, v, b, en)
    assert ctx.L.nvgs_sort_pairs(ctx.h, None, None, 4, 0, 32) == nvgs.E_INVALID


def test_sort_pairs_repeated_calls_reuse_the_workspace(env):
    """A smaller sort after a larger one: stale histogram words of the larger
    one's blocks must not leak into the smaller one."""
    rng = np.random.default_rng(5)
    for n in (500_000, 70_000, 2049, 500_000):
        _check(env, _keys("uniform", n, rng), 0, 32, n)
