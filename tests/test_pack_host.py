"""The host encoder of packed columns against the documented format, decoded
bit by bit with plain numpy (no GPU: the encoder is host code)."""
import numpy as np
import pytest


def np_decode(blocks, words, n):
    # value j of block b: bits [j*bits, (j+1)*bits) of the block's little-endian 32-bit words
    w = words.view(np.uint32)
    out = []
    for b in range(len(blocks) - 1):
        base, off = int(blocks[b, 0]), int(blocks[b, 1])
        bits = (int(blocks[b + 1, 1]) - off) // 32
        assert bits * 32 == int(blocks[b + 1, 1]) - off
        for j in range(min(1024, n - b * 1024)):
            x = 0
            for t in range(bits):
                q, r = divmod(j * bits + t, 32)
                x |= ((int(w[off + q]) >> r) & 1) << t
            out.append(((base + x + 2**63) % 2**64) - 2**63)
    return np.array(out, dtype=np.int64)


@pytest.fixture(scope="module")
def lib():
    from paper_2512_02862_amd import pyst
    pyst.load()
    return pyst


CASES = {
    "constant": lambda rng: np.full(3000, 7, np.int64),
    "full_int64": lambda rng: rng.integers(-2**63, 2**63 - 1, 2500, dtype=np.int64),
    "full_int32": lambda rng: rng.integers(-2**31, 2**31 - 1, 2049, dtype=np.int64).astype(np.int32),
    "ramp_int32": lambda rng: np.arange(1025, dtype=np.int32) * 3 - 100,
    "40_bits": lambda rng: rng.integers(0, 2**40, 1024, dtype=np.int64),
    "extremes": lambda rng: np.array([-2**63, 2**63 - 1], np.int64),
    "empty": lambda rng: np.zeros(0, np.int32),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_pack_encode_round_trips(lib, case):
    import torch
    a = CASES[case](np.random.default_rng(len(case)))
    blocks, words = lib.pack(torch.from_numpy(a), pinned=False)
    nblk = (len(a) + 1023) // 1024
    assert blocks.shape == (nblk + 1, 2) and int(blocks[0, 1]) == 0 and int(blocks[-1, 1]) == words.numel()
    np.testing.assert_array_equal(np_decode(blocks.numpy(), words.numpy(), len(a)), a.astype(np.int64))
    # each block uses the fewest bits that hold its range
    for b in range(nblk):
        blk = a[b * 1024:(b + 1) * 1024].astype(np.int64)
        rng_ = int(blk.max()) - int(blk.min())
        assert (int(blocks[b + 1, 1]) - int(blocks[b, 1])) // 32 == rng_.bit_length()
        assert int(blocks[b, 0]) == int(blk.min())


def test_pack_rejects_bad_columns(lib):
    import torch
    with pytest.raises(ValueError):
        lib.pack(torch.zeros(4, dtype=torch.float32))


def test_pack_encode_large_column_across_host_threads(lib):
    # 20M values: the encoder splits the blocks over several host threads; the
    # block widths vary so every word offset depends on all earlier blocks.
    import torch
    rng = np.random.default_rng(99)
    n = 20_000_003
    width = rng.integers(0, 41, (n + 1023) // 1024)
    a = (rng.integers(0, 2**40, n, dtype=np.int64) % (np.int64(1) << np.repeat(width, 1024)[:n])) - 12345
    blocks, words = lib.pack(torch.from_numpy(a), pinned=False)
    bl, w = blocks.numpy(), words.numpy()
    nblk = (n + 1023) // 1024
    assert int(bl[0, 1]) == 0 and int(bl[-1, 1]) == w.size
    steps = np.diff(bl[:, 1])
    assert (steps % 32 == 0).all()
    # every block's width and base are those of its values
    blk_min = np.minimum.reduceat(a, np.arange(0, n, 1024))
    blk_max = np.maximum.reduceat(a, np.arange(0, n, 1024))
    bits = np.array([int(r).bit_length() for r in (blk_max - blk_min)])
    np.testing.assert_array_equal(steps // 32, bits)
    np.testing.assert_array_equal(bl[:-1, 0], blk_min)
    # bit-by-bit decode of the blocks at every possible thread boundary and a random sample
    pick = set([0, 1, nblk - 2, nblk - 1])
    for t in range(1, 65):
        for c in (nblk * t // 64, nblk * t // 8, nblk * t // 5, nblk * t // 3):
            pick.update(x for x in (c - 1, c, c + 1) if 0 <= x < nblk)
    pick.update(int(x) for x in rng.integers(0, nblk, 20))
    for b in sorted(pick):
        sub_blocks = bl[b:b + 2].copy()
        base_off = int(sub_blocks[0, 1])
        sub_blocks[:, 1] -= base_off
        m = min(1024, n - b * 1024)
        got = np_decode(sub_blocks, w[base_off:int(bl[b + 1, 1])], m)
        np.testing.assert_array_equal(got, a[b * 1024:b * 1024 + m])
