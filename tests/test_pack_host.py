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
