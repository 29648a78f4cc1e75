"""GPU parity of the packed-column path: device decoding of host-encoded
columns equals the original columns, and the streamed chain query over packed
pinned host columns equals the oracle's result."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Ctx(0, 4 << 30)
    yield c
    c.close()


def columns():
    rng = np.random.default_rng(9)
    n = 1_000_003
    mixed = rng.integers(-2**62, 2**62, n)
    mixed[:200_000] //= 2**50  # blocks of narrow and wide ranges
    mixed[500_000:520_000] = 12345  # constant blocks (0 bits)
    return [
        mixed,
        rng.integers(-2**63, 2**63 - 1, 4097, dtype=np.int64),
        rng.integers(-2**31, 2**31 - 1, 70_001, dtype=np.int64).astype(np.int32),
        (np.arange(300_000) % 2407).astype(np.int32),
        np.array([5], np.int32),
    ]


@pytest.mark.parametrize("i", range(5))
def test_decode_equals_original(gpu, ctx, i):
    import torch
    a = columns()[i]
    blocks, words = gpu.pack(torch.from_numpy(a), pinned=False)
    out = gpu.unpack(ctx, blocks.cuda(), words.cuda(), len(a), torch.from_numpy(a).dtype)
    ctx.check()
    np.testing.assert_array_equal(out.cpu().numpy(), a)


def test_decode_rejects_malformed_blocks(gpu, ctx):
    import torch
    a = np.arange(5000, dtype=np.int64) * 1000
    blocks, words = gpu.pack(torch.from_numpy(a), pinned=False)
    bad = blocks.clone()
    bad[2, 1] += 7  # not a whole number of 32-word steps
    out = gpu.unpack(ctx, bad.cuda(), words.cuda(), len(a), torch.int64)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_INDEX
    got = out.cpu().numpy()
    np.testing.assert_array_equal(got[:1024], a[:1024])  # the blocks before it are decoded
    # words beyond the buffer
    out = gpu.unpack(ctx, blocks.cuda(), words[:10].cuda(), len(a), torch.int64)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_INDEX


@pytest.mark.parametrize("chunk,nbuf", [(1024, 2), (1 << 18, 3), (1 << 20, 2)])
def test_streamed_packed_chain_matches_oracle(gpu, ctx, chunk, nbuf):
    import torch
    na, nb, n = 30_000, 3_000, 2_000_001 if chunk > 1024 else 50_001
    a, b = gen.chain_dims(na, nb)
    f = gen.chain_fact(n, na, nb, 1.0)
    cols = ("a_fk", "b_fk", "date", "price", "discount")
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()}, max_groups=400_000)
    packed = []
    for c in cols:
        t = torch.from_numpy(f[c])
        blocks, words = gpu.pack(t)
        packed.append((blocks, words, n, t.dtype))
    k, s, ng = gpu.query_streamed_packed(ctx, plan, packed, chunk_rows=chunk, nbuf=nbuf)
    ctx.check()
    m = int(ng.item())
    gk, gs = k[:m].cpu().numpy(), s[:m].cpu().numpy()
    o = np.argsort(gk)
    wk, ws = oracle.chain_query(a, b, f)
    np.testing.assert_array_equal(gk[o], wk)
    np.testing.assert_array_equal(gs[o], ws)


def test_streamed_packed_arguments(gpu, ctx):
    import torch
    a, b = gen.chain_dims(1000, 100)
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()}, max_groups=1000)
    f = gen.chain_fact(5000, 1000, 100, 0.0)
    packed = [(*gpu.pack(torch.from_numpy(f[c])), 5000, torch.from_numpy(f[c]).dtype)
              for c in ("a_fk", "b_fk", "date", "price", "discount")]
    with pytest.raises(gpu.PystError) as e:
        gpu.query_streamed_packed(ctx, plan, packed, chunk_rows=1000)  # not a multiple of 1024
    assert e.value.status == gpu.ERR_ARG
    bad = packed[0][0].clone()
    bad[1, 1] = 10**6  # a block of more than 32 bits a value in an int32 column
    packed[0] = (bad, packed[0][1], 5000, torch.int32)
    with pytest.raises(gpu.PystError) as e:
        gpu.query_streamed_packed(ctx, plan, packed, chunk_rows=2048)
    assert e.value.status == gpu.ERR_ARG
