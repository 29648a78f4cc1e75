"""GPU parity of the streamed query: chunked pinned-host input must give exactly
the unchunked result (integer sums are order independent) and the oracle's."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pinned(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory()


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Ctx(0, 4 << 30)
    yield c
    c.close()


def sorted_out(k, s, ng):
    m = int(ng.item())
    k, s = k[:m].cpu().numpy(), s[:m].cpu().numpy()
    o = np.argsort(k)
    return k[o], s[o]


@pytest.mark.parametrize("chunk,nbuf", [(4, 2), (100_000, 2), (262_144, 3), (1 << 22, 2)])
def test_streamed_star(gpu, ctx, chunk, nbuf):
    n = 1_000_003 if chunk > 4 else 4001
    b, p = gen.star_tables(50_000, n)
    bd = {k: dev(v) for k, v in b.items()}
    host = [pinned(p[c]) for c in ("fk", "date", "price")]
    k, s, ng = gpu.query_streamed(ctx, gpu.star_plan(bd), host, chunk_rows=chunk, nbuf=nbuf)
    ctx.check()
    got = sorted_out(k, s, ng)
    wk, ws = oracle.star_query(b, p)
    np.testing.assert_array_equal(got[0], wk)
    np.testing.assert_array_equal(got[1], ws)


@pytest.mark.parametrize("zs", [0.0, 1.0])
def test_streamed_chain_equals_resident(gpu, ctx, zs):
    na, nb, n = 30_000, 3_000, 2_000_001
    a, b = gen.chain_dims(na, nb)
    f = gen.chain_fact(n, na, nb, zs)
    cols = ("a_fk", "b_fk", "date", "price", "discount")
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()}, max_groups=400_000)
    k, s, ng = gpu.query_streamed(ctx, plan, [pinned(f[c]) for c in cols], chunk_rows=300_000, nbuf=2)
    ctx.check()
    got = sorted_out(k, s, ng)
    r = gpu.query(ctx, plan, [dev(f[c]) for c in cols])
    ctx.check()
    res = sorted_out(*r)
    wk, ws = oracle.chain_query(a, b, f)
    np.testing.assert_array_equal(got[0], wk)
    np.testing.assert_array_equal(got[1], ws)
    np.testing.assert_array_equal(res[0], wk)
    np.testing.assert_array_equal(res[1], ws)


def test_streamed_rejects_pageable_and_bad_chunks(gpu, ctx):
    import torch
    b, p = gen.star_tables(1000, 10_000)
    bd = {k: dev(v) for k, v in b.items()}
    with pytest.raises(ValueError):
        gpu.query_streamed(ctx, gpu.star_plan(bd), [torch.from_numpy(p[c]) for c in ("fk", "date", "price")],
                           chunk_rows=1024)
    host = [pinned(p[c]) for c in ("fk", "date", "price")]
    with pytest.raises(gpu.PystError):
        gpu.query_streamed(ctx, gpu.star_plan(bd), host, chunk_rows=1001)
    with pytest.raises(gpu.PystError):
        gpu.query_streamed(ctx, gpu.star_plan(bd), host, chunk_rows=1024, nbuf=1)
