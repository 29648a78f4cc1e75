"""The partition entry point that allocates nothing (pyst_partition_noalloc)
against pyst_partition, through the C ABI: bit-identical outputs and offsets on
two calls in a row, the second smaller, and the size limit of its fixed
scratch refused on the host before any work."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _noalloc(gpu, key, pays, fanout, sel=None, nsel=None):
    import torch
    n = key.numel()
    outs = [torch.full((max(n, 1),), -7, dtype=t.dtype, device="cuda") for t in [key] + pays]
    offs = torch.full((fanout + 1,), -7, dtype=torch.int64, device="cuda")
    gpu.partition_noalloc(key, pays, fanout, outs, offs, sel=sel, nsel=nsel)
    return outs, offs


def test_noalloc_partition_equals_pyst_partition_twice(gpu):
    import torch
    ctx = gpu.Ctx(0, 1 << 30)
    # first call: 5,000,003 rows (ragged last tile), fanout 64, three columns
    _, p = gen.star_tables(150_000, 5_000_003, workload=7)
    key, pays = _dev(p["fk"]), [_dev(p["date"]), _dev(p["price"])]
    outs, offs = _noalloc(gpu, key, pays, 64)
    rk, rp, roffs = gpu.partition(ctx, key, pays, 64)
    torch.cuda.synchronize()
    n = key.numel()
    assert torch.equal(outs[0][:n], rk) and torch.equal(outs[1][:n], rp[0]) and torch.equal(outs[2][:n], rp[1])
    assert torch.equal(offs, roffs) and int(offs[-1]) == n
    # second call, smaller: 777,777 rows of another table, a selection, fanout 8
    _, q = gen.star_tables(20_000, 777_777, workload=8)
    key2, pays2 = _dev(q["fk"]), [_dev(q["price"])]
    sel, nsel = gpu.filter(ctx, [key2, _dev(q["date"])], [(1, "<", 1200)])
    outs2, offs2 = _noalloc(gpu, key2, pays2, 8, sel=sel, nsel=nsel)
    rk2, rp2, roffs2 = gpu.partition(ctx, key2, pays2, 8, sel=sel, nsel=nsel)
    ctx.check()
    m = int(nsel.item())
    assert torch.equal(offs2, roffs2) and int(offs2[-1]) == m
    assert torch.equal(outs2[0][:m], rk2[:m]) and torch.equal(outs2[1][:m], rp2[0][:m])
    # and the oracle's stable partition of the same selected rows
    psel = oracle.filter([q["fk"], q["date"]], [(1, "<", 1200)])
    wk, wp, woffs = oracle.partition(q["fk"], [q["price"]], 8, sel=psel)
    np.testing.assert_array_equal(outs2[0][:m].cpu().numpy(), wk)
    np.testing.assert_array_equal(outs2[1][:m].cpu().numpy(), wp[0])
    np.testing.assert_array_equal(offs2.cpu().numpy(), woffs)
    ctx.close()


def test_noalloc_partition_refuses_sizes_beyond_its_scratch(gpu):
    import torch
    n = 17_000_000  # fanout 1024 needs 8 * ceil(n / 4096) * 1024 bytes > 32 MiB
    key = torch.arange(n, dtype=torch.int32, device="cuda")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    offs = torch.empty(1025, dtype=torch.int64, device="cuda")
    with pytest.raises(gpu.PystError) as e:
        gpu.partition_noalloc(key, [], 1024, [out], offs)
    assert e.value.status == gpu.ERR_CAPACITY and "scratch" in str(e.value)
    # within the limit at the same size with a smaller fanout
    offs64 = torch.empty(65, dtype=torch.int64, device="cuda")
    gpu.partition_noalloc(key, [], 64, [out], offs64)
    torch.cuda.synchronize()
    assert int(offs64[0]) == 0 and int(offs64[64]) == n
    assert bool((offs64[1:] >= offs64[:-1]).all())
