"""GPU parity of the materializing join (build + probe + gather of k payload
columns per side, the join microbenchmark's per-GPU work) and of the gather
primitive under it, element by element against the CPU oracle.  Unique build
keys, so the match order (ascending probe row) is defined and compared as is.
Sizes span several gather tiles (2048 rows) and a ragged tail."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t, n=None):
    a = t.cpu().numpy()
    return a if n is None else a[:n]


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Ctx(0, 4 << 30)
    yield c
    c.close()


def mixed_cols(rng, n, k):
    # alternate int64 and int32 payload columns
    return [rng.integers(-2**62, 2**62, n) if c % 2 == 0 else rng.integers(-2**31, 2**31, n).astype(np.int32)
            for c in range(k)]


@pytest.mark.parametrize("n,m,k,ordered", [(1, 1, 1, True), (5000, 255, 3, False), (5000, 2048, 8, True),
                                           (70_001, 2049, 2, False), (1_000_000, 100_003, 8, False),
                                           (300_000, 300_000, 5, True)])
def test_gather_against_indexing(gpu, ctx, n, m, k, ordered):
    rng = np.random.default_rng(n + m + k)
    cols = mixed_cols(rng, n, k)
    idx = rng.integers(0, n, m).astype(np.int32)
    if ordered:
        idx.sort()
    outs = gpu.gather(ctx, dev(idx), [dev(c) for c in cols])
    ctx.check()
    for o, c in zip(outs, cols):
        np.testing.assert_array_equal(host(o), c[idx])
    # a device count below the capacity: only that prefix is written
    cnt = m // 3
    outs = gpu.gather(ctx, dev(idx), [dev(c) for c in cols], n=dev(np.array([cnt], np.int64)))
    ctx.check()
    for o, c in zip(outs, cols):
        np.testing.assert_array_equal(host(o, cnt), c[idx[:cnt]])


def test_gather_count_above_capacity_and_empty(gpu, ctx):
    rng = np.random.default_rng(5)
    cols = mixed_cols(rng, 1000, 2)
    idx = rng.integers(0, 1000, 4097).astype(np.int32)
    outs = gpu.gather(ctx, dev(idx), [dev(c) for c in cols], n=dev(np.array([10**9], np.int64)))
    ctx.check()
    for o, c in zip(outs, cols):
        np.testing.assert_array_equal(host(o), c[idx])
    outs = gpu.gather(ctx, dev(np.zeros(0, np.int32)), [dev(c) for c in cols])
    ctx.check()
    assert all(o.numel() == 0 for o in outs)


def test_gather_bad_index_and_arguments(gpu, ctx):
    import torch
    c = np.arange(100, dtype=np.int64) * 7
    idx = np.array([3, 100, 5, -1, 99] + [1] * 3000, np.int32)
    dc, di = dev(c), dev(idx)
    out = torch.full((len(idx),), -5, dtype=torch.int64, device="cuda")
    carr = (gpu.Col * 1)(gpu.col(dc))
    oarr = (gpu.ctypes.c_void_p * 1)(out.data_ptr())
    lib = gpu.load()
    st = lib.pyst_gather(ctx.h, gpu.ctypes.c_void_p(di.data_ptr()), None, len(idx), carr, 1, oarr,
                         gpu._stream())
    assert st == gpu.OK
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_INDEX
    got = host(out)
    ok = (idx >= 0) & (idx < 100)
    np.testing.assert_array_equal(got[ok], c[idx[ok]])
    assert np.all(got[~ok] == -5)  # rows with a bad index are left unwritten
    with pytest.raises(gpu.PystError) as e:
        gpu.gather(ctx, dev(idx[:3]), [])
    assert e.value.status == gpu.ERR_ARG
    with pytest.raises(gpu.PystError) as e:
        gpu.gather(ctx, dev(idx[:3]), [dc] * 9)
    assert e.value.status == gpu.ERR_ARG
    with pytest.raises(gpu.PystError) as e:
        gpu.gather(ctx, dev(idx[:3]), [dc, dev(c[:50])])
    assert e.value.status == gpu.ERR_ARG


@pytest.mark.parametrize("nb,npr,k", [(1000, 5000, 1), (20_000, 100_003, 4), (50_000, 400_000, 8),
                                      (3, 4097, 2), (300_000, 2_000_000, 3)])
def test_join_materialize_matches_oracle(gpu, ctx, nb, npr, k):
    b, p = gen.join_tables(nb, npr, k)
    bc = [b["c%d" % c] for c in range(k)]
    pc = [p["c%d" % c] for c in range(k)]
    if k > 1:  # one int32 column per side
        bc[1] = (bc[1] >> 33).astype(np.int32)
        pc[1] = (pc[1] >> 33).astype(np.int32)
    prow, brow, cols, nout = gpu.join_materialize(ctx, dev(b["key"]), [dev(c) for c in bc], dev(p["key"]),
                                                  [dev(c) for c in pc])
    ctx.check()
    wp, wb, wcols = oracle.join_materialize(b["key"], bc, p["key"], pc)
    m = int(host(nout)[0])
    assert m == len(wp)
    np.testing.assert_array_equal(host(prow, m), wp)
    np.testing.assert_array_equal(host(brow, m), wb)
    assert len(cols) == len(wcols) == 2 * k
    for g, w in zip(cols, wcols):
        assert host(g, m).dtype == w.dtype
        np.testing.assert_array_equal(host(g, m), w)


@pytest.mark.parametrize("unique", [True, False])
def test_join_materialize_int64_keys(gpu, ctx, unique):
    # int64 keys (16-byte table slots): keys above 2^32 and a mixed-width probe
    rng = np.random.default_rng(44)
    nb, npr = 40_000, 300_000
    base = np.unique(np.concatenate([rng.integers(-2**62, 2**62, nb, dtype=np.int64),
                                     rng.integers(-2**31 + 1, 2**31, 1000, dtype=np.int64), [-2**31]]))
    bk = base if unique else base[rng.integers(0, len(base), len(base))]
    pk = np.concatenate([bk[rng.integers(0, len(bk), npr // 2)], rng.integers(-2**62, 2**62, npr // 2, dtype=np.int64)])
    pk = pk[rng.permutation(len(pk))]
    bc = [rng.integers(-2**40, 2**40, len(bk), dtype=np.int64)]
    pc = [rng.integers(-2**31, 2**31 - 1, len(pk), dtype=np.int64).astype(np.int32)]
    wp, wb, wcols = oracle.join_materialize(bk, bc, pk, pc)
    prow, brow, cols, nout = gpu.join_materialize(ctx, dev(bk), [dev(c) for c in bc], dev(pk), [dev(c) for c in pc],
                                                  unique_keys=unique, out_cap=len(wp) + 8)
    ctx.check()
    m = int(host(nout)[0])
    assert m == len(wp) and m > npr // 4
    gp, gb = host(prow, m), host(brow, m)
    o = np.lexsort((gb, gp))
    np.testing.assert_array_equal(gp[o], wp)
    np.testing.assert_array_equal(gb[o], wb)
    for g, w in zip(cols, wcols):
        np.testing.assert_array_equal(host(g, m)[o], w)
    # an int32 probe column against the int64 table compares by value
    # (INT32_MIN, an ordinary int64 build key, is the int32 probe column's EMPTY: no match)
    small = bk[(bk > -2**31) & (bk < 2**31)]
    assert len(small) >= 900
    pk32 = np.concatenate([small, [0, 1]]).astype(np.int32)
    wp, wb, _ = oracle.join_materialize(bk, [], pk32, [])  # without the last probe row below
    pk32 = np.append(pk32, np.int32(-2**31))
    prow, brow, _, nout = gpu.join_materialize(ctx, dev(bk), [], dev(pk32), [], unique_keys=unique,
                                               out_cap=len(wp) + 8)
    ctx.check()
    m = int(host(nout)[0])
    assert m == len(wp)
    gp, gb = host(prow, m), host(brow, m)
    o = np.lexsort((gb, gp))
    np.testing.assert_array_equal(gp[o], wp)
    np.testing.assert_array_equal(gb[o], wb)


def test_join_materialize_one_side_and_empty(gpu, ctx):
    b, p = gen.join_tables(4000, 30_000, 2)
    bc, pc = [b["c0"], b["c1"]], [p["c0"], p["c1"]]
    wp, wb, wcols = oracle.join_materialize(b["key"], bc, p["key"], pc)
    # build columns only
    prow, brow, cols, nout = gpu.join_materialize(ctx, dev(b["key"]), [dev(c) for c in bc], dev(p["key"]), [])
    ctx.check()
    m = int(host(nout)[0])
    assert m == len(wp) and len(cols) == 2
    for g, w in zip(cols, wcols[2:]):
        np.testing.assert_array_equal(host(g, m), w)
    # probe columns only, no columns at all
    prow, brow, cols, nout = gpu.join_materialize(ctx, dev(b["key"]), [], dev(p["key"]), [dev(c) for c in pc])
    ctx.check()
    for g, w in zip(cols, wcols[:2]):
        np.testing.assert_array_equal(host(g, m), w)
    prow, brow, cols, nout = gpu.join_materialize(ctx, dev(b["key"]), [], dev(p["key"]), [])
    ctx.check()
    np.testing.assert_array_equal(host(brow, m), wb)
    # an empty build side and an empty probe side
    e32 = np.zeros(0, np.int32)
    prow, brow, cols, nout = gpu.join_materialize(ctx, dev(e32), [dev(np.zeros(0, np.int64))], dev(p["key"]),
                                                  [dev(pc[0])])
    ctx.check()
    assert int(host(nout)[0]) == 0
    prow, brow, cols, nout = gpu.join_materialize(ctx, dev(b["key"]), [dev(bc[0])], dev(e32),
                                                  [dev(np.zeros(0, np.int64))])
    ctx.check()
    assert int(host(nout)[0]) == 0


def test_join_materialize_capacity_and_duplicate_key(gpu, ctx):
    b, p = gen.join_tables(5000, 50_000, 1)
    wp, wb, wcols = oracle.join_materialize(b["key"], [b["c0"]], p["key"], [p["c0"]])
    prow, brow, cols, nout = gpu.join_materialize(ctx, dev(b["key"]), [dev(b["c0"])], dev(p["key"]),
                                                  [dev(p["c0"])], out_cap=1000)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_CAPACITY
    assert int(host(nout)[0]) == len(wp)  # the count holds the need
    np.testing.assert_array_equal(host(prow), wp[:1000])
    for g, w in zip(cols, wcols):
        np.testing.assert_array_equal(host(g), w[:1000])
    key = b["key"].copy()
    key[17] = key[4000]
    gpu.join_materialize(ctx, dev(key), [dev(b["c0"])], dev(p["key"]), [dev(p["c0"])])
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_DUP_KEY
    with pytest.raises(gpu.PystError) as e:
        gpu.join_materialize(ctx, dev(b["key"]), [dev(b["c0"][:10])], dev(p["key"]), [dev(p["c0"])])
    assert e.value.status == gpu.ERR_ARG


def _partitioned_join(gpu, ctx, b, p, k, fanout):
    """Both sides partitioned by key (each carrying its original row ids as a
    last payload column), then every destination joined and materialized; the
    matches mapped back to original rows and put in canonical order."""
    rid_b = dev(np.arange(len(b["key"]), dtype=np.int32))
    rid_p = dev(np.arange(len(p["key"]), dtype=np.int32))
    ob = gpu.partition(ctx, dev(b["key"]), [dev(b["c%d" % c]) for c in range(k)] + [rid_b], fanout)
    op = gpu.partition(ctx, dev(p["key"]), [dev(p["c%d" % c]) for c in range(k)] + [rid_p], fanout)
    offs_b, offs_p = host(ob[2]), host(op[2])
    pr_all, br_all, cols_all = [], [], [[] for _ in range(2 * k)]
    for q in range(fanout):
        b0, b1, p0, p1 = int(offs_b[q]), int(offs_b[q + 1]), int(offs_p[q]), int(offs_p[q + 1])
        prow, brow, cols, nout = gpu.join_materialize(ctx, ob[0][b0:b1], [c[b0:b1] for c in ob[1][:k]],
                                                      op[0][p0:p1], [c[p0:p1] for c in op[1][:k]])
        ctx.check()
        m = int(nout.item())
        pr_all.append(host(op[1][k])[p0:p1][host(prow, m)])
        br_all.append(host(ob[1][k])[b0:b1][host(brow, m)])
        for c in range(2 * k):
            cols_all[c].append(host(cols[c], m))
    pr, br = np.concatenate(pr_all), np.concatenate(br_all)
    o = np.argsort(pr, kind="stable")
    return ob, op, offs_b, offs_p, pr[o], br[o], [np.concatenate(c)[o] for c in cols_all]


@pytest.mark.parametrize("nb,np_,k,fanout", [(50_000, 130_001, 8, 2), (20_000, 70_003, 3, 16), (3_000, 5_000, 1, 1),
                                             (40_000, 90_000, 8, 8)])
def test_partitioned_join_matches_oracle(gpu, ctx, nb, np_, k, fanout):
    # the join microbenchmark's whole per-GPU flow: partition + build + probe + materialize
    b, p = gen.join_tables(nb, np_, k)
    ob, op, offs_b, offs_p, pr, br, cols = _partitioned_join(gpu, ctx, b, p, k, fanout)
    # the send side is the oracle's stable partition, counts included
    for side, tab, got, offs in (("build", b, ob, offs_b), ("probe", p, op, offs_p)):
        rid = np.arange(len(tab["key"]), dtype=np.int32)
        wk, wp, woffs = oracle.partition(tab["key"], [tab["c%d" % c] for c in range(k)] + [rid], fanout)
        np.testing.assert_array_equal(offs, woffs)
        np.testing.assert_array_equal(host(got[0]), wk)
        for c in range(k + 1):
            np.testing.assert_array_equal(host(got[1][c]), wp[c])
    # the receive side's result equals the oracle's join of the unpartitioned tables
    wpr, wbr, wcols = oracle.join_materialize(b["key"], [b["c%d" % c] for c in range(k)], p["key"],
                                              [p["c%d" % c] for c in range(k)])
    np.testing.assert_array_equal(pr, wpr)
    np.testing.assert_array_equal(br, wbr)
    for g, w in zip(cols, wcols):
        np.testing.assert_array_equal(g, w)


def test_partition_carries_fifteen_payload_columns(gpu, ctx):
    # the most payload columns one call carries (a key and k = 8 columns plus row ids fit easily)
    rng = np.random.default_rng(15)
    n = 123_457
    key = rng.integers(1, 50_000, n).astype(np.int32)
    pays = mixed_cols(rng, n, 15)
    ok, op, offs = gpu.partition(ctx, dev(key), [dev(c) for c in pays], 64)
    ctx.check()
    wk, wp, woffs = oracle.partition(key, pays, 64)
    np.testing.assert_array_equal(host(offs), woffs)
    np.testing.assert_array_equal(host(ok), wk)
    for g, w in zip(op, wp):
        np.testing.assert_array_equal(host(g), w)
    with pytest.raises(gpu.PystError) as e:
        gpu.partition(ctx, dev(key), [dev(c) for c in pays] + [dev(key)], 64)
    assert e.value.status == gpu.ERR_ARG


def _canonical(prow, brow, cols, m):
    pr, br = host(prow, m), host(brow, m)
    o = np.lexsort((br, pr))
    return pr[o], br[o], [host(c, m)[o] for c in cols]


@pytest.mark.parametrize("nb,npr,k,nkeys,zs", [(20_000, 50_003, 3, 5_000, 0.0), (30_000, 40_000, 2, 3_000, 1.0),
                                               (4_097, 9_000, 1, 4_097, 0.0), (100_000, 250_000, 4, 25_000, 0.5)])
def test_many_to_many_join_matches_oracle(gpu, ctx, nb, npr, k, nkeys, zs):
    # duplicate build keys: every (probe row, build row) pair with equal keys, element by element
    # against the oracle once both are in canonical (probe row, build row) order
    b, p = gen.join_tables_dup(nb, npr, k, nkeys, zs)
    bc = [dev(b["c%d" % c]) for c in range(k)]
    pc = [dev(p["c%d" % c]) for c in range(k)]
    wpr, wbr, wcols = oracle.join_materialize(b["key"], [b["c%d" % c] for c in range(k)], p["key"],
                                              [p["c%d" % c] for c in range(k)])
    prow, brow, cols, nout = gpu.join_materialize(ctx, dev(b["key"]), bc, dev(p["key"]), pc, unique_keys=False,
                                                  out_cap=len(wpr) + 7)
    ctx.check()
    m = int(nout.item())
    assert m == len(wpr)
    pr = host(prow, m)
    assert (np.diff(pr) >= 0).all()  # ascending probe row, each row's matches together
    gpr, gbr, gcols = _canonical(prow, brow, cols, m)
    np.testing.assert_array_equal(gpr, wpr)
    np.testing.assert_array_equal(gbr, wbr)
    for g, w in zip(gcols, wcols):
        np.testing.assert_array_equal(g, w)


def test_many_to_many_capacity_and_unique_agreement(gpu, ctx):
    b, p = gen.join_tables_dup(10_000, 30_000, 1, 2_500)
    bk, pk = dev(b["key"]), dev(p["key"])
    need = len(oracle.join(b["key"], p["key"])[0])
    # too little room: the count holds the need and the error is latched
    prow, brow, cols, nout = gpu.join_materialize(ctx, bk, [dev(b["c0"])], pk, [dev(p["c0"])], unique_keys=False,
                                                  out_cap=need // 3)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_CAPACITY
    assert int(nout.item()) == need
    # on unique keys the many-to-many path gives the unique-key result
    b, p = gen.join_tables(20_000, 60_000, 2)
    args = (ctx, dev(b["key"]), [dev(b["c0"]), dev(b["c1"])], dev(p["key"]), [dev(p["c0"]), dev(p["c1"])])
    r1 = gpu.join_materialize(*args)
    r2 = gpu.join_materialize(*args, unique_keys=False)
    ctx.check()
    m = int(r1[3].item())
    assert m == int(r2[3].item())
    for x, y in zip([r1[0], r1[1]] + r1[2], [r2[0], r2[1]] + r2[2]):
        np.testing.assert_array_equal(host(x, m), host(y, m))
