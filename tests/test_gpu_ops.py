"""GPU parity of every operator of the C ABI against the CPU oracle.

Integer work, so the bar is bit-exact.  Outputs whose order the method leaves
open (group-by in table order, duplicate-key matches) are compared after
sorting; everything with a defined order (filter, stable partition, unique-key
probe, sorted group-by) is compared as is.  Sizes span several tiles and a
ragged tail.
"""
import json
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


# ------------------------------------------------------------------ filter

@pytest.mark.parametrize("n", [0, 1, 63, 4095, 4096, 4097, 100_003, 1_500_000])
def test_filter_sizes(gpu, ctx, n):
    b, p = gen.star_tables(max(n // 10, 1), n)
    cols = [p["fk"], p["date"], p["price"]]
    preds = [(1, "<", 1200), (2, ">=", 3_000_000)]
    sel, nsel = gpu.filter(ctx, [dev(c) for c in cols], preds)
    ctx.check()
    want = oracle.filter(cols, preds)
    m = int(host(nsel)[0])
    assert m == len(want)
    np.testing.assert_array_equal(host(sel, m), want)


@pytest.mark.parametrize("preds", [[], [(0, "==", 7)], [(0, "!=", 7), (1, "<=", 5)], [(1, ">", 100)],
                                   [(1, "<", 0)], [(2, "<", 2**40)]])
def test_filter_predicates(gpu, ctx, preds):
    rng = np.random.default_rng(3)
    cols = [rng.integers(0, 20, 70_001).astype(np.int32), rng.integers(0, 200, 70_001).astype(np.int32),
            rng.integers(-2**45, 2**45, 70_001)]
    sel, nsel = gpu.filter(ctx, [dev(c) for c in cols], preds)
    ctx.check()
    want = oracle.filter(cols, preds)
    m = int(host(nsel)[0])
    assert m == len(want)
    np.testing.assert_array_equal(host(sel, m), want)


# ------------------------------------------------------------------ partition

@pytest.mark.parametrize("fanout", [1, 2, 3, 8, 64, 100, 256, 1024])
@pytest.mark.parametrize("n", [5, 4096, 250_001])
def test_partition_matches_oracle(gpu, ctx, fanout, n):
    b, p = gen.star_tables(max(n // 10, 1), n)
    ok, (od, op), off = gpu.partition(ctx, dev(p["fk"]), [dev(p["date"]), dev(p["price"])], fanout)
    ctx.check()
    wk, (wd, wp), woff = oracle.partition(p["fk"], [p["date"], p["price"]], fanout)
    np.testing.assert_array_equal(host(off), woff)
    np.testing.assert_array_equal(host(ok), wk)
    np.testing.assert_array_equal(host(od), wd)
    np.testing.assert_array_equal(host(op), wp)


@pytest.mark.parametrize("fanout", [8, 64])
def test_partition_int64_key_with_selection(gpu, ctx, fanout):
    rng = np.random.default_rng(8)
    n = 300_000
    key = rng.integers(-2**62, 2**62, n)
    pay = np.arange(n, dtype=np.int32)
    sel = np.sort(rng.choice(n, 123_457, replace=False)).astype(np.int32)
    ok, (op,), off = gpu.partition(ctx, dev(key), [dev(pay)], fanout, sel=dev(sel),
                                   nsel=dev(np.array([len(sel)], np.int64)))
    ctx.check()
    wk, (wp,), woff = oracle.partition(key, [pay], fanout, sel=sel)
    np.testing.assert_array_equal(host(off), woff)
    np.testing.assert_array_equal(host(ok, len(sel)), wk)
    np.testing.assert_array_equal(host(op, len(sel)), wp)


# ------------------------------------------------------------------ join

@pytest.mark.parametrize("nb,np_", [(1, 1), (1000, 20_000), (150_000, 1_500_000)])
def test_join_unique_keys_ordered(gpu, ctx, nb, np_):
    b, p = gen.star_tables(nb, np_)
    bsel = oracle.filter([b["key"], b["segment"]], [(1, "==", 1)])
    psel = oracle.filter([p["fk"], p["date"], p["price"]], [(1, "<", 1200)])
    t = gpu.join_build(ctx, dev(b["key"]), None, dev(bsel), dev(np.array([len(bsel)], np.int64)), max_load=0.5)
    rows, pays, nout = gpu.join_probe(ctx, t, dev(p["fk"]), dev(psel), dev(np.array([len(psel)], np.int64)))
    ctx.check()
    wr, wb = oracle.join(b["key"], p["fk"], bsel, psel)
    m = int(host(nout)[0])
    assert m == len(wr)
    np.testing.assert_array_equal(host(rows, m), wr)
    np.testing.assert_array_equal(host(pays, m), wb)
    cap, offered = t.info()
    assert offered == len(bsel) and cap >= 64 and cap & (cap - 1) == 0 and len(bsel) / cap <= 0.5
    t.destroy()


def test_join_duplicate_keys(gpu, ctx):
    rng = np.random.default_rng(12)
    bk = rng.integers(0, 5000, 40_000).astype(np.int32)
    pk = rng.integers(0, 6000, 300_000).astype(np.int32)
    t = gpu.join_build(ctx, dev(bk), None, max_load=0.5, unique_keys=False)
    rows, pays, nout = gpu.join_probe(ctx, t, dev(pk), out_cap=4_000_000)
    ctx.check()
    wr, wb = oracle.join(bk, pk)
    m = int(host(nout)[0])
    assert m == len(wr)
    got = np.stack([host(rows, m), host(pays, m)], 1)
    assert np.all(np.diff(got[:, 0]) >= 0)  # ascending probe row
    got = got[np.lexsort((got[:, 1], got[:, 0]))]
    np.testing.assert_array_equal(got[:, 0], wr)
    np.testing.assert_array_equal(got[:, 1], wb)
    t.destroy()


def test_join_payload_and_capacity_error(gpu, ctx):
    b, p = gen.star_tables(5000, 50_000)
    pay = (b["key"] * 3).astype(np.int32)
    t = gpu.join_build(ctx, dev(b["key"]), dev(pay), max_load=0.7)
    rows, pays, nout = gpu.join_probe(ctx, t, dev(p["fk"]), out_cap=100)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_CAPACITY
    assert int(host(nout)[0]) == 50_000  # every fk matches; the count holds the need
    wr, wb = oracle.join(b["key"], p["fk"])
    np.testing.assert_array_equal(host(rows, 100), wr[:100])
    np.testing.assert_array_equal(host(pays, 100), pay[wb[:100]])
    t.destroy()


@pytest.mark.parametrize("unique", [True, False])
def test_join_probe_sentinel_key_matches_nothing(gpu, ctx, unique):
    # the EMPTY sentinel as a probe key must not match an empty slot
    bk = np.array([5, 6, 7], np.int32)
    pk = np.array([-2**31, 5, -2**31, 7] + [-2**31] * 5000 + [6], np.int32)
    t = gpu.join_build(ctx, dev(bk), unique_keys=unique)
    rows, pays, nout = gpu.join_probe(ctx, t, dev(pk))
    ctx.check()
    wr, wb = oracle.join(bk, pk)
    m = int(host(nout)[0])
    assert m == len(wr) == 3
    np.testing.assert_array_equal(host(rows, m), wr)
    np.testing.assert_array_equal(host(pays, m), wb)
    t.destroy()


def test_join_sentinel_key_and_duplicate_promise(gpu, ctx):
    key = np.array([1, 2, -2**31, 4], np.int32)
    t = gpu.join_build(ctx, dev(key))
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_KEY
    t.destroy()
    t = gpu.join_build(ctx, dev(np.array([5, 6, 5], np.int32)), unique_keys=True)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_DUP_KEY
    t.destroy()
    ctx.check()  # the latch was cleared


@pytest.mark.parametrize("bdt,pdt,paydt,unique", [
    (np.int64, np.int64, None, True),
    (np.int64, np.int64, np.int64, False),
    (np.int32, np.int32, np.int64, True),
    (np.int32, np.int64, None, False),
    (np.int64, np.int32, np.int32, True),
])
def test_join_int64_keys_and_payloads(gpu, ctx, bdt, pdt, paydt, unique):
    # keys spread over the whole int64 (or int32) range; the probe also holds
    # keys no build row has, keys outside int32 range and each column's EMPTY
    rng = np.random.default_rng(31)
    lo, hi = (np.iinfo(bdt).min + 1, np.iinfo(bdt).max)
    n_keys = 30_000
    pool = np.unique(np.concatenate([rng.integers(lo, hi, n_keys, dtype=np.int64, endpoint=True),
                                     rng.integers(-2**31 + 1, 2**31 - 1, n_keys, dtype=np.int64, endpoint=True)]))
    if unique:
        bk = rng.permutation(pool).astype(bdt)
    else:
        bk = pool[rng.integers(0, len(pool), 2 * len(pool))].astype(bdt)
    plo, phi = np.iinfo(pdt).min + 1, np.iinfo(pdt).max
    hits = bk.astype(np.int64)[rng.integers(0, len(bk), 150_000)]
    hits = hits[(hits >= plo) & (hits <= phi)]
    miss = rng.integers(plo, phi, 50_000, dtype=np.int64, endpoint=True)
    pk = np.concatenate([hits, miss, [np.iinfo(pdt).min] * 7]).astype(pdt)
    pk = pk[rng.permutation(len(pk))]
    pay = None
    if paydt is not None:
        pay = rng.integers(np.iinfo(paydt).min, np.iinfo(paydt).max, len(bk), dtype=np.int64, endpoint=True).astype(paydt)
    t = gpu.join_build(ctx, dev(bk), dev(pay) if pay is not None else None, max_load=0.5, unique_keys=unique)
    wr, wb = oracle.join(bk, pk)
    rows, pays, nout = gpu.join_probe(ctx, t, dev(pk), out_cap=len(wr) + 16)
    ctx.check()
    m = int(host(nout)[0])
    assert m == len(wr) and m > 50_000
    got_r, got_p = host(rows, m), host(pays, m)
    assert np.all(np.diff(got_r) >= 0)  # ascending probe row
    want_p = (pay.astype(np.int64) if pay is not None else np.arange(len(bk), dtype=np.int64))[wb]
    o = np.lexsort((got_p, got_r))
    w = np.lexsort((want_p, wr))
    np.testing.assert_array_equal(got_r[o], wr[w])
    np.testing.assert_array_equal(got_p[o], want_p[w])
    t.destroy()


def test_join_int64_sentinel_and_duplicate_promise(gpu, ctx):
    e64 = np.iinfo(np.int64).min
    t = gpu.join_build(ctx, dev(np.array([1, e64, 3], np.int64)))
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_KEY
    t.destroy()
    t = gpu.join_build(ctx, dev(np.array([2**40, 7, 2**40], np.int64)), unique_keys=True)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_DUP_KEY
    t.destroy()
    # INT32_MIN is an ordinary key in an int64 column; in an int32 probe column
    # it is that column's EMPTY and matches nothing
    t = gpu.join_build(ctx, dev(np.array([-2**31, 5], np.int64)))
    rows, pays, nout = gpu.join_probe(ctx, t, dev(np.array([-2**31, 5, 6], np.int64)))
    ctx.check()
    assert int(host(nout)[0]) == 2
    np.testing.assert_array_equal(host(rows, 2), [0, 1])
    np.testing.assert_array_equal(host(pays, 2), [0, 1])
    rows, pays, nout = gpu.join_probe(ctx, t, dev(np.array([-2**31, 5], np.int32)))
    ctx.check()
    assert int(host(nout)[0]) == 1
    assert host(rows, 1)[0] == 1 and host(pays, 1)[0] == 1
    t.destroy()


# ------------------------------------------------------------------ group-by

@pytest.mark.parametrize("n,nkeys", [(1, 1), (10_000, 10), (500_000, 200_000), (2_000_000, 1_000_000)])
def test_groupby_matches_oracle(gpu, ctx, n, nkeys):
    rng = np.random.default_rng(n)
    k = rng.integers(0, nkeys, n).astype(np.int32)
    v = rng.integers(-10**12, 10**12, n)
    gk, gs, ng = gpu.groupby_sum(ctx, dev(k), dev(v))
    ctx.check()
    wk, ws = oracle.groupby_sum(k, v)
    m = int(host(ng)[0])
    assert m == len(wk)
    a, s = host(gk, m), host(gs, m)
    o = np.argsort(a)
    np.testing.assert_array_equal(a[o], wk)
    np.testing.assert_array_equal(s[o], ws)


def test_groupby_sorted_int64_keys_with_selection(gpu, ctx):
    rng = np.random.default_rng(21)
    n = 400_000
    k = rng.integers(-2**50, 2**50, n) // 1000 * 1000 % (2**40)
    k[::7] = -k[::7]
    v = rng.integers(0, 100, n).astype(np.int32)
    sel = np.sort(rng.choice(n, 250_000, replace=False)).astype(np.int32)
    gk, gs, ng = gpu.groupby_sum(ctx, dev(k), dev(v), sel=dev(sel), nsel=dev(np.array([len(sel)], np.int64)),
                                 sort_by_key=True)
    ctx.check()
    wk, ws = oracle.groupby_sum(k, v, sel)
    m = int(host(ng)[0])
    assert m == len(wk)
    np.testing.assert_array_equal(host(gk, m), wk)
    np.testing.assert_array_equal(host(gs, m), ws)


def test_groupby_wraps_and_capacity(gpu, ctx):
    big = 2**63 - 1
    k = np.array([3, 3, 3, 9], np.int64)
    v = np.array([big, big, 5, 1], np.int64)
    gk, gs, ng = gpu.groupby_sum(ctx, dev(k), dev(v), sort_by_key=True)
    ctx.check()
    wk, ws = oracle.groupby_sum(k, v)
    np.testing.assert_array_equal(host(gk, 2), wk)
    np.testing.assert_array_equal(host(gs, 2), ws)
    k = np.arange(1000, dtype=np.int32)
    gk, gs, ng = gpu.groupby_sum(ctx, dev(k), dev(k), max_groups=10)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status in (gpu.ERR_CAPACITY, gpu.ERR_TABLE_FULL)


# ------------------------------------------------------------------ fused queries

def _sorted_pair(keys, sums, m):
    a, s = host(keys, m), host(sums, m)
    o = np.argsort(a)
    return a[o], s[o]


def test_star_query_golden(gpu, ctx):
    g = json.load(open(os.path.join(GOLDEN, "star_tiny.json")))
    b = {k: dev(np.array(v, np.int32)) for k, v in g["build"].items()}
    fact = [dev(np.array(g["probe"]["fk"], np.int32)), dev(np.array(g["probe"]["date"], np.int32)),
            dev(np.array(g["probe"]["price"], np.int64))]
    k, s, ng = gpu.query(ctx, gpu.star_plan(b), fact)
    ctx.check()
    m = int(host(ng)[0])
    a, ss = _sorted_pair(k, s, m)
    assert a.tolist() == g["expect"]["keys"] and ss.tolist() == g["expect"]["sums"]


@pytest.mark.parametrize("nb,np_", [(1, 7), (1000, 9_999), (150_000, 1_500_000)])
@pytest.mark.parametrize("max_load", [0.5, 0.7])
def test_star_query_matches_oracle(gpu, ctx, nb, np_, max_load):
    b, p = gen.star_tables(nb, np_)
    bd = {"key": dev(b["key"]), "segment": dev(b["segment"])}
    k, s, ng = gpu.query(ctx, gpu.star_plan(bd, max_load=max_load), [dev(p["fk"]), dev(p["date"]), dev(p["price"])])
    ctx.check()
    wk, ws = oracle.star_query(b, p)
    m = int(host(ng)[0])
    assert m == len(wk)
    a, ss = _sorted_pair(k, s, m)
    np.testing.assert_array_equal(a, wk)
    np.testing.assert_array_equal(ss, ws)


def test_chain_query_golden(gpu, ctx):
    g = json.load(open(os.path.join(GOLDEN, "chain_tiny.json")))
    a = {k: dev(np.array(v, np.int32)) for k, v in g["A"].items()}
    b = {k: dev(np.array(v, np.int32)) for k, v in g["B"].items()}
    f = g["fact"]
    fact = [dev(np.array(f[c], np.int64 if c == "price" else np.int32))
            for c in ("a_fk", "b_fk", "date", "price", "discount")]
    k, s, ng = gpu.query(ctx, gpu.chain_plan(a, b), fact)
    ctx.check()
    m = int(host(ng)[0])
    kk, ss = _sorted_pair(k, s, m)
    assert kk.tolist() == g["expect"]["keys"] and ss.tolist() == g["expect"]["sums"]


@pytest.mark.parametrize("zs", [0.0, 1.0])
@pytest.mark.parametrize("max_groups", [0, 400_000])
def test_chain_query_matches_oracle(gpu, ctx, zs, max_groups):
    na, nb, nf = 30_000, 3_000, 1_200_001
    a, b = gen.chain_dims(na, nb)
    f = gen.chain_fact(nf, na, nb, zs)
    ad = {k: dev(v) for k, v in a.items()}
    bd = {k: dev(v) for k, v in b.items()}
    fact = [dev(f[c]) for c in ("a_fk", "b_fk", "date", "price", "discount")]
    k, s, ng = gpu.query(ctx, gpu.chain_plan(ad, bd, max_groups=max_groups), fact)
    ctx.check()
    wk, ws = oracle.chain_query(a, b, f)
    m = int(host(ng)[0])
    assert m == len(wk)
    kk, ss = _sorted_pair(k, s, m)
    np.testing.assert_array_equal(kk, wk)
    np.testing.assert_array_equal(ss, ws)


def test_query_is_deterministic(gpu, ctx):
    # Group order follows table slots, which depend on insertion races; the set
    # of (key, sum) pairs must not.
    b, p = gen.star_tables(20_000, 400_000)
    bd = {"key": dev(b["key"]), "segment": dev(b["segment"])}
    fact = [dev(p["fk"]), dev(p["date"]), dev(p["price"])]
    r1 = gpu.query(ctx, gpu.star_plan(bd), fact)
    r2 = gpu.query(ctx, gpu.star_plan(bd), fact)
    ctx.check()
    m = int(host(r1[2])[0])
    assert m == int(host(r2[2])[0])
    k1, s1 = _sorted_pair(r1[0], r1[1], m)
    k2, s2 = _sorted_pair(r2[0], r2[1], m)
    np.testing.assert_array_equal(k1, k2)
    np.testing.assert_array_equal(s1, s2)
