"""Pins for the CPU oracle: it is checked against things other than itself.

* the hash finalizers against published MurmurHash3 values (fmix32 by the
  x86_32 empty-key vectors, fmix64 by the x64_128 SMHasher verification value)
  and against their algebraic inverses (built from the constants' modular
  inverses);
* every operator against brute force on small inputs and against numpy
  library routines that compute the same result another way;
* invariants (counts sum to n, join cardinality = sum_k b(k) p(k), sums of
  groups = sum of joined values, wrap-around modulo 2^64);
* hand-computed worked examples in tests/golden/.
"""
import json
import os

import numpy as np
import pytest

import gen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M32 = 0xFFFFFFFF
M64 = 0xFFFFFFFFFFFFFFFF


# ------------------------------------------------------------------ fmix32 / fmix64

def _unxorshift(y, s, bits):
    x, k = y, 1
    while k * s < bits:
        x ^= y >> (k * s)
        k += 1
    return x


def _inv_fmix32(h):
    h = _unxorshift(h, 16, 32)
    h = (h * pow(0xC2B2AE35, -1, 2**32)) & M32
    h = _unxorshift(h, 13, 32)
    h = (h * pow(0x85EBCA6B, -1, 2**32)) & M32
    return _unxorshift(h, 16, 32)


def _inv_fmix64(h):
    h = _unxorshift(h, 33, 64)
    h = (h * pow(0xC4CEB9FE1A85EC53, -1, 2**64)) & M64
    h = _unxorshift(h, 33, 64)
    h = (h * pow(0xFF51AFD7ED558CCD, -1, 2**64)) & M64
    return _unxorshift(h, 33, 64)


def test_fmix32_published_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "murmur3_empty_key.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for seed_hex, hash_hex in rows:
        assert oracle.fmix32(int(seed_hex, 16)) == int(hash_hex, 16)


def test_fmix32_is_inverted_by_its_algebraic_inverse():
    rng = np.random.default_rng(1)
    for x in [0, 1, 2, 0x7FFFFFFF, 0x80000000, M32] + list(rng.integers(0, 2**32, 500)):
        x = int(x)
        assert _inv_fmix32(oracle.fmix32(x)) == x


def test_fmix64_is_inverted_by_its_algebraic_inverse():
    rng = np.random.default_rng(2)
    assert oracle.fmix64(0) == 0
    for x in [1, M64, 2**63] + [int(v) for v in rng.integers(0, 2**63, 300)]:
        assert _inv_fmix64(oracle.fmix64(x)) == x


def _mm3_x64_128(data, seed, fmix):
    """MurmurHash3_x64_128 (Appleby, public domain) written out from its
    published definition, with the 64-bit finalizer passed in."""
    c1, c2 = 0x87C37B91114253D5, 0x4CF5AD432745937F

    def rotl(x, r):
        return ((x << r) | (x >> (64 - r))) & M64

    def mix_k1(k):
        return (rotl((k * c1) & M64, 31) * c2) & M64

    def mix_k2(k):
        return (rotl((k * c2) & M64, 33) * c1) & M64

    n = len(data)
    h1 = h2 = seed & M32
    for i in range(n // 16):
        k1 = int.from_bytes(data[16 * i:16 * i + 8], "little")
        k2 = int.from_bytes(data[16 * i + 8:16 * i + 16], "little")
        h1 ^= mix_k1(k1)
        h1 = (((rotl(h1, 27) + h2) & M64) * 5 + 0x52DCE729) & M64
        h2 ^= mix_k2(k2)
        h2 = (((rotl(h2, 31) + h1) & M64) * 5 + 0x38495AB5) & M64
    tail = data[16 * (n // 16):]
    if len(tail) > 8:
        h2 ^= mix_k2(int.from_bytes(tail[8:], "little"))
    if len(tail) > 0:
        h1 ^= mix_k1(int.from_bytes(tail[:8], "little"))
    h1 ^= n
    h2 ^= n
    h1 = (h1 + h2) & M64
    h2 = (h2 + h1) & M64
    h1, h2 = fmix(h1), fmix(h2)
    h1 = (h1 + h2) & M64
    h2 = (h2 + h1) & M64
    return h1.to_bytes(8, "little") + h2.to_bytes(8, "little")


def test_fmix64_reproduces_the_published_murmur3_x64_128_verification_value():
    # The oracle's fmix64 is the finalizer of MurmurHash3_x64_128; with it the
    # whole hash must reproduce SMHasher's published verification value.
    rows = [l.split() for l in open(os.path.join(GOLDEN, "murmur3_x64_128_verification.txt"))
            if l.strip() and not l.startswith("#")]
    expected = int(rows[0][0], 16)
    key = bytes(range(256))
    hashes = b"".join(_mm3_x64_128(key[:i], 256 - i, oracle.fmix64) for i in range(256))
    final = _mm3_x64_128(hashes, 0, oracle.fmix64)
    assert int.from_bytes(final[:4], "little") == expected
    # a finalizer with one constant changed does not reproduce it
    def bad(k):
        return oracle.fmix64(k) ^ 1 if k else 0
    final_bad = _mm3_x64_128(b"".join(_mm3_x64_128(key[:i], 256 - i, bad) for i in range(256)), 0, bad)
    assert int.from_bytes(final_bad[:4], "little") != expected


# ------------------------------------------------------------------ filter

def _brute_filter(cols, preds):
    ops = {"==": lambda a, b: a == b, "!=": lambda a, b: a != b, "<": lambda a, b: a < b,
           "<=": lambda a, b: a <= b, ">": lambda a, b: a > b, ">=": lambda a, b: a >= b}
    n = len(cols[0])
    return [i for i in range(n) if all(ops[o](int(cols[c][i]), v) for c, o, v in preds)]


@pytest.mark.parametrize("seed", range(6))
def test_filter_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 400))
    cols = [rng.integers(-5, 5, n).astype(np.int32), rng.integers(-2**40, 2**40, n),
            rng.integers(0, 3, n).astype(np.int32)]
    ops = ["==", "!=", "<", "<=", ">", ">="]
    preds = [(int(rng.integers(0, 3)), ops[int(rng.integers(0, 6))], int(rng.integers(-3, 3)))
             for _ in range(int(rng.integers(0, 4)))]
    got = oracle.filter(cols, preds)
    assert got.dtype == np.int32
    assert list(got) == _brute_filter(cols, preds)


def test_filter_matches_numpy_mask_and_edge_cases():
    b, p = gen.star_tables(5000, 50000)
    sel = oracle.filter([p["fk"], p["date"], p["price"]], [(1, "<", 1200)])
    np.testing.assert_array_equal(sel, np.nonzero(p["date"] < 1200)[0])
    assert len(oracle.filter([p["date"]], [(0, ">=", 0)])) == 50000          # all pass
    assert len(oracle.filter([p["date"]], [(0, "<", 0)])) == 0               # none pass
    assert len(oracle.filter([p["date"]], [])) == 50000                      # no predicate
    assert len(oracle.filter([np.zeros(0, np.int32)], [(0, "==", 0)])) == 0  # empty
    # int64 constant outside the int32 range compares without clipping
    assert len(oracle.filter([p["date"]], [(0, "<", 2**40)])) == 50000


# ------------------------------------------------------------------ partition

def _np_fmix32(x):
    h = x.astype(np.uint32)
    h ^= h >> np.uint32(16)
    h *= np.uint32(0x85EBCA6B)
    h ^= h >> np.uint32(13)
    h *= np.uint32(0xC2B2AE35)
    h ^= h >> np.uint32(16)
    return h


@pytest.mark.parametrize("fanout", [1, 2, 3, 8, 64, 256])
def test_partition_invariants(fanout):
    b, p = gen.star_tables(3000, 20000)
    fk, date, price = p["fk"], p["date"], p["price"]
    rowid = np.arange(len(fk), dtype=np.int32)
    ok, (od, op, orow), off = oracle.partition(fk, [date, price, rowid], fanout)
    assert off[0] == 0 and off[-1] == len(fk)                         # counts sum to n
    assert np.all(np.diff(off) >= 0)
    for d in range(fanout):
        seg = slice(off[d], off[d + 1])
        assert all(oracle.fmix32(int(k)) % fanout == d for k in ok[seg][:50])
        assert np.all(np.diff(orow[seg]) > 0)                          # stable
    np.testing.assert_array_equal(fk[orow], ok)                        # a permutation of rows
    np.testing.assert_array_equal(date[orow], od)
    np.testing.assert_array_equal(price[orow], op)
    dest = (_np_fmix32(fk) % np.uint32(fanout)).astype(np.int64)
    order = np.argsort(dest, kind="stable")                            # library counting sort
    np.testing.assert_array_equal(orow, order)
    np.testing.assert_array_equal(np.diff(off), np.bincount(dest, minlength=fanout))
    if fanout == 1:
        np.testing.assert_array_equal(ok, fk)


def test_partition_with_selection_and_int64_key():
    rng = np.random.default_rng(5)
    key = rng.integers(-2**62, 2**62, 3000)
    sel = np.sort(rng.choice(3000, 1000, replace=False)).astype(np.int32)
    ok, (orow,), off = oracle.partition(key, [np.arange(3000, dtype=np.int32)], 16, sel=sel)
    assert off[-1] == 1000
    assert set(orow.tolist()) == set(sel.tolist())
    for d in range(16):
        for k in ok[off[d]:off[d + 1]][:20]:
            assert (oracle.fmix64(int(k)) & M32) % 16 == d
    empty = oracle.partition(np.zeros(0, np.int32), [], 8)
    assert list(empty[2]) == [0] * 9


# ------------------------------------------------------------------ join

def _brute_join(bk, pk, bsel=None, psel=None):
    bs = range(len(bk)) if bsel is None else bsel
    ps = range(len(pk)) if psel is None else psel
    return [(int(i), int(j)) for i in ps for j in bs if bk[j] == pk[i]]


@pytest.mark.parametrize("seed", range(6))
def test_join_brute_force_with_duplicates(seed):
    rng = np.random.default_rng(100 + seed)
    nb, npr = int(rng.integers(0, 300)), int(rng.integers(0, 600))
    bk = rng.integers(0, 40, nb).astype(np.int32)
    pk = rng.integers(0, 50, npr).astype(np.int32)
    bsel = np.sort(rng.choice(nb, nb // 2, replace=False)).astype(np.int32) if nb else None
    psel = np.sort(rng.choice(npr, npr // 3, replace=False)).astype(np.int32) if npr else None
    pr, br = oracle.join(bk, pk, bsel, psel)
    assert list(zip(pr.tolist(), br.tolist())) == _brute_join(bk, pk, bsel, psel)


def test_join_cardinality_and_searchsorted():
    rng = np.random.default_rng(7)
    bk = rng.integers(0, 5000, 20000).astype(np.int32)
    pk = rng.integers(0, 6000, 50000).astype(np.int32)
    pr, br = oracle.join(bk, pk)
    ub, cb = np.unique(bk, return_counts=True)
    up, cp = np.unique(pk, return_counts=True)
    common, ib, ip = np.intersect1d(ub, up, return_indices=True)
    assert len(pr) == int(np.sum(cb[ib].astype(np.int64) * cp[ip]))
    np.testing.assert_array_equal(bk[br], pk[pr])
    # unique build keys: the join is a sorted-array lookup
    b, p = gen.star_tables(4000, 30000)
    pr, br = oracle.join(b["key"], p["fk"])
    order = np.argsort(b["key"])
    pos = np.searchsorted(b["key"][order], p["fk"])
    hit = (pos < 4000) & (b["key"][order][np.minimum(pos, 3999)] == p["fk"])
    np.testing.assert_array_equal(pr, np.nonzero(hit)[0])
    np.testing.assert_array_equal(br, order[pos[hit]])
    # empty build side
    assert len(oracle.join(np.zeros(0, np.int32), pk)[0]) == 0


@pytest.mark.parametrize("seed", range(4))
def test_join_materialize_brute_force(seed):
    # every output tuple is (probe columns at p, build columns at b) for each
    # matching pair in ascending (p, b) order, written out with plain loops
    rng = np.random.default_rng(300 + seed)
    nb, npr, k = int(rng.integers(0, 200)), int(rng.integers(0, 400)), int(rng.integers(1, 9))
    bk = rng.integers(0, 60, nb).astype(np.int32)
    pk = rng.integers(0, 80, npr).astype(np.int32)
    bc = [rng.integers(-2**62, 2**62, nb) if c % 2 else rng.integers(-2**31, 2**31, nb).astype(np.int32)
          for c in range(k)]
    pc = [rng.integers(-2**62, 2**62, npr) for _ in range(k)]
    pr, br, cols = oracle.join_materialize(bk, bc, pk, pc)
    want = [(i, j) for i in range(npr) for j in range(nb) if bk[j] == pk[i]]
    assert list(zip(pr.tolist(), br.tolist())) == want
    assert len(cols) == 2 * k
    for t, (i, j) in enumerate(want):
        assert [int(c[t]) for c in cols] == [int(c[i]) for c in pc] + [int(c[j]) for c in bc]
    for c, src in zip(cols, pc + bc):
        assert c.dtype == src.dtype


def test_q18_recipe():
    li = gen.q18_lineitem(400_000, 100_000)
    assert li["orderkey"].min() >= 1 and li["orderkey"].max() <= 100_000
    assert li["quantity"].min() == 1 and li["quantity"].max() == 50
    k, s = oracle.groupby_sum(li["orderkey"], li["quantity"])
    # keys drawn 4 times each on average: 1 - e^-4 of them occur
    assert abs(len(k) / 100_000 - (1 - np.exp(-4.0))) < 0.01
    assert int(s.sum()) == int(li["quantity"].astype(np.int64).sum())


def test_join_tables_recipe():
    nb, npr, k = 20000, 400000, 3
    b, p = gen.join_tables(nb, npr, k)
    assert sorted(b["key"].tolist()) == list(range(1, nb + 1))
    assert p["key"].min() >= 1 and p["key"].max() <= 2 * nb
    assert abs(np.mean(p["key"] <= nb) - 0.5) < 0.005  # hit ratio 0.5
    for c in range(k):
        for t in (b, p):
            assert t["c%d" % c].dtype == np.int64
            assert np.abs(t["c%d" % c]).max() <= 2**62
    assert not np.array_equal(b["c0"], b["c1"]) and not np.array_equal(p["c0"][:nb], b["c0"])
    pr, br, cols = oracle.join_materialize(b["key"], [b["c0"]], p["key"], [p["c0"]])
    assert len(pr) == int(np.sum(p["key"] <= nb))


# ------------------------------------------------------------------ group-by

@pytest.mark.parametrize("seed", range(5))
def test_groupby_brute_force(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(0, 500))
    k = rng.integers(-20, 20, n).astype(np.int32)
    v = rng.integers(-10**6, 10**6, n)
    sel = np.sort(rng.choice(n, n // 2, replace=False)).astype(np.int32) if n else None
    gk, gs = oracle.groupby_sum(k, v, sel)
    ref = {}
    for i in (range(n) if sel is None else sel):
        ref[int(k[i])] = ref.get(int(k[i]), 0) + int(v[i])
    assert gk.tolist() == sorted(ref)
    assert gs.tolist() == [ref[x] for x in sorted(ref)]


def test_groupby_matches_add_at_and_invariants():
    rng = np.random.default_rng(9)
    k = rng.integers(0, 3000, 100000)
    v = rng.integers(90000, 10500000, 100000)
    gk, gs = oracle.groupby_sum(k, v)
    acc = np.zeros(3000, dtype=np.int64)
    np.add.at(acc, k, v)
    present = np.bincount(k, minlength=3000) > 0
    np.testing.assert_array_equal(gk, np.nonzero(present)[0])
    np.testing.assert_array_equal(gs, acc[present])
    assert int(gs.sum()) == int(v.sum())
    # all distinct keys -> sums are the values; one key -> one total
    gk, gs = oracle.groupby_sum(np.arange(50, dtype=np.int32)[::-1].copy(), np.arange(50))
    np.testing.assert_array_equal(gs, np.arange(50)[::-1])
    gk, gs = oracle.groupby_sum(np.full(10, 4, np.int32), np.arange(10))
    assert gk.tolist() == [4] and gs.tolist() == [45]


def test_groupby_wraps_modulo_2_64():
    big = 2**63 - 1
    gk, gs = oracle.groupby_sum(np.array([1, 1, 1], np.int64), np.array([big, big, 5], np.int64))
    want = (3 * 0 + big + big + 5) % 2**64
    want = want - 2**64 if want >= 2**63 else want
    assert gs.tolist() == [want]


# ------------------------------------------------------------------ composed queries

def _brute_star(build, probe, seg=1, date_lt=1200):
    seg_of = {int(k): int(s) for k, s in zip(build["key"], build["segment"])}
    out = {}
    for f, d, pr in zip(probe["fk"], probe["date"], probe["price"]):
        if d < date_lt and seg_of.get(int(f)) == seg:
            out[int(f)] = out.get(int(f), 0) + int(pr)
    return sorted(out), [out[k] for k in sorted(out)]


def test_star_query_golden():
    g = json.load(open(os.path.join(GOLDEN, "star_tiny.json")))
    b = {k: np.array(v, np.int32) for k, v in g["build"].items()}
    p = {"fk": np.array(g["probe"]["fk"], np.int32), "date": np.array(g["probe"]["date"], np.int32),
         "price": np.array(g["probe"]["price"], np.int64)}
    k, s = oracle.star_query(b, p)
    assert k.tolist() == g["expect"]["keys"] and s.tolist() == g["expect"]["sums"]


@pytest.mark.parametrize("nb,np_", [(200, 3000), (1500, 15000), (1, 10)])
def test_star_query_brute_force_and_composition(nb, np_):
    b, p = gen.star_tables(nb, np_)
    k, s = oracle.star_query(b, p)
    bk, bs = _brute_star(b, p)
    assert k.tolist() == bk and s.tolist() == bs
    # composition of the separate operators gives the same answer
    bsel = oracle.filter([b["key"], b["segment"]], [(1, "==", 1)])
    psel = oracle.filter([p["fk"], p["date"], p["price"]], [(1, "<", 1200)])
    pr, br = oracle.join(b["key"], p["fk"], bsel, psel)
    ck, cs = oracle.groupby_sum(b["key"][br], p["price"][pr])
    np.testing.assert_array_equal(ck, k)
    np.testing.assert_array_equal(cs, s)


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
def test_threaded_baseline_equals_the_oracle(threads):
    # The threaded CPU baseline runs the oracle's algorithm over row ranges;
    # its result must be the oracle's for any thread count, including ranges
    # with no rows, duplicate build keys and wrap-around sums.
    b, p = gen.star_tables(3000, 40000)
    k, s = oracle.star_query(b, p)
    tk, ts, used = oracle.star_query_threaded(b, p, threads=threads)
    assert used == threads
    np.testing.assert_array_equal(tk, k)
    np.testing.assert_array_equal(ts, s)
    tiny_b, tiny_p = gen.star_tables(1, 2)
    np.testing.assert_array_equal(oracle.star_query_threaded(tiny_b, tiny_p, threads=threads)[1],
                                  oracle.star_query(tiny_b, tiny_p)[1])
    rng = np.random.default_rng(threads)
    db = {"key": rng.integers(1, 50, 300).astype(np.int32), "segment": rng.integers(0, 2, 300).astype(np.int32)}
    dp = {"fk": rng.integers(1, 60, 5000).astype(np.int32), "date": rng.integers(0, 2400, 5000).astype(np.int32),
          "price": rng.integers(2**61, 2**62, 5000)}
    preds = (("segment", "==", 1),)
    k, s = oracle.star_query(db, dp, build_preds=preds)
    tk, ts, _ = oracle.star_query_threaded(db, dp, build_preds=preds, threads=threads)
    np.testing.assert_array_equal(tk, k)
    np.testing.assert_array_equal(ts, s)


def _brute_chain(a, b, f, vconst=100):
    out = {}
    for i in range(len(f["a_fk"])):
        if not f["date"][i] < 1200:
            continue
        for jb in range(len(b["key"])):
            if b["key"][jb] != f["b_fk"][i] or b["segment"][jb] != 1:
                continue
            for ja in range(len(a["key"])):
                if a["key"][ja] != f["a_fk"][i]:
                    continue
                g = (int(b["key"][jb]) << 32) | (int(a["date"][ja]) & M32)
                out[g] = out.get(g, 0) + int(f["price"][i]) * (vconst - int(f["discount"][i]))
    return sorted(out), [out[k] for k in sorted(out)]


def test_chain_query_golden():
    g = json.load(open(os.path.join(GOLDEN, "chain_tiny.json")))
    a = {k: np.array(v, np.int32) for k, v in g["A"].items()}
    b = {k: np.array(v, np.int32) for k, v in g["B"].items()}
    f = {k: np.array(v, np.int64 if k == "price" else np.int32) for k, v in g["fact"].items()}
    k, s = oracle.chain_query(a, b, f)
    assert k.tolist() == g["expect"]["keys"] and s.tolist() == g["expect"]["sums"]
    assert (k.tolist(), s.tolist()) == _brute_chain(a, b, f)


@pytest.mark.parametrize("zs", [0.0, 1.0])
def test_chain_query_brute_force(zs):
    a, b = gen.chain_dims(60, 30)
    f = gen.chain_fact(600, 60, 30, zs)
    k, s = oracle.chain_query(a, b, f)
    assert (k.tolist(), s.tolist()) == _brute_chain(a, b, f)


def test_chain_query_duplicate_dimension_keys():
    rng = np.random.default_rng(11)
    a = {"key": rng.integers(1, 8, 20).astype(np.int32), "date": rng.integers(0, 5, 20).astype(np.int32)}
    b = {"key": rng.integers(1, 6, 15).astype(np.int32), "segment": rng.integers(0, 2, 15).astype(np.int32)}
    f = {"a_fk": rng.integers(1, 9, 200).astype(np.int32), "b_fk": rng.integers(1, 7, 200).astype(np.int32),
         "date": rng.integers(1100, 1300, 200).astype(np.int32), "price": rng.integers(1, 100, 200),
         "discount": rng.integers(0, 11, 200).astype(np.int32)}
    k, s = oracle.chain_query(a, b, f)
    assert (k.tolist(), s.tolist()) == _brute_chain(a, b, f)


# ------------------------------------------------------------------ generator sanity

def test_generator_ranges_and_chunk_consistency():
    b, p = gen.star_tables(10000, 200000)
    assert sorted(b["key"].tolist()) == list(range(1, 10001))
    assert b["segment"].min() == 0 and b["segment"].max() == 4
    assert p["fk"].min() >= 1 and p["fk"].max() <= 10000
    assert p["date"].min() == 0 and p["date"].max() == 2406
    assert p["price"].min() >= 90000 and p["price"].max() <= 10500000
    chunk = gen.star_probe(5000, 10000, offset=123456)
    for c in ("fk", "date", "price"):
        np.testing.assert_array_equal(chunk[c], p[c][123456:128456])
    f = gen.chain_fact(200000, 3000, 3000, 1.0)
    # Zipf s=1: P(rank 1) = 1 / H_3000
    h = sum(1.0 / r for r in range(1, 3001))
    assert abs(np.mean(f["b_fk"] == 1) - 1.0 / h) < 0.005
    sizes, builds = gen.fragment_sizes(512)
    assert sizes.min() >= 10000 and sizes.max() <= 20_000_000
    np.testing.assert_array_equal(builds, sizes // 10)
