"""GPU parity of pyst_query on both of its fact-pass implementations (the
plan-shape-specialized kernel and the generic one) and on plan variants that
route predicates, values and group keys differently.  Expected values come from
the oracle's operators composed in plan order."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

FACT_STAR = ("fk", "date", "price")
FACT_CHAIN = ("a_fk", "b_fk", "date", "price", "discount")


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ctx(gpu):
    c = gpu.Ctx(0, 4 << 30)
    yield c
    c.close()


def run(gpu, ctx, plan, fact, path, out_cap=None):
    # "fast": the specialized kernel, which direct-addresses a dimension table
    # whose selected keys span a small enough range; "fast_hash": the same
    # kernel with hash tables only; "generic": the generic fact pass
    ctx.generic_only(path == "generic")
    ctx.hash_join_only(path == "fast_hash")
    try:
        k, s, ng = gpu.query(ctx, plan, fact, out_cap=out_cap)
        ctx.check()
    finally:
        ctx.generic_only(False)
        ctx.hash_join_only(False)
    m = int(ng.item())
    k, s = k[:m].cpu().numpy(), s[:m].cpu().numpy()
    o = np.argsort(k, kind="stable")
    return k[o], s[o]


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
@pytest.mark.parametrize("nb,np_", [(2, 3), (30_000, 300_001), (150_000, 1_500_000)])
def test_star_both_paths(gpu, ctx, path, nb, np_):
    b, p = gen.star_tables(nb, np_)
    bd = {k: dev(v) for k, v in b.items()}
    k, s = run(gpu, ctx, gpu.star_plan(bd), [dev(p[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(b, p)
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
def test_star_predicate_on_join_column_and_no_predicate(gpu, ctx, path):
    b, p = gen.star_tables(20_000, 400_000)
    bd = {k: dev(v) for k, v in b.items()}
    fact = [dev(p[c]) for c in FACT_STAR]
    plan = gpu.star_plan(bd)
    plan.preds = [(1, "<", 1200), (0, "!=", 17)]
    k, s = run(gpu, ctx, plan, fact, path)
    wk, ws = oracle.star_query(b, p, probe_preds=(("date", "<", 1200), ("fk", "!=", 17)))
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)
    plan.preds = []
    k, s = run(gpu, ctx, plan, fact, path)
    wk, ws = oracle.star_query(b, p, probe_preds=())
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
def test_star_int32_value_column(gpu, ctx, path):
    b, p = gen.star_tables(10_000, 200_003)
    bd = {k: dev(v) for k, v in b.items()}
    plan = gpu.star_plan(bd)
    plan.value = ("col", 1)  # SUM(date)
    k, s = run(gpu, ctx, plan, [dev(p[c]) for c in FACT_STAR], path)
    bsel = oracle.filter([b["key"], b["segment"]], [(1, "==", 1)])
    psel = oracle.filter([p["fk"], p["date"], p["price"]], [(1, "<", 1200)])
    pr, br = oracle.join(b["key"], p["fk"], bsel, psel)
    wk, ws = oracle.groupby_sum(b["key"][br], p["date"][pr])
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
def test_star_every_comparison_at_its_boundaries(gpu, ctx, path):
    # date is U[0, 2406]; constants at, inside and outside the int32 range
    b, p = gen.star_tables(5_000, 60_001)
    bd = {k: dev(v) for k, v in b.items()}
    fact = [dev(p[c]) for c in FACT_STAR]
    plan = gpu.star_plan(bd)
    consts = [-(2 ** 40), -(2 ** 31) - 1, -(2 ** 31), -1, 0, 1200, 2406, 2407, 2 ** 31 - 1, 2 ** 31, 2 ** 40]
    for op in ("==", "!=", "<", "<=", ">", ">="):
        for c in consts:
            plan.preds = [(1, op, c)]
            k, s = run(gpu, ctx, plan, fact, path)
            wk, ws = oracle.star_query(b, p, probe_preds=(("date", op, c),))
            np.testing.assert_array_equal(k, wk, err_msg="%s %d" % (op, c))
            np.testing.assert_array_equal(s, ws, err_msg="%s %d" % (op, c))


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
@pytest.mark.parametrize("np_", [1, 4, 255, 256, 257, 258, 259, 4095, 4097, 262_143, 262_145])
def test_star_ragged_fact_lengths(gpu, ctx, path, np_):
    # wave steps of 256 rows, 4 rows per lane: every remainder of the last step
    b, p = gen.star_tables(3_000, np_)
    bd = {k: dev(v) for k, v in b.items()}
    k, s = run(gpu, ctx, gpu.star_plan(bd), [dev(p[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(b, p)
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
def test_star_every_row_matches(gpu, ctx, path):
    # no predicate on either side: every fact row joins, so the fast path's LDS
    # staging overflows every step and the excess is added directly
    b, p = gen.star_tables(100_000, 3_000_001)
    bd = {k: dev(v) for k, v in b.items()}
    plan = gpu.star_plan(bd)
    plan.joins[0]["preds"] = []
    plan.preds = []
    k, s = run(gpu, ctx, plan, [dev(p[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(b, p, build_preds=(), probe_preds=())
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
def test_star_groups_whose_sum_is_zero(gpu, ctx, path):
    # each fact row is followed by a copy with the negated price: every group
    # that exists sums to 0 and must still be reported
    b, p = gen.star_tables(20_000, 200_000)
    q = {"fk": np.repeat(p["fk"], 2), "date": np.repeat(p["date"], 2),
         "price": np.stack([p["price"], -p["price"]], axis=1).ravel()}
    bd = {k: dev(v) for k, v in b.items()}
    k, s = run(gpu, ctx, gpu.star_plan(bd), [dev(q[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(b, q)
    assert len(wk) > 1000 and not ws.any()
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
def test_star_values_of_every_width(gpu, ctx, path):
    # values shifted left by 0..62 bits (wrapping): the fast path stages the
    # ones that fit in 43 bits and adds the others directly; sums wrap mod 2^64
    b, p = gen.star_tables(20_000, 400_003)
    shift = (np.arange(len(p["price"])) % 63).astype(np.uint64)
    q = dict(p)
    q["price"] = (p["price"].astype(np.uint64) << shift).view(np.int64)
    bd = {k: dev(v) for k, v in b.items()}
    k, s = run(gpu, ctx, gpu.star_plan(bd), [dev(q[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(b, q)
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
@pytest.mark.parametrize("nb", [600_000, 2_200_000])
def test_star_tables_too_large_to_stage(gpu, ctx, path, nb):
    # no dimension predicate: 600k keys make a 2^21-slot table (sized on the
    # device, too many buckets to stage: the pairs are added directly), 2.2M
    # keys a 2^23-slot one (the host does not set up bucketed sums at all)
    b, p = gen.star_tables(nb, 2_000_003)
    bd = {k: dev(v) for k, v in b.items()}
    plan = gpu.star_plan(bd)
    plan.joins[0]["preds"] = []
    k, s = run(gpu, ctx, plan, [dev(p[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(b, p, build_preds=())
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
@pytest.mark.parametrize("preds", [True, False])
def test_star_nearly_full_table(gpu, ctx, path, preds):
    # the join table at load ~0.92: many probes run past their first 16-byte
    # group (carried into the next step, carried again, walked at once when the
    # lane already carries one, or walked after the last step); without
    # predicates every row is live, so every wave step has more than 64 live
    # rows and the staging area fills within a step
    nb = 150_000 if preds else 240_000  # 30k or 240k keys in a 32k- or 256k-slot table
    b, p = gen.star_tables(nb, 2_000_003)
    bd = {k: dev(v) for k, v in b.items()}
    plan = gpu.star_plan(bd, max_load=0.95)
    if not preds:
        plan.joins[0]["preds"] = []
        plan.preds = []
    k, s = run(gpu, ctx, plan, [dev(p[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(b, p) if preds else oracle.star_query(b, p, build_preds=(), probe_preds=())
    assert len(wk) > 0
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


def _dense_star(rng_keys, n_keys, base, n_fact, seed=0, select_ends=True):
    """A star build side whose keys are n_keys distinct values of [base, base + rng_keys)
    (both ends included and, with select_ends, selected by segment == 1), and a fact
    table whose fk also falls just outside that range."""
    r = np.random.default_rng(seed)
    inner = r.choice(np.arange(1, rng_keys - 1, dtype=np.int64), n_keys - 2, replace=False)
    keys = np.concatenate([[0, rng_keys - 1], inner]) + base
    seg = r.integers(0, 5, len(keys)).astype(np.int32)
    if select_ends:
        seg[:2] = 1
    o = r.permutation(len(keys))
    b = {"key": keys[o].astype(np.int32), "segment": seg[o]}
    near = np.clip(base + r.integers(-20, rng_keys + 20, 64), -2 ** 31 + 1, 2 ** 31 - 1)
    fk = np.concatenate([keys[r.integers(0, len(keys), n_fact - 64)], near]).astype(np.int32)
    p = {"fk": fk[r.permutation(n_fact)], "date": r.integers(0, 2407, n_fact).astype(np.int32),
         "price": r.integers(90_000, 10_500_001, n_fact).astype(np.int64)}
    return b, p


@pytest.mark.parametrize("path", ["fast", "fast_hash"])
@pytest.mark.parametrize("rng_keys,base", [
    (1 << 20, 0),                    # exact LDS filter, the largest such range
    ((1 << 20) + 1, -(2 ** 31) + 5),  # paired filter bits, the bitmap read from the L2
    (1 << 21, 2 ** 31 - (1 << 21)),  # the largest direct range, ending at INT32_MAX
    ((1 << 21) + 1, 1000),           # one past it: hash table
    (3_000, 7),                      # a small range
])
def test_star_direct_addressing_ranges(gpu, ctx, path, rng_keys, base):
    b, p = _dense_star(rng_keys, min(rng_keys, 400_000), base, 1_500_001)
    bd = {k: dev(v) for k, v in b.items()}
    plan = gpu.star_plan(bd, max_load=0.2)  # reserves >= 2^21 slots for 400k keys
    k, s = run(gpu, ctx, plan, [dev(p[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(b, p)
    assert len(wk) > 1000 or rng_keys < 10_000
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash"])
def test_star_sparse_and_single_keys(gpu, ctx, path):
    # keys spread over the whole int32 range (a hash table either way), then a
    # dimension whose filter keeps a single key (a range of one)
    b, p = gen.star_tables(50_000, 500_003)
    sb, sp = dict(b), dict(p)
    sb["key"] = (b["key"].astype(np.int64) * 40_503 - 2 ** 31 + 1).astype(np.int32)
    sp["fk"] = (p["fk"].astype(np.int64) * 40_503 - 2 ** 31 + 1).astype(np.int32)
    k, s = run(gpu, ctx, gpu.star_plan({k_: dev(v) for k_, v in sb.items()}), [dev(sp[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(sb, sp)
    assert len(wk) > 1000
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)
    one = dict(b)
    one["segment"] = np.where(b["key"] == 777, 1, 0).astype(np.int32)
    k, s = run(gpu, ctx, gpu.star_plan({k_: dev(v) for k_, v in one.items()}), [dev(p[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(one, p)
    assert len(wk) == 1
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash"])
def test_star_duplicate_and_sentinel_dimension_keys(gpu, ctx, path):
    # keys 1..20000 shifted down to just above INT32_MIN, so that the reserved
    # key INT32_MIN still leaves a range small enough for direct addressing
    b, p = gen.star_tables(20_000, 100_000)
    shift = -2 ** 31
    for bad, status in [(5, gpu.ERR_DUP_KEY), (0, gpu.ERR_KEY)]:
        d = dict(b)
        d["key"] = (b["key"].astype(np.int64) + shift).astype(np.int32)
        d["segment"] = b["segment"].copy()
        i = int(np.flatnonzero(b["key"] == 11)[0])
        d["key"][i] = bad + shift  # a second key 5, or INT32_MIN, both selected
        d["segment"][i] = 1
        d["segment"][np.flatnonzero(b["key"] == 5)[0]] = 1
        fact = [dev((p["fk"].astype(np.int64) + shift).astype(np.int32)), dev(p["date"]), dev(p["price"])]
        ctx.hash_join_only(path == "fast_hash")
        try:
            gpu.query(ctx, gpu.star_plan({k_: dev(v) for k_, v in d.items()}), fact)
            with pytest.raises(gpu.PystError) as e:
                ctx.check()
        finally:
            ctx.hash_join_only(False)
        assert e.value.status == status


def _chain(n=1_000_003, na=40_000, nb=4_000, zs=0.0):
    a, b = gen.chain_dims(na, nb)
    f = gen.chain_fact(n, na, nb, zs)
    return a, b, f


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
@pytest.mark.parametrize("zs", [0.0, 1.0])
@pytest.mark.parametrize("max_groups", [0, 300_000])
def test_chain_both_paths(gpu, ctx, path, zs, max_groups):
    a, b, f = _chain(zs=zs)
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()},
                          max_groups=max_groups)
    k, s = run(gpu, ctx, plan, [dev(f[c]) for c in FACT_CHAIN], path)
    wk, ws = oracle.chain_query(a, b, f)
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
@pytest.mark.parametrize("preds", [True, False])
def test_chain_nearly_full_tables(gpu, ctx, path, preds):
    # both join tables near load 0.92 (B keys-only, A key + payload, two slots
    # per 16-byte group): runs past the first group in both probes, read for all
    # lanes of a wave together; without predicates every row is live, so a
    # wave step has several windows of 64 live rows
    nb = 18_840 if preds else 3_768  # 3768 selected B keys in a 4096-slot table
    a, b, f = _chain(n=1_000_003, na=30_000, nb=nb)
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()}, max_load=0.95)
    if not preds:
        plan.joins[0]["preds"] = []
        plan.preds = []
    k, s = run(gpu, ctx, plan, [dev(f[c]) for c in FACT_CHAIN], path)
    wk, ws = oracle.chain_query(a, b, f) if preds else oracle.chain_query(a, b, f, b_preds=(), fact_preds=())
    assert len(wk) > 0
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
def test_chain_group_by_two_join_keys(gpu, ctx, path):
    # GROUP BY (A.key, B.key): join 1 needs no payload (keys-only table)
    a, b, f = _chain(n=500_001)
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()})
    plan.hi, plan.lo = ("join_key", 1), ("join_key", 0)
    k, s = run(gpu, ctx, plan, [dev(f[c]) for c in FACT_CHAIN], path)
    bsel = oracle.filter([b["key"], b["segment"]], [(1, "==", 1)])
    fsel = oracle.filter([f[c] for c in FACT_CHAIN], [(2, "<", 1200)])
    fr, _ = oracle.join(b["key"], f["b_fk"], bsel, fsel)
    fr2, _ = oracle.join(a["key"], f["a_fk"], None, fr)
    gkey = (f["a_fk"][fr2].astype(np.int64) << 32) | f["b_fk"][fr2].astype(np.int64)
    val = f["price"][fr2] * (100 - f["discount"][fr2].astype(np.int64))
    wk, ws = oracle.groupby_sum(gkey, val)
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
@pytest.mark.parametrize("n", [1, 5, 4097])
def test_chain_small_and_empty(gpu, ctx, path, n):
    # a handful of fact rows (few or no pairs reach the group-by), and a
    # predicate no row passes (no pairs at all)
    a, b, f = _chain(n=n, na=1_000, nb=100)
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()})
    fact = [dev(f[c]) for c in FACT_CHAIN]
    k, s = run(gpu, ctx, plan, fact, path)
    wk, ws = oracle.chain_query(a, b, f)
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)
    plan.preds = [(2, "<", -5)]
    k, s = run(gpu, ctx, plan, fact, path)
    assert len(k) == 0 and len(oracle.chain_query(a, b, f, fact_preds=(("date", "<", -5),))[0]) == 0


def _shift_keys(a, b, f, a_map, b_map):
    a, b, f = dict(a), dict(b), dict(f)
    a["key"], f["a_fk"] = a_map(a["key"]), a_map(f["a_fk"])
    b["key"], f["b_fk"] = b_map(b["key"]), b_map(f["b_fk"])
    return a, b, f


def _affine(mul, add):
    return lambda x: (x.astype(np.int64) * mul + add).astype(np.int32)


@pytest.mark.parametrize("path", ["fast", "fast_hash"])
@pytest.mark.parametrize("case", ["b_wide", "a_sparse", "top", "bottom"])
def test_chain_direct_addressing_ranges(gpu, ctx, path, case):
    # B's selected keys over more than 2^20 values (B hashed, A direct), A's
    # keys sparse (A hashed, B direct), and both dense with the ranges ending
    # at INT32_MAX or starting just above the reserved INT32_MIN; some probe
    # keys fall just outside each range
    a, b, f = _chain(n=700_001, na=40_000, nb=6_000)
    na, nb = 40_000, 6_000
    maps = {"b_wide": (_affine(1, 0), _affine(200, 0)),
            "a_sparse": (_affine(65_537, -2 ** 30), _affine(1, 0)),
            "top": (_affine(1, 2 ** 31 - 1 - na), _affine(1, 2 ** 31 - 1 - nb)),
            "bottom": (_affine(1, -2 ** 31), _affine(1, -2 ** 31))}[case]
    a, b, f = _shift_keys(a, b, f, *maps)
    f["a_fk"][::97] = (int(a["key"].min()) - 1) if case != "bottom" else int(a["key"].max()) + 3
    f["b_fk"][5::89] = (int(b["key"].max()) + 1) if case != "top" else int(b["key"].min()) - 2
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()})
    k, s = run(gpu, ctx, plan, [dev(f[c]) for c in FACT_CHAIN], path)
    wk, ws = oracle.chain_query(a, b, f)
    assert len(wk) > 10_000
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


def _chain_ranges(b_range, a_range, n_fact=500_001, nb=6_000, na=40_000, seed=3):
    """Chain tables whose selected B keys span exactly b_range values and whose
    A keys span exactly a_range values (both ends present, B's ends selected);
    some fact keys fall just outside each range."""
    r = np.random.default_rng(seed)

    def keys(n, rng_, base):
        inner = r.choice(np.arange(1, rng_ - 1, dtype=np.int64), n - 2, replace=False)
        return (np.concatenate([[0, rng_ - 1], inner]) + base).astype(np.int32)

    bk, ak = keys(nb, b_range, 11), keys(na, a_range, -500)
    bseg = r.integers(0, 5, nb).astype(np.int32)
    bseg[:2] = 1
    b = {"key": bk, "segment": bseg}
    a = {"key": ak, "date": r.integers(0, 2407, na).astype(np.int32)}
    fa = ak[r.integers(0, na, n_fact)]
    fb = bk[r.integers(0, nb, n_fact)]
    fa[::101] = ak.min() - 1
    fa[50::101] = ak.max() + 1
    fb[7::97] = bk.max() + 1
    f = {"a_fk": fa, "b_fk": fb, "date": r.integers(0, 2407, n_fact).astype(np.int32),
         "price": r.integers(90_000, 10_500_001, n_fact).astype(np.int64),
         "discount": r.integers(0, 11, n_fact).astype(np.int32)}
    return a, b, f


@pytest.mark.parametrize("path", ["fast", "fast_hash"])
@pytest.mark.parametrize("b_range,a_range", [
    (1 << 20, 1 << 17),              # both at their direct limits (A reserves 2^17 slots for 40k keys)
    ((1 << 20) + 1, (1 << 17) + 1),  # one past each: both hashed
    ((1 << 20) - 1, (1 << 17) - 1),  # odd ranges: A's last 16-byte group holds one slot
])
def test_chain_direct_range_limits(gpu, ctx, path, b_range, a_range):
    a, b, f = _chain_ranges(b_range, a_range)
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()})
    k, s = run(gpu, ctx, plan, [dev(f[c]) for c in FACT_CHAIN], path)
    wk, ws = oracle.chain_query(a, b, f)
    assert len(wk) > 5_000
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash", "generic"])
def test_chain_filtered_payload_join(gpu, ctx, path):
    # a predicate on A as well: A's table holds only the selected keys (its
    # build goes through the filter's selection) and the probe of an A key
    # that was filtered out must miss, direct-addressed or hashed
    a, b, f = _chain(n=600_001, na=50_000, nb=5_000)
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()})
    plan.joins[1]["cols"] = [plan.joins[1]["key"], plan.joins[1]["payload"]]
    plan.joins[1]["preds"] = [(1, "<", 900)]
    k, s = run(gpu, ctx, plan, [dev(f[c]) for c in FACT_CHAIN], path)
    wk, ws = oracle.chain_query(a, b, f, a_preds=(("date", "<", 900),))
    assert len(wk) > 5_000
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "fast_hash"])
@pytest.mark.parametrize("side", ["a", "b"])
def test_chain_duplicate_dimension_key(gpu, ctx, path, side):
    # a repeated key in A, or in B's selected rows: reported whether the table
    # is direct-addressed or hashed
    a, b, f = _chain(n=200_001, na=20_000, nb=3_000)
    a, b = {k: v.copy() for k, v in a.items()}, {k: v.copy() for k, v in b.items()}
    t = a if side == "a" else b
    i, j = int(np.flatnonzero(t["key"] == 17)[0]), int(np.flatnonzero(t["key"] == 29)[0])
    t["key"][i] = 29
    if side == "b":
        b["segment"][i] = b["segment"][j] = 1
    plan = gpu.chain_plan({k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()})
    ctx.hash_join_only(path == "fast_hash")
    try:
        gpu.query(ctx, plan, [dev(f[c]) for c in FACT_CHAIN])
        with pytest.raises(gpu.PystError) as e:
            ctx.check()
    finally:
        ctx.hash_join_only(False)
    assert e.value.status == gpu.ERR_DUP_KEY


def test_fast_query_capacity_error(gpu, ctx):
    b, p = gen.star_tables(10_000, 100_000)
    bd = {k: dev(v) for k, v in b.items()}
    k, s, ng = gpu.query(ctx, gpu.star_plan(bd), [dev(p[c]) for c in FACT_STAR], out_cap=10)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_CAPACITY
    assert int(ng.item()) == len(oracle.star_query(b, p)[0])
