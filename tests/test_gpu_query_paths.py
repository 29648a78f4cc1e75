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
    ctx.generic_only(path == "generic")
    try:
        k, s, ng = gpu.query(ctx, plan, fact, out_cap=out_cap)
        ctx.check()
    finally:
        ctx.generic_only(False)
    m = int(ng.item())
    k, s = k[:m].cpu().numpy(), s[:m].cpu().numpy()
    o = np.argsort(k, kind="stable")
    return k[o], s[o]


@pytest.mark.parametrize("path", ["fast", "generic"])
@pytest.mark.parametrize("nb,np_", [(2, 3), (30_000, 300_001), (150_000, 1_500_000)])
def test_star_both_paths(gpu, ctx, path, nb, np_):
    b, p = gen.star_tables(nb, np_)
    bd = {k: dev(v) for k, v in b.items()}
    k, s = run(gpu, ctx, gpu.star_plan(bd), [dev(p[c]) for c in FACT_STAR], path)
    wk, ws = oracle.star_query(b, p)
    np.testing.assert_array_equal(k, wk)
    np.testing.assert_array_equal(s, ws)


@pytest.mark.parametrize("path", ["fast", "generic"])
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


@pytest.mark.parametrize("path", ["fast", "generic"])
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


def _chain(n=1_000_003, na=40_000, nb=4_000, zs=0.0):
    a, b = gen.chain_dims(na, nb)
    f = gen.chain_fact(n, na, nb, zs)
    return a, b, f


@pytest.mark.parametrize("path", ["fast", "generic"])
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


@pytest.mark.parametrize("path", ["fast", "generic"])
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


def test_fast_query_capacity_error(gpu, ctx):
    b, p = gen.star_tables(10_000, 100_000)
    bd = {k: dev(v) for k, v in b.items()}
    k, s, ng = gpu.query(ctx, gpu.star_plan(bd), [dev(p[c]) for c in FACT_STAR], out_cap=10)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_CAPACITY
    assert int(ng.item()) == len(oracle.star_query(b, p)[0])
