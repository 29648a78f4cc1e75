"""GPU parity of the group-by's two paths -- the radix-partitioned one (pairs
moved twice into 4096 hash buckets, each summed in an LDS table) that
pyst_groupby_sum takes from 1M rows up to 16M groups, and the HBM hash table
it takes otherwise or when PYST_OPT_GROUPBY_HASH_ONLY is set -- against the
oracle, on group counts from one heavy key to all-distinct keys."""
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
    c.groupby_hash_only(False)
    c.close()


def run(gpu, ctx, k, v, hash_only, **kw):
    ctx.groupby_hash_only(hash_only)
    try:
        gk, gs, ng = gpu.groupby_sum(ctx, dev(k), dev(v), **kw)
        ctx.check()
    finally:
        ctx.groupby_hash_only(False)
    m = int(host(ng)[0])
    return host(gk, m), host(gs, m)


def check(got, want, sorted_out=False):
    gk, gs = got
    wk, ws = want
    assert len(gk) == len(wk)
    if not sorted_out:
        o = np.argsort(gk, kind="stable")
        gk, gs = gk[o], gs[o]
    np.testing.assert_array_equal(gk, wk)
    np.testing.assert_array_equal(gs, ws)


@pytest.mark.parametrize("hash_only", [False, True])
@pytest.mark.parametrize("n,nkeys", [(1 << 20, 300_000), (1_500_000, 1 << 40), (3_000_001, 50), (2_500_000, 1)])
def test_groupby_paths_match_oracle(gpu, ctx, hash_only, n, nkeys):
    rng = np.random.default_rng(n + nkeys)
    k = rng.integers(0, nkeys, n)  # int64 keys; 2^40 of them makes nearly every key distinct
    v = rng.integers(-10**12, 10**12, n)
    check(run(gpu, ctx, k, v, hash_only), oracle.groupby_sum(k, v))


@pytest.mark.parametrize("hash_only", [False, True])
def test_groupby_q18_shape_with_selection_sorted(gpu, ctx, hash_only):
    li = gen.q18_lineitem(4_000_000, 1_000_000)
    k, v = li["orderkey"], li["quantity"]
    sel = np.nonzero(v > 10)[0].astype(np.int32)
    got = run(gpu, ctx, k, v, hash_only, sel=dev(sel), nsel=dev(np.array([len(sel)], np.int64)), sort_by_key=True)
    check(got, oracle.groupby_sum(k, v, sel), sorted_out=True)


def test_groupby_radix_errors(gpu, ctx):
    n = 1 << 20
    k = np.arange(n, dtype=np.int64)
    k[777] = -2**63  # the EMPTY sentinel
    ctx.groupby_hash_only(False)
    gpu.groupby_sum(ctx, dev(k), dev(k))
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_KEY
    # more groups than max_groups: the count holds the need
    k = np.arange(n, dtype=np.int32)
    gk, gs, ng = gpu.groupby_sum(ctx, dev(k), dev(k), max_groups=1000)
    with pytest.raises(gpu.PystError) as e:
        ctx.check()
    assert e.value.status == gpu.ERR_CAPACITY
    assert int(host(ng)[0]) == n
    got = host(gk)
    assert len(np.unique(got)) == 1000 and got.min() >= 0 and got.max() < n


@pytest.mark.parametrize("n,nkeys,sel_every", [(1 << 20, 300_000, 0), (2_000_003, 2**32, 0), (3_000_001, 7, 3),
                                               (1_200_000, 1, 0), (5_000_000, 4_000_000, 2)])
def test_groupby_narrow_pairs_match_oracle(gpu, ctx, n, nkeys, sel_every):
    # int32 keys and values: the radix path moves 8-byte pairs; keys span the
    # whole int32 range (INT32_MIN included: only the int64 EMPTY key is reserved)
    rng = np.random.default_rng(n ^ nkeys)
    if nkeys >= 2**32:
        k = rng.integers(-2**31, 2**31, n).astype(np.int32)
        k[:5] = [-2**31, 2**31 - 1, 0, -1, -2**31]
    else:
        k = (rng.integers(0, nkeys, n) - nkeys // 2).astype(np.int32)
    v = rng.integers(-2**31, 2**31, n).astype(np.int32)
    kw = {}
    sel = None
    if sel_every:
        sel = np.nonzero(rng.integers(0, sel_every, n) == 0)[0].astype(np.int32)
        kw = {"sel": dev(sel), "nsel": dev(np.array([len(sel)], np.int64))}
    want = oracle.groupby_sum(k, v, sel)
    check(run(gpu, ctx, k, v, False, **kw), want)
    check(run(gpu, ctx, k, v, True, **kw), want)
