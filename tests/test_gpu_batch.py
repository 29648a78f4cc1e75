"""GPU parity of batched fragment execution: every fragment of a batch gets
exactly its one-at-a-time pyst_query result and the oracle's, under every
tuning of the autotuner's grid."""
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


def make_fragments(gpu, nfrag, lo=1e3, hi=2e5):
    sizes, builds = gen.fragment_sizes(nfrag, lo=lo, hi=hi)
    frags, host = [], []
    for f, (p, b) in enumerate(zip(sizes, builds)):
        bt, pt = gen.star_tables(max(int(b), 1), int(p), workload=3, fragment=f)
        bd = {k: dev(v) for k, v in bt.items()}
        fact = [dev(pt[c]) for c in ("fk", "date", "price")]
        frags.append((gpu.star_plan(bd), fact))
        host.append((bt, pt))
    return frags, host


def sorted_np(k, s):
    k, s = k.cpu().numpy(), s.cpu().numpy()
    o = np.argsort(k)
    return k[o], s[o]


@pytest.mark.parametrize("hash_only", [False, True])
@pytest.mark.parametrize("tuning", [None, (16, 256, 0.5), (256, 1024, 0.7), (64, 512, 0.5), (1, 256, 0.0)])
def test_batch_matches_oracle(gpu, ctx, tuning, hash_only):
    # staged tunings (1024-thread blocks) direct-address the fragments' dense
    # dimension keys unless hash tables are forced
    frags, host = make_fragments(gpu, 40)
    batch = gpu.Batch(ctx, frags)
    ctx.hash_join_only(hash_only)
    try:
        batch.run(tuning)
        ctx.check()
    finally:
        ctx.hash_join_only(False)
    for (k, s), (bt, pt) in zip(batch.results(), host):
        wk, ws = oracle.star_query(bt, pt)
        gk, gs = sorted_np(k, s)
        np.testing.assert_array_equal(gk, wk)
        np.testing.assert_array_equal(gs, ws)


def test_batch_equals_one_at_a_time_and_autotune(gpu, ctx):
    frags, host = make_fragments(gpu, 24, lo=1e4, hi=1e6)
    batch = gpu.Batch(ctx, frags)
    best, ms = batch.autotune(reps=1)
    assert best[1] in (256, 512, 1024) and best[2] in (0.5, 0.7) and best[0] in (16, 32, 64, 128, 256)
    assert ms > 0
    batch.run(best)
    ctx.check()
    for (k, s), (plan, fact) in zip(batch.results(), frags):
        r = gpu.query(ctx, plan, fact)
        ctx.check()
        m = int(r[2].item())
        ak, asum = sorted_np(r[0][:m], r[1][:m])
        gk, gs = sorted_np(k, s)
        np.testing.assert_array_equal(gk, ak)
        np.testing.assert_array_equal(gs, asum)


def test_batch_with_empty_fragments(gpu, ctx):
    frags, host = make_fragments(gpu, 6)
    bt, pt = gen.star_tables(1, 0, workload=3, fragment=99)  # empty fact table
    import torch
    frags.insert(2, (gpu.star_plan({k: dev(v) for k, v in bt.items()}),
                     [torch.empty(0, dtype=torch.int32, device="cuda"), torch.empty(0, dtype=torch.int32, device="cuda"),
                      torch.empty(0, dtype=torch.int64, device="cuda")]))
    host.insert(2, (bt, pt))
    batch = gpu.Batch(ctx, frags)
    batch.run((32, 256, 0.5))
    ctx.check()
    for (k, s), (bt, pt) in zip(batch.results(), host):
        wk, ws = oracle.star_query(bt, pt)
        gk, gs = sorted_np(k, s)
        np.testing.assert_array_equal(gk, wk)
        np.testing.assert_array_equal(gs, ws)


def test_batch_large_and_small_fragments(gpu, ctx):
    # filters of every shape in one batch: tables of fewer than 32768 slots use
    # one filter word per slot, larger ones several slots per word, and a
    # fragment of a few rows copies a few words
    spec = [(3_000_001, 1_000_000), (2_000, 200), (500_000, 400_000), (17, 5), (1_200_000, 40_000)]
    frags, host = [], []
    for f, (p, b) in enumerate(spec):
        bt, pt = gen.star_tables(b, p, workload=3, fragment=100 + f)
        bd = {k: dev(v) for k, v in bt.items()}
        frags.append((gpu.star_plan(bd), [dev(pt[c]) for c in ("fk", "date", "price")]))
        host.append((bt, pt))
    batch = gpu.Batch(ctx, frags)
    batch.run((64, 1024, 0.5))
    ctx.check()
    for (k, s), (bt, pt) in zip(batch.results(), host):
        wk, ws = oracle.star_query(bt, pt)
        gk, gs = sorted_np(k, s)
        np.testing.assert_array_equal(gk, wk)
        np.testing.assert_array_equal(gs, ws)


def test_batch_graph_replays_match(gpu, ctx):
    # the batch captured once as a graph and replayed three times, with eager
    # work (a batch run under another tuning) and synchronizations between
    # replays; every output is overwritten before each replay, so each replay
    # must write all of them again
    import torch
    frags, host = make_fragments(gpu, 24, lo=1e3, hi=4e5)
    batch = gpu.Batch(ctx, frags)
    g = batch.graph((64, 1024, 0.5))
    try:
        for rep in range(3):
            if rep == 1:
                batch.run((16, 256, 0.7))
                ctx.check()
            for ok, osum, ng in batch.outs:
                ok.fill_(-7)
                osum.fill_(-7)
                ng.fill_(12345)
            torch.cuda.synchronize()
            g.launch()
            ctx.check()
            for (k, s), (bt, pt) in zip(batch.results(), host):
                wk, ws = oracle.star_query(bt, pt)
                gk, gs = sorted_np(k, s)
                np.testing.assert_array_equal(gk, wk)
                np.testing.assert_array_equal(gs, ws)
    finally:
        g.close()


def test_batch_mixed_key_ranges(gpu, ctx):
    # fragments whose dimension keys are dense, sparse (hash table) or span the
    # largest direct range, in one staged batch
    import torch
    frags, host = [], []
    for f in range(6):
        bt, pt = gen.star_tables(20_000 + 7_000 * f, 300_001, workload=3, fragment=f)
        if f % 3 == 1:  # sparse keys
            bt["key"] = (bt["key"].astype(np.int64) * 65_537 - 2 ** 30).astype(np.int32)
            pt["fk"] = (pt["fk"].astype(np.int64) * 65_537 - 2 ** 30).astype(np.int32)
        elif f % 3 == 2:  # keys spread over [1, 2^21]
            bt["key"] = (bt["key"].astype(np.int64) * 40).astype(np.int32)
            pt["fk"] = (pt["fk"].astype(np.int64) * 40).astype(np.int32)
        frags.append((gpu.star_plan({k: dev(v) for k, v in bt.items()}, max_load=0.02),
                      [dev(pt[c]) for c in ("fk", "date", "price")]))
        host.append((bt, pt))
    batch = gpu.Batch(ctx, frags)
    batch.run((8, 1024, 0.0))
    ctx.check()
    for (k, s), (bt, pt) in zip(batch.results(), host):
        wk, ws = oracle.star_query(bt, pt)
        assert len(wk) > 100
        gk, gs = sorted_np(k, s)
        np.testing.assert_array_equal(gk, wk)
        np.testing.assert_array_equal(gs, ws)


@pytest.mark.parametrize("hash_only", [False, True])
def test_batch_sums_added_directly(gpu, ctx, hash_only):
    # every fact row matches (no predicate on either side): the pools, sized
    # for an eighth of a fragment's rows, run out and the rest is added into
    # the slot sums directly; one fragment's values are too wide to stage
    frags, host = [], []
    for f in range(4):
        bt, pt = gen.star_tables(5_000 + 3_000 * f, 400_003, workload=3, fragment=200 + f)
        if f == 3:
            pt["price"] = (pt["price"].astype(np.uint64) << np.uint64(40)).view(np.int64)
        plan = gpu.star_plan({k: dev(v) for k, v in bt.items()})
        plan.joins[0]["preds"] = []
        plan.preds = []
        frags.append((plan, [dev(pt[c]) for c in ("fk", "date", "price")]))
        host.append((bt, pt))
    batch = gpu.Batch(ctx, frags)
    ctx.hash_join_only(hash_only)
    try:
        batch.run((4, 1024, 0.5))
        ctx.check()
    finally:
        ctx.hash_join_only(False)
    for (k, s), (bt, pt) in zip(batch.results(), host):
        wk, ws = oracle.star_query(bt, pt, build_preds=(), probe_preds=())
        gk, gs = sorted_np(k, s)
        np.testing.assert_array_equal(gk, wk)
        np.testing.assert_array_equal(gs, ws)


@pytest.mark.parametrize("hash_only", [False, True])
def test_batch_duplicate_dimension_key(gpu, ctx, hash_only):
    # one fragment of three repeats a selected dimension key: the batch reports
    # a duplicate key whether its table is direct-addressed or hashed
    frags = []
    for f in range(3):
        bt, pt = gen.star_tables(30_000, 200_001, workload=3, fragment=300 + f)
        if f == 1:
            i = int(np.flatnonzero(bt["key"] == 17)[0])
            j = int(np.flatnonzero(bt["key"] == 23)[0])
            bt["key"][i] = 23
            bt["segment"][i] = bt["segment"][j] = 1
        frags.append((gpu.star_plan({k: dev(v) for k, v in bt.items()}),
                      [dev(pt[c]) for c in ("fk", "date", "price")]))
    batch = gpu.Batch(ctx, frags)
    ctx.hash_join_only(hash_only)
    try:
        batch.run((4, 1024, 0.5))
        with pytest.raises(gpu.PystError) as e:
            ctx.check()
    finally:
        ctx.hash_join_only(False)
    assert e.value.status == gpu.ERR_DUP_KEY
