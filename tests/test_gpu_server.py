"""GPU tests of the serving loop: every request's result equals the oracle's on
its fact prefix, equals its result when served alone, and admission control
keeps load beyond the memory budget waiting instead of failing."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

COLS = ("a_fk", "b_fk", "date", "price", "discount")
NA, NB, NF = 30_000, 3_000, 3_000_000


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def db():
    import torch
    a, b = gen.chain_dims(NA, NB)
    f = gen.chain_fact(NF, NA, NB, 0.0)
    host = [torch.from_numpy(f[c]).pin_memory() for c in COLS]
    return a, b, f, host, {k: dev(v) for k, v in a.items()}, {k: dev(v) for k, v in b.items()}


def expected(kind, a, b, f, rows):
    pref = {c: v[:rows] for c, v in f.items()}
    if kind == "star":
        return oracle.star_query(b, {"fk": pref["b_fk"], "date": pref["date"], "price": pref["price"]})
    return oracle.chain_query(a, b, pref)


def plan_for(gpu, kind, ad, bd):
    if kind == "star":
        return gpu.fact_star_plan(bd), NB
    return gpu.chain_plan(ad, bd, max_groups=400_000), 400_000


def sorted_np(k, s):
    k, s = k.cpu().numpy(), s.cpu().numpy()
    o = np.argsort(k)
    return k[o], s[o]


def test_server_mix_matches_oracle_and_alone(gpu, db):
    a, b, f, host, ad, bd = db
    rng = np.random.default_rng(5)
    reqs = [("star" if i % 2 == 0 else "chain", int(rng.integers(1, NF + 1))) for i in range(12)]
    reqs[3] = ("chain", NF)
    srv = gpu.Server(host, budget=1 << 30, max_active=6, nbuf=3, chunk_rows=250_000)
    tickets = []
    for kind, rows in reqs:
        plan, cap = plan_for(gpu, kind, ad, bd)
        tickets.append(srv.submit(plan, rows, cap))
    mixed = [srv.wait(t) for t in tickets]
    srv.check()
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["max_active_seen"] > 1
    # the shared scan copied fewer chunks than private scans would have
    assert st["chunks_copied"] < sum(-(-r // 250_000) for _, r in reqs)
    srv.close()
    alone_srv = gpu.Server(host, budget=1 << 30, max_active=1, nbuf=2, chunk_rows=250_000)
    for (kind, rows), (k, s, lat) in zip(reqs, mixed):
        assert lat > 0
        got = sorted_np(k, s)
        wk, ws = expected(kind, a, b, f, rows)
        np.testing.assert_array_equal(got[0], wk)
        np.testing.assert_array_equal(got[1], ws)
    for kind, rows in reqs[:4]:
        plan, cap = plan_for(gpu, kind, ad, bd)
        k, s, _ = alone_srv.wait(alone_srv.submit(plan, rows, cap))
        got = sorted_np(k, s)
        wk, ws = expected(kind, a, b, f, rows)
        np.testing.assert_array_equal(got[0], wk)
        np.testing.assert_array_equal(got[1], ws)
    alone_srv.check()
    alone_srv.close()


def test_server_admission_waits_for_memory(gpu, db):
    a, b, f, host, ad, bd = db
    # each chain request reserves a 400k-group table (~16 MiB); a ~40 MiB budget admits two at a time
    srv = gpu.Server(host, budget=40 << 20, max_active=8, nbuf=2, chunk_rows=500_000)
    plan, cap = plan_for(gpu, "chain", ad, bd)
    tickets = [srv.submit(plan, NF - 1000 * i, cap) for i in range(6)]
    res = [srv.wait(t) for t in tickets]
    srv.check()
    st = srv.stats()
    assert st["admission_waits"] > 0 and st["max_active_seen"] <= 3
    for i, (k, s, _) in enumerate(res):
        got = sorted_np(k, s)
        wk, ws = expected("chain", a, b, f, NF - 1000 * i)
        np.testing.assert_array_equal(got[0], wk)
        np.testing.assert_array_equal(got[1], ws)
    srv.close()


def test_server_rejects_request_that_cannot_fit(gpu, db):
    a, b, f, host, ad, bd = db
    srv = gpu.Server(host, budget=8 << 20, max_active=2, nbuf=2, chunk_rows=500_000)
    plan, cap = plan_for(gpu, "chain", ad, bd)
    t = srv.submit(plan, NF, cap)
    with pytest.raises(gpu.PystError) as e:
        srv.wait(t)
    assert e.value.status == gpu.ERR_NOMEM
    # a request that fits is still served afterwards
    plan, cap = plan_for(gpu, "star", ad, bd)
    k, s, _ = srv.wait(srv.submit(plan, 100_000, cap))
    got = sorted_np(k, s)
    wk, ws = expected("star", a, b, f, 100_000)
    np.testing.assert_array_equal(got[0], wk)
    np.testing.assert_array_equal(got[1], ws)
    srv.close()


def test_packed_server_matches_oracle(gpu, db):
    # the same mix served from bit-packed host columns: each chunk crosses the link packed
    # and is decoded on the device; a chunk of 262144 rows is a whole number of blocks
    import torch
    a, b, f, host, ad, bd = db
    packed = [(*gpu.pack(t), NF, t.dtype) for t in host]
    rng = np.random.default_rng(6)
    reqs = [("star" if i % 2 == 0 else "chain", int(rng.integers(1, NF + 1))) for i in range(8)]
    reqs[1] = ("chain", NF)
    reqs[2] = ("star", 1)
    srv = gpu.Server(None, budget=1 << 30, max_active=5, nbuf=3, chunk_rows=262_144, packed=packed)
    tickets = []
    for kind, rows in reqs:
        plan, cap = plan_for(gpu, kind, ad, bd)
        tickets.append(srv.submit(plan, rows, cap))
    results = [srv.wait(t) for t in tickets]
    srv.check()
    st = srv.stats()
    assert st["completed"] == len(reqs)
    # packed chunks: fewer bytes per copied chunk than one raw chunk (24 B a row)
    assert 0 < st["bytes_copied"] / st["chunks_copied"] < 262_144 * 24
    srv.close()
    for (kind, rows), (k, s, lat) in zip(reqs, results):
        got = sorted_np(k, s)
        wk, ws = expected(kind, a, b, f, rows)
        np.testing.assert_array_equal(got[0], wk)
        np.testing.assert_array_equal(got[1], ws)
    with pytest.raises(gpu.PystError) as e:
        gpu.Server(None, chunk_rows=250_000, packed=packed)  # not a multiple of 1024
    assert e.value.status == gpu.ERR_ARG


def test_server_request_failing_on_the_host_is_finished(gpu, db):
    # The second fact pass of a six-chunk request fails on the host (test hook,
    # no device work involved): the request must be finished with that error,
    # give back its slot and memory, and leave the server serving.
    a, b, f, host, ad, bd = db
    srv = gpu.Server(host, budget=256 << 20, max_active=2, nbuf=2, chunk_rows=500_000)
    srv.option(gpu.OPT_FAIL_FACT_PASS, 2)
    plan, cap = plan_for(gpu, "chain", ad, bd)
    t = srv.submit(plan, NF, cap)
    with pytest.raises(gpu.PystError) as e:
        srv.wait(t)
    assert e.value.status == gpu.ERR_HIP
    for kind, rows in (("star", NF), ("chain", 1_234_567)):
        plan, cap = plan_for(gpu, kind, ad, bd)
        k, s, _ = srv.wait(srv.submit(plan, rows, cap))
        got = sorted_np(k, s)
        wk, ws = expected(kind, a, b, f, rows)
        np.testing.assert_array_equal(got[0], wk)
        np.testing.assert_array_equal(got[1], ws)
    st = srv.stats()
    assert st["completed"] == 3
    srv.close()  # returns: nothing is left active


def test_server_device_errors_belong_to_their_request(gpu, db):
    # In one mix: a request whose groups overflow its output capacity, and a
    # request over a dimension with a duplicate key.  Each fails with its own
    # error; every other request of the mix is exact.
    import torch
    a, b, f, host, ad, bd = db
    bdup = {k: v.clone() for k, v in bd.items()}
    bdup["key"][7] = bdup["key"][8]
    bdup["segment"][7] = bdup["segment"][8] = 1  # both rows pass the dimension filter
    srv = gpu.Server(host, budget=1 << 30, max_active=6, nbuf=3, chunk_rows=250_000)
    good = []
    plan, cap = plan_for(gpu, "chain", ad, bd)
    good.append((("chain", 2_000_000), srv.submit(plan, 2_000_000, cap)))
    t_cap = srv.submit(plan, 1_500_000, 10)  # far more than 10 groups
    plan_s, cap_s = plan_for(gpu, "star", ad, bd)
    good.append((("star", NF), srv.submit(plan_s, NF, cap_s)))
    t_dup = srv.submit(gpu.fact_star_plan(bdup), 1_000_000, NB)
    good.append((("star", 777_777), srv.submit(plan_s, 777_777, cap_s)))
    with pytest.raises(gpu.PystError) as e:
        srv.wait(t_cap)
    assert e.value.status == gpu.ERR_CAPACITY
    with pytest.raises(gpu.PystError) as e:
        srv.wait(t_dup)
    assert e.value.status == gpu.ERR_DUP_KEY
    for (kind, rows), t in good:
        k, s, _ = srv.wait(t)
        got = sorted_np(k, s)
        wk, ws = expected(kind, a, b, f, rows)
        np.testing.assert_array_equal(got[0], wk)
        np.testing.assert_array_equal(got[1], ws)
    srv.check()  # nothing was latched in the server-wide word
    srv.close()
    del torch


def test_server_forget_tables_rebuilds_over_new_contents(gpu, db):
    # Resident tables are keyed by column addresses: after the caller changes a
    # dimension column in place and says so, the next request sees the new
    # contents.
    a, b, f, host, ad, bd = db
    b2 = {k: v.copy() for k, v in b.items()}
    bd2 = {k: dev(v) for k, v in b2.items()}
    srv = gpu.Server(host, budget=1 << 30, max_active=4, nbuf=2, chunk_rows=500_000)
    plan = gpu.fact_star_plan(bd2)
    k, s, _ = srv.wait(srv.submit(plan, 2_000_000, NB))
    got = sorted_np(k, s)
    wk, ws = expected("star", a, b2, f, 2_000_000)
    np.testing.assert_array_equal(got[0], wk)
    np.testing.assert_array_equal(got[1], ws)
    addr = bd2["segment"].data_ptr()
    b2["segment"] = ((b2["segment"] + 1) % 5).astype(np.int32)
    bd2["segment"].copy_(dev(b2["segment"]))
    assert bd2["segment"].data_ptr() == addr
    srv.forget_tables(bd2["segment"])
    k, s, _ = srv.wait(srv.submit(gpu.fact_star_plan(bd2), 2_000_000, NB))
    got = sorted_np(k, s)
    wk, ws = expected("star", a, b2, f, 2_000_000)
    np.testing.assert_array_equal(got[0], wk)
    np.testing.assert_array_equal(got[1], ws)
    srv.forget_tables()  # everything
    k, s, _ = srv.wait(srv.submit(gpu.fact_star_plan(bd2), 1_000, NB))
    wk, ws = expected("star", a, b2, f, 1_000)
    np.testing.assert_array_equal(sorted_np(k, s)[1], ws)
    srv.close()


def test_server_evicts_idle_tables_when_memory_is_short(gpu, db):
    # Many distinct dimension tables in a row, each only used once: idle cached
    # tables give way instead of failing new requests with NOMEM.
    a, b, f, host, ad, bd = db
    srv = gpu.Server(host, budget=3 << 20, max_active=1, nbuf=2, chunk_rows=500_000)
    keep = []  # distinct live addresses: every request builds its own tables (about 0.2 MiB each)
    for i in range(30):
        keep.append({k: dev(v) for k, v in b.items()})
        k, s, _ = srv.wait(srv.submit(gpu.fact_star_plan(keep[-1]), 300_000 + i, NB))
        wk, ws = expected("star", a, b, f, 300_000 + i)
        np.testing.assert_array_equal(sorted_np(k, s)[1], ws)
    srv.close()


def test_server_poll_reports_each_request_once(gpu, db):
    # poll never blocks: a client loop collects every request by polling alone
    import time
    a, b, f, host, ad, bd = db
    rows = [NF, 700_001, 1, 2_000_000]
    srv = gpu.Server(host, budget=1 << 30, max_active=2, nbuf=2, chunk_rows=250_000)
    kinds = ["chain", "star", "star", "chain"]
    tickets = {}
    for kind, r in zip(kinds, rows):
        plan, cap = plan_for(gpu, kind, ad, bd)
        tickets[srv.submit(plan, r, cap)] = (kind, r)
    got, polls = {}, 0
    deadline = time.monotonic() + 60
    while len(got) < len(tickets) and time.monotonic() < deadline:
        for t in tickets:
            if t in got:
                continue
            polls += 1
            res = srv.poll(t)
            if res is not None:
                got[t] = res
        time.sleep(0.001)
    assert len(got) == len(tickets)
    assert polls > len(tickets)  # the first poll of the full-size chain request found it running
    for t, (kind, r) in tickets.items():
        k, s, lat = got[t]
        assert lat > 0
        wk, ws = expected(kind, a, b, f, r)
        gk, gs = sorted_np(k, s)
        np.testing.assert_array_equal(gk, wk)
        np.testing.assert_array_equal(gs, ws)
    with pytest.raises(gpu.PystError) as e:  # reported once, then unknown
        gpu._check(gpu._lib.pyst_server_poll(srv.h, next(iter(tickets)), gpu.ctypes.byref(gpu.ctypes.c_int()), None))
    assert e.value.status == gpu.ERR_ARG
    srv.check()
    srv.close()
