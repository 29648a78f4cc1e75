"""CPU oracle for the relational hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never loads it
and shares no code with it.

The arithmetic lives in ``oracle.cpp`` (plain single-threaded C++ built with
g++); this module only builds it and marshals numpy arrays.  Every function
returns numpy arrays.

Predicates are lists of ``(column index, op, constant)`` with op one of
``== != < <= > >=``; a row passes when all of them hold (values compared as
int64).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_SRC_MT = os.path.join(_HERE, "threaded.cpp")  # the threaded CPU baseline (same algorithm)
_LIB = os.path.join(_HERE, "liboracle.so")
_OPS = {"==": 0, "!=": 1, "<": 2, "<=": 3, ">": 4, ">=": 5}

_lib = None


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_MT))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, _SRC_MT])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.oracle_fmix32.argtypes = [ctypes.c_uint32]
        lib.oracle_fmix32.restype = ctypes.c_uint32
        lib.oracle_fmix64.argtypes = [ctypes.c_uint64]
        lib.oracle_fmix64.restype = ctypes.c_uint64
        lib.oracle_filter.argtypes = [p, p, i32, i64, p, p, p, i32, p]
        lib.oracle_filter.restype = i64
        lib.oracle_partition.argtypes = [p, i32, i64, p, i64, p, p, i32, ctypes.c_uint32, p, p, p]
        lib.oracle_partition.restype = i64
        lib.oracle_join.argtypes = [p, i32, i64, p, i64, p, i32, i64, p, i64, p, p, i64]
        lib.oracle_join.restype = i64
        lib.oracle_groupby_sum.argtypes = [p, i32, p, i32, i64, p, i64, p, p]
        lib.oracle_groupby_sum.restype = i64
        lib.oracle_star_query.argtypes = [p, p, i64, p, p, p, i32, p, p, p, i64, p, p, p, i32, p, p]
        lib.oracle_star_query.restype = i64
        lib.oracle_chain_query.argtypes = ([p, p, i64, p, p, p, i32] + [p, p, i64, p, p, p, i32]
                                           + [p, p, p, p, p, i64, p, p, p, i32, i64, p, p])
        lib.oracle_chain_query.restype = i64
        lib.baseline_star_query_mt.argtypes = [p, p, i64, p, p, p, i32, p, p, p, i64, p, p, p, i32, i32, p, p, p]
        lib.baseline_star_query_mt.restype = i64
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _col(a):
    a = np.ascontiguousarray(a)
    if a.dtype not in (np.int32, np.int64):
        raise TypeError("oracle columns are int32 or int64")
    return a


def _preds(preds):
    preds = list(preds or [])
    c = np.array([p[0] for p in preds], dtype=np.int32)
    o = np.array([_OPS[p[1]] for p in preds], dtype=np.int32)
    v = np.array([p[2] for p in preds], dtype=np.int64)
    return c, o, v, len(preds)


def _sel(sel):
    if sel is None:
        return None, 0
    s = np.ascontiguousarray(sel, dtype=np.int32)
    return s, len(s)


def fmix32(x: int) -> int:
    return int(_load().oracle_fmix32(x & 0xFFFFFFFF))


def fmix64(x: int) -> int:
    return int(_load().oracle_fmix64(x & 0xFFFFFFFFFFFFFFFF))


def filter(cols, preds):
    """Ascending int32 row ids of the rows that satisfy every predicate."""
    cols = [_col(c) for c in cols]
    n = len(cols[0]) if cols else 0
    ptrs = (ctypes.c_void_p * max(1, len(cols)))(*[c.ctypes.data for c in cols])
    is64 = np.array([c.dtype == np.int64 for c in cols] or [0], dtype=np.int32)
    c, o, v, npred = _preds(preds)
    out = np.empty(max(n, 1), dtype=np.int32)
    m = _load().oracle_filter(ptrs, _ptr(is64), len(cols), n, _ptr(c), _ptr(o), _ptr(v), npred,
                              _ptr(out))
    if m < 0:
        raise ValueError("predicate column out of range")
    return out[:m].copy()


def partition(key, payloads, fanout, sel=None):
    """Stable hash partition; returns (out_key, [out_payloads], offsets[F+1])."""
    key = _col(key)
    pays = [np.ascontiguousarray(p) for p in payloads]
    s, ns = _sel(sel)
    m = ns if s is not None else len(key)
    out_key = np.empty(m, dtype=key.dtype)
    out_pay = [np.empty(m, dtype=p.dtype) for p in pays]
    offsets = np.empty(fanout + 1, dtype=np.int64)
    k = max(1, len(pays))
    pin = (ctypes.c_void_p * k)(*[p.ctypes.data for p in pays])
    pout = (ctypes.c_void_p * k)(*[p.ctypes.data for p in out_pay])
    widths = np.array([p.dtype.itemsize for p in pays] or [0], dtype=np.int32)
    r = _load().oracle_partition(key.ctypes.data, int(key.dtype == np.int64), len(key), _ptr(s),
                                 ns, pin, _ptr(widths), len(pays), fanout, out_key.ctypes.data,
                                 pout, offsets.ctypes.data)
    if r < 0:
        raise ValueError("fanout must be >= 1")
    return out_key, out_pay, offsets


def join(build_key, probe_key, build_sel=None, probe_sel=None):
    """Inner equi-join; returns (probe_row, build_row) int32 arrays in canonical order."""
    bk, pk = _col(build_key), _col(probe_key)
    bs, nbs = _sel(build_sel)
    ps, nps = _sel(probe_sel)
    lib = _load()
    args = (bk.ctypes.data, int(bk.dtype == np.int64), len(bk), _ptr(bs), nbs, pk.ctypes.data,
            int(pk.dtype == np.int64), len(pk), _ptr(ps), nps)
    m = lib.oracle_join(*args, None, None, 0)
    op = np.empty(max(m, 1), dtype=np.int32)
    ob = np.empty(max(m, 1), dtype=np.int32)
    lib.oracle_join(*args, op.ctypes.data, ob.ctypes.data, m)
    return op[:m].copy(), ob[:m].copy()


def join_materialize(build_key, build_cols, probe_key, probe_cols):
    """Inner equi-join with materialized result tuples (Sec. 3.1, "Anatomy of a
    Distributed Hash Join": the probe emits every matching (probe tuple, build
    tuple) pair).  Returns (probe_row, build_row, columns): the match pairs in
    the canonical order of join() and, per match, the probe columns at its probe
    row followed by the build columns at its build row."""
    pr, br = join(build_key, probe_key)
    cols = [np.asarray(c)[pr] for c in probe_cols] + [np.asarray(c)[br] for c in build_cols]
    return pr, br, cols


def groupby_sum(key, val, sel=None):
    """GROUP BY key SUM(val): (keys int64 ascending, sums int64)."""
    k, v = _col(key), _col(val)
    s, ns = _sel(sel)
    n = max(len(k), 1)
    ok = np.empty(n, dtype=np.int64)
    osum = np.empty(n, dtype=np.int64)
    g = _load().oracle_groupby_sum(k.ctypes.data, int(k.dtype == np.int64), v.ctypes.data,
                                   int(v.dtype == np.int64), len(k), _ptr(s), ns, ok.ctypes.data,
                                   osum.ctypes.data)
    return ok[:g].copy(), osum[:g].copy()


def star_query(build, probe, build_preds=(("segment", "==", 1),),
               probe_preds=(("date", "<", 1200),)):
    """Star query over build {key, segment} and probe {fk, date, price}.

    Predicates name columns (build: key, segment; probe: fk, date, price).
    Returns (keys ascending, sums).
    """
    bnames, pnames = ["key", "segment"], ["fk", "date", "price"]
    bk = np.ascontiguousarray(build["key"], dtype=np.int32)
    bs = np.ascontiguousarray(build["segment"], dtype=np.int32)
    fk = np.ascontiguousarray(probe["fk"], dtype=np.int32)
    dt = np.ascontiguousarray(probe["date"], dtype=np.int32)
    pr = np.ascontiguousarray(probe["price"], dtype=np.int64)
    bc, bo, bv, nbp = _preds([(bnames.index(c), o, v) for c, o, v in build_preds])
    pc, po, pv, npp = _preds([(pnames.index(c), o, v) for c, o, v in probe_preds])
    n = max(len(fk), 1)
    ok = np.empty(n, dtype=np.int64)
    osum = np.empty(n, dtype=np.int64)
    g = _load().oracle_star_query(bk.ctypes.data, bs.ctypes.data, len(bk), _ptr(bc), _ptr(bo),
                                  _ptr(bv), nbp, fk.ctypes.data, dt.ctypes.data, pr.ctypes.data,
                                  len(fk), _ptr(pc), _ptr(po), _ptr(pv), npp, ok.ctypes.data,
                                  osum.ctypes.data)
    return ok[:g].copy(), osum[:g].copy()


def star_query_threaded(build, probe, build_preds=(("segment", "==", 1),),
                        probe_preds=(("date", "<", 1200),), threads=0):
    """The star query on `threads` host threads (0: all), the threaded CPU
    baseline of ``threaded.cpp``.  Returns (keys ascending, sums, threads used)."""
    bnames, pnames = ["key", "segment"], ["fk", "date", "price"]
    bk = np.ascontiguousarray(build["key"], dtype=np.int32)
    bs = np.ascontiguousarray(build["segment"], dtype=np.int32)
    fk = np.ascontiguousarray(probe["fk"], dtype=np.int32)
    dt = np.ascontiguousarray(probe["date"], dtype=np.int32)
    pr = np.ascontiguousarray(probe["price"], dtype=np.int64)
    bc, bo, bv, nbp = _preds([(bnames.index(c), o, v) for c, o, v in build_preds])
    pc, po, pv, npp = _preds([(pnames.index(c), o, v) for c, o, v in probe_preds])
    n = max(len(fk), 1)
    ok = np.empty(n, dtype=np.int64)
    osum = np.empty(n, dtype=np.int64)
    used = np.zeros(1, dtype=np.int32)
    g = _load().baseline_star_query_mt(bk.ctypes.data, bs.ctypes.data, len(bk), _ptr(bc), _ptr(bo),
                                       _ptr(bv), nbp, fk.ctypes.data, dt.ctypes.data, pr.ctypes.data,
                                       len(fk), _ptr(pc), _ptr(po), _ptr(pv), npp, int(threads),
                                       ok.ctypes.data, osum.ctypes.data, used.ctypes.data)
    return ok[:g].copy(), osum[:g].copy(), int(used[0])


def chain_query(a, b, fact, a_preds=(), b_preds=(("segment", "==", 1),),
                fact_preds=(("date", "<", 1200),), vconst=100):
    """Two-join chain; returns (packed (B.key<<32 | A.date) keys ascending, sums)."""
    an, bn = ["key", "date"], ["key", "segment"]
    fn = ["a_fk", "b_fk", "date", "price", "discount"]
    ak = np.ascontiguousarray(a["key"], dtype=np.int32)
    ad = np.ascontiguousarray(a["date"], dtype=np.int32)
    bk = np.ascontiguousarray(b["key"], dtype=np.int32)
    bs = np.ascontiguousarray(b["segment"], dtype=np.int32)
    fa = np.ascontiguousarray(fact["a_fk"], dtype=np.int32)
    fb = np.ascontiguousarray(fact["b_fk"], dtype=np.int32)
    fd = np.ascontiguousarray(fact["date"], dtype=np.int32)
    fp = np.ascontiguousarray(fact["price"], dtype=np.int64)
    fdc = np.ascontiguousarray(fact["discount"], dtype=np.int32)
    ac, ao, av, nap = _preds([(an.index(c), o, v) for c, o, v in a_preds])
    bc, bo, bv, nbp = _preds([(bn.index(c), o, v) for c, o, v in b_preds])
    fc, fo, fv, nfp = _preds([(fn.index(c), o, v) for c, o, v in fact_preds])
    n = max(len(fa), 1)
    ok = np.empty(n, dtype=np.int64)
    osum = np.empty(n, dtype=np.int64)
    g = _load().oracle_chain_query(
        ak.ctypes.data, ad.ctypes.data, len(ak), _ptr(ac), _ptr(ao), _ptr(av), nap,
        bk.ctypes.data, bs.ctypes.data, len(bk), _ptr(bc), _ptr(bo), _ptr(bv), nbp,
        fa.ctypes.data, fb.ctypes.data, fd.ctypes.data, fp.ctypes.data, fdc.ctypes.data, len(fa),
        _ptr(fc), _ptr(fo), _ptr(fv), nfp, vconst, ok.ctypes.data, osum.ctypes.data)
    return ok[:g].copy(), osum[:g].copy()
