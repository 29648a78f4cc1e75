"""Seeded synthetic inputs for the relational hot path.

This module produces INPUT columns only and holds none of the query arithmetic:
no hashing, no predicates, no joins, no sums.  Both the GPU path and the CPU
oracle are fed from it, so neither side's result can leak into the other.

The tables have the shapes and value distributions of the workloads the path
is measured on (a star join with a 5-valued dimension segment, a fact table
with a ~2407-day date, a scaled-cents price and a 0..10 discount):

* star  : build {key = shuffled 1..Nb, segment U[0,4]},
          probe {fk U[1,Nb], date U[0,2406], price int64 U[90000,10500000]}
* join  : build {key = shuffled 1..Nb, c0..c(k-1) int64 U[-2^62, 2^62]},
          probe {key U[1, 2 Nb] (half the probe keys find a build key),
                 c0..c(k-1) int64 U[-2^62, 2^62]}
* q18   : lineitem-like {orderkey U[1,No], quantity U[1,50]} (about 4 rows per key
          at No = N/4, the TPC-H lineitem/orders ratio)
* chain : A {key = shuffled 1..Na, date U[0,2406]},
          B {key = shuffled 1..Nb, segment U[0,4]},
          fact {a_fk U[1,Na], b_fk Zipf_s over 1..Nb, date U[0,2406],
                price int64 U[90000,10500000], discount U[0,10]}

Every column has its own splitmix64 stream, seeded from
(workload id, table, column, fragment); draws are counter based, so a row range
of a column (a streamed chunk) equals the same rows of the whole column.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libpystgen.so")

SEED_BASE = 0x5059535400000000
DATE_MAX = 2406
PRICE_LO, PRICE_HI = 90_000, 10_500_000
SEGMENTS = 5
DISCOUNT_MAX = 10

_lib = None


def build(force: bool = False) -> str:
    """Compile gen.c into libpystgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        # libgomp reads this when it loads; an unset value can oversubscribe a container
        os.environ.setdefault("OMP_NUM_THREADS", str(max(1, min(16, len(os.sched_getaffinity(0))))))
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, u64, p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        lib.gen_draw.argtypes = [u64, u64]
        lib.gen_draw.restype = u64
        lib.gen_uniform_i32.argtypes = [p, i64, i64, i64, u64, i64]
        lib.gen_uniform_i64.argtypes = [p, i64, i64, i64, u64, i64]
        lib.gen_perm_i32.argtypes = [p, i64, i64, u64]
        lib.gen_zipf_i32.argtypes = [p, i64, i64, ctypes.c_double, u64, i64]
        lib.gen_zipf_i32.restype = ctypes.c_int
        lib.gen_loguniform_i64.argtypes = [p, i64, ctypes.c_double, ctypes.c_double, u64]
        lib.gen_poisson_arrivals.argtypes = [p, i64, ctypes.c_double, u64]
        for f in ("gen_uniform_i32", "gen_uniform_i64", "gen_perm_i32",
                  "gen_loguniform_i64", "gen_poisson_arrivals"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def seed(workload: int, table: int, column: int, fragment: int = 0) -> int:
    """Stream seed for one column: base ^ workload<<40 ^ table<<32 ^ column<<24 ^ fragment."""
    return (SEED_BASE ^ (workload << 40) ^ (table << 32) ^ (column << 24) ^ fragment) & (2**64 - 1)


def _out(out, n, dtype):
    if out is None:
        return np.empty(n, dtype=dtype)
    assert out.dtype == dtype and out.shape == (n,) and out.flags["C_CONTIGUOUS"]
    return out


def draw(s: int, i: int) -> int:
    return int(_load().gen_draw(s, i))


def uniform_i32(n, lo, hi, s, offset=0, out=None):
    a = _out(out, n, np.int32)
    _load().gen_uniform_i32(a.ctypes.data, n, lo, hi, s, offset)
    return a


def uniform_i64(n, lo, hi, s, offset=0, out=None):
    a = _out(out, n, np.int64)
    _load().gen_uniform_i64(a.ctypes.data, n, lo, hi, s, offset)
    return a


def perm_i32(n, base, s, out=None):
    a = _out(out, n, np.int32)
    _load().gen_perm_i32(a.ctypes.data, n, base, s)
    return a


def zipf_i32(n, nkeys, zs, s, offset=0, out=None):
    a = _out(out, n, np.int32)
    if _load().gen_zipf_i32(a.ctypes.data, n, nkeys, float(zs), s, offset) != 0:
        raise MemoryError("zipf cdf")
    return a


def loguniform_i64(n, lo, hi, s):
    a = np.empty(n, dtype=np.int64)
    _load().gen_loguniform_i64(a.ctypes.data, n, float(lo), float(hi), s)
    return a


def poisson_arrivals(n, lam, s):
    a = np.empty(n, dtype=np.float64)
    _load().gen_poisson_arrivals(a.ctypes.data, n, float(lam), s)
    return a


# ----------------------------------------------------------------------------------------
# Workload recipes
# ----------------------------------------------------------------------------------------

def star_build(n_build: int, workload: int = 0, fragment: int = 0, out=None):
    """Build (dimension) table of the star query: key = shuffled 1..Nb, segment U[0,4]."""
    out = out or {}
    return {
        "key": perm_i32(n_build, 1, seed(workload, 0, 0, fragment), out=out.get("key")),
        "segment": uniform_i32(n_build, 0, SEGMENTS - 1, seed(workload, 0, 1, fragment),
                               out=out.get("segment")),
    }


def star_probe(n_probe: int, n_build: int, workload: int = 0, fragment: int = 0,
               offset: int = 0, out=None):
    """Probe (fact) table of the star query: fk U[1,Nb], date U[0,2406], price U[90000,10500000]."""
    out = out or {}
    return {
        "fk": uniform_i32(n_probe, 1, n_build, seed(workload, 1, 0, fragment), offset, out.get("fk")),
        "date": uniform_i32(n_probe, 0, DATE_MAX, seed(workload, 1, 1, fragment), offset,
                            out.get("date")),
        "price": uniform_i64(n_probe, PRICE_LO, PRICE_HI, seed(workload, 1, 2, fragment), offset,
                             out.get("price")),
    }


def star_tables(n_build: int, n_probe: int, workload: int = 0, fragment: int = 0):
    return star_build(n_build, workload, fragment), star_probe(n_probe, n_build, workload, fragment)


def chain_dims(n_a: int, n_b: int, workload: int = 2):
    a = {"key": perm_i32(n_a, 1, seed(workload, 0, 0)),
         "date": uniform_i32(n_a, 0, DATE_MAX, seed(workload, 0, 1))}
    b = {"key": perm_i32(n_b, 1, seed(workload, 1, 0)),
         "segment": uniform_i32(n_b, 0, SEGMENTS - 1, seed(workload, 1, 1))}
    return a, b


def chain_fact(n_fact: int, n_a: int, n_b: int, zipf_s: float, workload: int = 2,
               offset: int = 0, out=None):
    out = out or {}
    return {
        "a_fk": uniform_i32(n_fact, 1, n_a, seed(workload, 2, 0), offset, out.get("a_fk")),
        "b_fk": zipf_i32(n_fact, n_b, zipf_s, seed(workload, 2, 1), offset, out.get("b_fk")),
        "date": uniform_i32(n_fact, 0, DATE_MAX, seed(workload, 2, 2), offset, out.get("date")),
        "price": uniform_i64(n_fact, PRICE_LO, PRICE_HI, seed(workload, 2, 3), offset,
                             out.get("price")),
        "discount": uniform_i32(n_fact, 0, DISCOUNT_MAX, seed(workload, 2, 4), offset,
                                out.get("discount")),
    }


JOIN_WORKLOAD = 6
PAYLOAD_BOUND = 1 << 62


def join_tables(n_build: int, n_probe: int, k: int, workload: int = JOIN_WORKLOAD):
    """Tables of the join microbenchmark: unique build keys 1..Nb (shuffled), probe keys
    uniform over 1..2Nb (hit ratio 0.5), and k 8-byte payload columns on each side."""
    b = {"key": perm_i32(n_build, 1, seed(workload, 0, 0))}
    p = {"key": uniform_i32(n_probe, 1, 2 * max(n_build, 1), seed(workload, 1, 0))}
    for c in range(k):
        b["c%d" % c] = uniform_i64(n_build, -PAYLOAD_BOUND, PAYLOAD_BOUND, seed(workload, 0, 1 + c))
        p["c%d" % c] = uniform_i64(n_probe, -PAYLOAD_BOUND, PAYLOAD_BOUND, seed(workload, 1, 1 + c))
    return b, p


JOIN_DUP_WORKLOAD = 8


def join_tables_dup(n_build: int, n_probe: int, k: int, n_keys: int, zipf_s: float = 0.0,
                    workload: int = JOIN_DUP_WORKLOAD):
    """Tables of the many-to-many join: build keys drawn Zipf_s over 1..n_keys (s = 0:
    uniform, so each key appears about n_build / n_keys times), probe keys uniform over
    1..2 n_keys (half of them hit a key that occurs), k 8-byte payload columns a side."""
    b = {"key": zipf_i32(n_build, max(n_keys, 1), zipf_s, seed(workload, 0, 0))}
    p = {"key": uniform_i32(n_probe, 1, 2 * max(n_keys, 1), seed(workload, 1, 0))}
    for c in range(k):
        b["c%d" % c] = uniform_i64(n_build, -PAYLOAD_BOUND, PAYLOAD_BOUND, seed(workload, 0, 1 + c))
        p["c%d" % c] = uniform_i64(n_probe, -PAYLOAD_BOUND, PAYLOAD_BOUND, seed(workload, 1, 1 + c))
    return b, p


Q18_WORKLOAD = 7
QUANTITY_MAX = 50


def q18_lineitem(n_rows: int, n_orders: int, workload: int = Q18_WORKLOAD):
    """Rows of a group-by with many more groups than the caches hold: orderkey U[1,No] int32,
    quantity U[1,50] int32."""
    return {"orderkey": uniform_i32(n_rows, 1, n_orders, seed(workload, 0, 0)),
            "quantity": uniform_i32(n_rows, 1, QUANTITY_MAX, seed(workload, 0, 1))}


def fragment_sizes(n_frag: int, lo: float = 1e4, hi: float = 2e7, workload: int = 3):
    """Probe sizes log-uniform in [lo, hi]; build sizes = probe // 10."""
    p = loguniform_i64(n_frag, lo, hi, seed(workload, 7, 0))
    return p, p // 10
