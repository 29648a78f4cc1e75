"""Python binding of libpyst: argument marshalling only.

Every step of the relational path runs in the HIP kernels of libpyst.so; this
module converts torch tensors (device memory) and the current torch stream to
the plain pointers and sizes of the C ABI declared in include/pyst.h.  There is
no fallback: if the library is missing or no GPU is visible, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpyst.so")

OK, ERR_ARG, ERR_NOMEM, ERR_HIP, ERR_CAPACITY, ERR_KEY, ERR_TABLE_FULL, ERR_UNSUPPORTED, ERR_DUP_KEY, ERR_INDEX = range(10)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_NOMEM", 3: "ERR_HIP", 4: "ERR_CAPACITY", 5: "ERR_KEY",
                6: "ERR_TABLE_FULL", 7: "ERR_UNSUPPORTED", 8: "ERR_DUP_KEY", 9: "ERR_INDEX"}
CMP = {"==": 0, "!=": 1, "<": 2, "<=": 3, ">": 4, ">=": 5}
I32, I64 = 0, 1
G_NONE, G_JOIN_KEY, G_JOIN_PAYLOAD, G_FACT_COL = 0, 1, 2, 3
V_COL, V_COL_TIMES_C_MINUS = 0, 1
OPT_GENERIC_ONLY = 1
OPT_GROUPBY_HASH_ONLY = 2
OPT_FAIL_FACT_PASS = 3
OPT_HASH_JOIN_ONLY = 4

EXPORTS = [
    "pyst_ctx_create", "pyst_ctx_destroy", "pyst_ctx_check", "pyst_ctx_used", "pyst_ctx_budget",
    "pyst_last_error", "pyst_filter", "pyst_partition", "pyst_join_build", "pyst_join_probe",
    "pyst_gather", "pyst_join_materialize", "pyst_pack_words", "pyst_pack_encode", "pyst_pack_decode",
    "pyst_query_streamed_packed", "pyst_table_info", "pyst_table_destroy", "pyst_groupby_sum", "pyst_query", "pyst_ctx_timing",
    "pyst_ctx_kernel_time", "pyst_ctx_option", "pyst_query_streamed", "pyst_query_batch", "pyst_autotune",
    "pyst_batch_graph_create", "pyst_batch_graph_launch", "pyst_batch_graph_destroy",
    "pyst_server_create", "pyst_server_create_packed", "pyst_server_submit", "pyst_server_wait", "pyst_server_poll", "pyst_server_get_stats", "pyst_server_check",
    "pyst_server_destroy", "pyst_server_forget_tables", "pyst_server_option", "pyst_partition_noalloc",
    "pyst_device_hbm",
]


class PystError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Col(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class PackBlock(ctypes.Structure):
    _fields_ = [("base", ctypes.c_int64), ("word_off", ctypes.c_int64)]


class PackedCol(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_void_p), ("words", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


PACK_BLOCK = 1024


class Pred(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("cmp", ctypes.c_int32), ("value", ctypes.c_int64)]


class JoinSpec(ctypes.Structure):
    _fields_ = [("key", Col), ("payload", Col), ("cols", ctypes.POINTER(Col)), ("ncols", ctypes.c_int32),
                ("npreds", ctypes.c_int32), ("preds", ctypes.POINTER(Pred)), ("probe_col", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("max_load", ctypes.c_double)]


class Plan(ctypes.Structure):
    _fields_ = [("njoins", ctypes.c_int32), ("npreds", ctypes.c_int32), ("joins", JoinSpec * 2),
                ("preds", ctypes.POINTER(Pred)), ("hi_src", ctypes.c_int32), ("hi_index", ctypes.c_int32),
                ("lo_src", ctypes.c_int32), ("lo_index", ctypes.c_int32), ("vexpr", ctypes.c_int32),
                ("v0", ctypes.c_int32), ("v1", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("vconst", ctypes.c_int64), ("max_groups", ctypes.c_int64), ("group_max_load", ctypes.c_double)]


class Fragment(ctypes.Structure):
    _fields_ = [("plan", ctypes.POINTER(Plan)), ("fact", ctypes.POINTER(Col)), ("nfact", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("out_keys", ctypes.c_void_p), ("out_sums", ctypes.c_void_p),
                ("out_cap", ctypes.c_int64), ("d_ngroups", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("fanout", ctypes.c_int32), ("block", ctypes.c_int32), ("max_load", ctypes.c_double)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32), ("nbuf", ctypes.c_int32),
                ("chunk_rows", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("plan", ctypes.POINTER(Plan)), ("rows", ctypes.c_int64), ("out_keys", ctypes.c_void_p),
                ("out_sums", ctypes.c_void_p), ("out_cap", ctypes.c_int64), ("d_ngroups", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("chunks_copied", ctypes.c_int64),
                ("admission_waits", ctypes.c_int64), ("max_active_seen", ctypes.c_int64),
                ("bytes_copied", ctypes.c_double), ("fact_rows_processed", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libpyst.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libpyst.so is not built: run __graft_entry__.build() or "
                           "python -m paper_2512_02862_amd.build")
    lib = ctypes.CDLL(path)
    p, i32, i64, u32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "pyst_ctx_create": ([i32, sz, P(p)], i32),
        "pyst_ctx_destroy": ([p], None),
        "pyst_ctx_check": ([p, p], i32),
        "pyst_ctx_used": ([p], sz),
        "pyst_ctx_budget": ([p], sz),
        "pyst_last_error": ([], ctypes.c_char_p),
        "pyst_filter": ([p, P(Col), i32, P(Pred), i32, p, p, p], i32),
        "pyst_partition": ([p, P(Col), P(Col), i32, p, p, u32, P(p), p, p], i32),
        "pyst_partition_noalloc": ([P(Col), P(Col), i32, p, p, u32, P(p), p, p], i32),
        "pyst_join_build": ([p, P(Col), P(Col), p, p, ctypes.c_double, i32, P(p), p], i32),
        "pyst_join_probe": ([p, p, P(Col), p, p, p, p, i64, p, p], i32),
        "pyst_gather": ([p, p, p, i64, P(Col), i32, P(p), p], i32),
        "pyst_join_materialize": ([p, P(Col), P(Col), i32, P(Col), P(Col), i32, ctypes.c_double, i32, P(p), p, p, i64,
                                   p, p], i32),
        "pyst_pack_words": ([P(Col)], i64),
        "pyst_pack_encode": ([P(Col), p, p], i32),
        "pyst_pack_decode": ([p, p, p, i64, i64, i32, p, p], i32),
        "pyst_query_streamed_packed": ([p, P(Plan), P(PackedCol), i32, i64, i32, p, p, i64, p, p], i32),
        "pyst_table_info": ([p, p, p], i32),
        "pyst_table_destroy": ([p, p], None),
        "pyst_groupby_sum": ([p, P(Col), P(Col), p, p, i64, ctypes.c_double, p, p, p, i32, p], i32),
        "pyst_query": ([p, P(Plan), P(Col), i32, p, p, i64, p, p], i32),
        "pyst_ctx_timing": ([p, i32], i32),
        "pyst_ctx_option": ([p, i32, i64], i32),
        "pyst_query_streamed": ([p, P(Plan), P(Col), i32, i64, i32, p, p, i64, p, p], i32),
        "pyst_query_batch": ([p, P(Fragment), i32, P(Tuning), p], i32),
        "pyst_autotune": ([p, P(Fragment), i32, i32, P(Tuning), P(ctypes.c_double)], i32),
        "pyst_batch_graph_create": ([p, P(Fragment), i32, P(Tuning), p, P(ctypes.c_void_p)], i32),
        "pyst_batch_graph_launch": ([p, p], i32),
        "pyst_batch_graph_destroy": ([p], i32),
        "pyst_server_create": ([i32, P(ServerCfg), P(Col), i32, P(p)], i32),
        "pyst_server_create_packed": ([i32, P(ServerCfg), P(PackedCol), i32, P(p)], i32),
        "pyst_server_submit": ([p, P(Request), P(ctypes.c_uint64)], i32),
        "pyst_server_wait": ([p, ctypes.c_uint64, P(ctypes.c_double)], i32),
        "pyst_server_poll": ([p, ctypes.c_uint64, P(ctypes.c_int), P(ctypes.c_double)], i32),
        "pyst_server_get_stats": ([p, P(ServerStats)], i32),
        "pyst_server_check": ([p], i32),
        "pyst_server_destroy": ([p], None),
        "pyst_server_forget_tables": ([p, p], i32),
        "pyst_server_option": ([p, i32, i64], i32),
        "pyst_ctx_kernel_time": ([p, ctypes.c_char_p, P(ctypes.c_double), P(i64)], i32),
        "pyst_device_hbm": ([i32, P(i64), P(i32), P(ctypes.c_double)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def device_hbm(device=0):
    """(memory clock kHz, bus width bits, implied HBM peak GB/s) from the device's properties."""
    lib = load()
    clk, bits, peak = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_double()
    _check(lib.pyst_device_hbm(int(device), ctypes.byref(clk), ctypes.byref(bits), ctypes.byref(peak)))
    return clk.value, bits.value, peak.value


def _check(status):
    if status != OK:
        raise PystError(status, _lib.pyst_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _sel_ptr(t):
    """Selection vector pointer; an empty selection still needs a valid address."""
    if t is None:
        return None
    if t.numel() == 0:
        if t.device not in _EMPTY_SEL:
            _EMPTY_SEL[t.device] = torch.zeros(1, dtype=torch.int32, device=t.device)
        t = _EMPTY_SEL[t.device]
    return ctypes.c_void_p(t.data_ptr())


_EMPTY_SEL = {}


def col(t: torch.Tensor) -> Col:
    if not t.is_cuda or not t.is_contiguous() or t.dtype not in (torch.int32, torch.int64):
        raise ValueError("columns are contiguous int32/int64 device tensors")
    return Col(t.data_ptr(), t.numel(), I64 if t.dtype == torch.int64 else I32, 0)


def _null_col():
    return Col(None, 0, I32, 0)


def _preds(preds):
    preds = list(preds or [])
    arr = (Pred * max(1, len(preds)))(*[Pred(c, CMP[o], int(v)) for c, o, v in preds])
    return arr, len(preds)


class Ctx:
    """A device context with a fixed device-memory arena (the budget)."""

    def __init__(self, device: int = 0, budget: int = 1 << 30):
        load()
        self.device = device
        h = ctypes.c_void_p()
        _check(_lib.pyst_ctx_create(device, budget, ctypes.byref(h)))
        self.h = h

    def check(self, stream=None):
        """Synchronize the stream and raise on any error latched by a kernel."""
        _check(_lib.pyst_ctx_check(self.h, _stream(stream)))

    def generic_only(self, enable: bool):
        """Force pyst_query's generic fact pass (no plan-shape-specialized kernel)."""
        _check(_lib.pyst_ctx_option(self.h, OPT_GENERIC_ONLY, int(bool(enable))))

    def groupby_hash_only(self, enable: bool):
        _check(_lib.pyst_ctx_option(self.h, OPT_GROUPBY_HASH_ONLY, int(bool(enable))))

    def hash_join_only(self, enable: bool):
        """Keep pyst_query's join tables hash tables (no direct addressing of dense keys)."""
        _check(_lib.pyst_ctx_option(self.h, OPT_HASH_JOIN_ONLY, int(bool(enable))))

    def timing(self, enable: bool):
        """Record HIP events around the library's timed kernels (see kernel_time)."""
        _check(_lib.pyst_ctx_timing(self.h, int(bool(enable))))

    def kernel_time(self, name: str):
        """(total milliseconds, launches) of the timed region `name` since the last read."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(_lib.pyst_ctx_kernel_time(self.h, name.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    @property
    def used(self):
        return _lib.pyst_ctx_used(self.h)

    @property
    def budget(self):
        return _lib.pyst_ctx_budget(self.h)

    def close(self):
        if self.h:
            _lib.pyst_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev(ctx):
    return torch.device("cuda", ctx.device)


def filter(ctx: Ctx, cols, preds, stream=None):
    """Ascending selection vector (int32, capacity n) and device count (int64[1])."""
    cols = list(cols)
    n = cols[0].numel()
    carr = (Col * len(cols))(*[col(c) for c in cols])
    parr, npred = _preds(preds)
    sel = torch.empty(max(n, 1), dtype=torch.int32, device=_dev(ctx))
    nsel = torch.empty(1, dtype=torch.int64, device=_dev(ctx))
    _check(_lib.pyst_filter(ctx.h, carr, len(cols), parr, npred, _sel_ptr(sel), _ptr(nsel), _stream(stream)))
    return sel, nsel


def partition(ctx: Ctx, key, payloads, fanout: int, sel=None, nsel=None, stream=None):
    """Stable hash partition: (out_key, [out_payloads], offsets int64[F+1])."""
    payloads = list(payloads)
    n = key.numel()
    outs = [torch.empty(max(n, 1), dtype=t.dtype, device=_dev(ctx)) for t in [key] + payloads]
    offsets = torch.empty(fanout + 1, dtype=torch.int64, device=_dev(ctx))
    kc = col(key)
    parr = (Col * max(1, len(payloads)))(*[col(t) for t in payloads])
    oarr = (ctypes.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
    _check(_lib.pyst_partition(ctx.h, ctypes.byref(kc), parr, len(payloads), _sel_ptr(sel), _ptr(nsel), fanout, oarr,
                               _ptr(offsets), _stream(stream)))
    return outs[0][:n], [o[:n] for o in outs[1:]], offsets


def partition_noalloc(key, payloads, fanout: int, outs, offsets, sel=None, nsel=None, stream=None):
    """pyst_partition_noalloc: the stable hash partition into caller-provided
    outputs (outs = [key out] + payload outs, each with room for key.numel()
    values; offsets int64[F+1]), with no context and no device allocation."""
    payloads = list(payloads)
    if len(outs) != 1 + len(payloads):
        raise ValueError("one output per key and payload column")
    kc = col(key)
    parr = (Col * max(1, len(payloads)))(*[col(t) for t in payloads])
    oarr = (ctypes.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
    _check(_lib.pyst_partition_noalloc(ctypes.byref(kc), parr, len(payloads), _sel_ptr(sel), _ptr(nsel), fanout,
                                       oarr, _ptr(offsets), _stream(stream)))


class Table:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def info(self, stream=None):
        """(effective capacity, rows offered for insertion), read from the device."""
        out = torch.empty(2, dtype=torch.int64, device=_dev(self.ctx))
        _check(_lib.pyst_table_info(self.h, _ptr(out), _stream(stream)))
        return tuple(int(x) for x in out.cpu())

    def destroy(self, stream=None):
        if self.h:
            _lib.pyst_table_destroy(self.h, _stream(stream))
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def join_build(ctx: Ctx, key, payload=None, sel=None, nsel=None, max_load=0.5, unique_keys=True, stream=None):
    kc = col(key)
    pc = col(payload) if payload is not None else None
    h = ctypes.c_void_p()
    _check(_lib.pyst_join_build(ctx.h, ctypes.byref(kc), ctypes.byref(pc) if pc is not None else None,
                                _sel_ptr(sel), _ptr(nsel), float(max_load), int(bool(unique_keys)), ctypes.byref(h),
                                _stream(stream)))
    return Table(ctx, h)


def join_probe(ctx: Ctx, table: Table, key, sel=None, nsel=None, out_cap=None, stream=None):
    """(probe rows int32, payloads int64, count int64[1]); outputs have out_cap entries."""
    n = key.numel()
    cap = n if out_cap is None else out_cap
    rows = torch.empty(max(cap, 1), dtype=torch.int32, device=_dev(ctx))
    pays = torch.empty(max(cap, 1), dtype=torch.int64, device=_dev(ctx))
    nout = torch.empty(1, dtype=torch.int64, device=_dev(ctx))
    kc = col(key)
    _check(_lib.pyst_join_probe(ctx.h, table.h, ctypes.byref(kc), _sel_ptr(sel), _ptr(nsel), _ptr(rows), _ptr(pays),
                                cap, _ptr(nout), _stream(stream)))
    return rows, pays, nout


def gather(ctx: Ctx, idx, cols, n=None, stream=None):
    """[col[idx[i]] for i < min(n, len(idx))] for each column: outputs of len(idx) entries.
    n: device int64[1] count of valid entries of idx, or None for all of them."""
    cols = list(cols)
    cap = idx.numel()
    outs = [torch.empty(max(cap, 1), dtype=c.dtype, device=_dev(ctx)) for c in cols]
    carr = (Col * len(cols))(*[col(c) for c in cols])
    oarr = (ctypes.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
    _check(_lib.pyst_gather(ctx.h, _ptr(idx) if cap > 0 else None, _ptr(n), cap, carr, len(cols), oarr,
                            _stream(stream)))
    return [o[:cap] for o in outs]


def join_materialize(ctx: Ctx, build_key, build_cols, probe_key, probe_cols, max_load=0.5, out_cap=None,
                     stream=None, unique_keys=True):
    """(probe rows int32, build rows int32, [probe columns..., build columns...], count int64[1]) of the
    equi-join, in ascending probe row; outputs have out_cap (default: probe rows) entries.  With
    unique_keys=False duplicate build keys are joined many-to-many (pass an out_cap that holds them)."""
    build_cols, probe_cols = list(build_cols), list(probe_cols)
    cap = probe_key.numel() if out_cap is None else out_cap
    d = _dev(ctx)
    prow = torch.empty(max(cap, 1), dtype=torch.int32, device=d)
    brow = torch.empty(max(cap, 1), dtype=torch.int32, device=d)
    outs = [torch.empty(max(cap, 1), dtype=c.dtype, device=d) for c in probe_cols + build_cols]
    nout = torch.empty(1, dtype=torch.int64, device=d)
    bk, pk = col(build_key), col(probe_key)
    barr = (Col * max(1, len(build_cols)))(*[col(c) for c in build_cols])
    parr = (Col * max(1, len(probe_cols)))(*[col(c) for c in probe_cols])
    oarr = (ctypes.c_void_p * max(1, len(outs)))(*[t.data_ptr() for t in outs])
    _check(_lib.pyst_join_materialize(ctx.h, ctypes.byref(bk), barr, len(build_cols), ctypes.byref(pk), parr,
                                      len(probe_cols), float(max_load), int(bool(unique_keys)), oarr, _ptr(prow),
                                      _ptr(brow), cap, _ptr(nout), _stream(stream)))
    return prow[:cap], brow[:cap], [o[:cap] for o in outs], nout


def groupby_sum(ctx: Ctx, key, val, sel=None, nsel=None, max_groups=0, max_load=0.5, sort_by_key=False,
                stream=None):
    """(keys int64, sums int64, count int64[1]); outputs have max_groups (or n) entries."""
    n = key.numel()
    cap = max_groups if max_groups > 0 else n
    ok = torch.empty(max(cap, 1), dtype=torch.int64, device=_dev(ctx))
    osum = torch.empty(max(cap, 1), dtype=torch.int64, device=_dev(ctx))
    ng = torch.empty(1, dtype=torch.int64, device=_dev(ctx))
    kc, vc = col(key), col(val)
    _check(_lib.pyst_groupby_sum(ctx.h, ctypes.byref(kc), ctypes.byref(vc), _sel_ptr(sel), _ptr(nsel), int(max_groups),
                                 float(max_load), _ptr(ok), _ptr(osum), _ptr(ng), int(bool(sort_by_key)),
                                 _stream(stream)))
    return ok, osum, ng


_GSRC = {None: G_NONE, "join_key": G_JOIN_KEY, "join_payload": G_JOIN_PAYLOAD, "fact": G_FACT_COL}


class QueryPlan:
    """A fused query plan (see pyst_plan in include/pyst.h).

    joins: list of dicts {key, payload (or None), cols (list), preds, probe_col, max_load}
    preds: fact predicates [(fact column index, op, constant)]
    hi, lo: group-key halves, each None or (source, index) with source in
            'join_key' | 'join_payload' | 'fact'
    value: ('col', c) or ('col_times_c_minus', c0, c1, const)
    """

    def __init__(self, joins, preds, lo, hi=None, value=("col", 2), max_groups=0, group_max_load=0.5):
        self.joins, self.preds, self.lo, self.hi = joins, preds, lo, hi
        self.value, self.max_groups, self.group_max_load = value, max_groups, group_max_load

    def to_c(self):
        keep = []
        p = Plan()
        p.njoins = len(self.joins)
        parr, npred = _preds(self.preds)
        keep.append(parr)
        p.preds = ctypes.cast(parr, ctypes.POINTER(Pred))
        p.npreds = npred
        for j, js in enumerate(self.joins):
            s = p.joins[j]
            s.key = col(js["key"])
            s.payload = col(js["payload"]) if js.get("payload") is not None else _null_col()
            dcols = list(js.get("cols", []))
            carr = (Col * max(1, len(dcols)))(*[col(t) for t in dcols])
            dp, ndp = _preds(js.get("preds", []))
            keep += [carr, dp]
            s.cols = ctypes.cast(carr, ctypes.POINTER(Col))
            s.ncols = len(dcols)
            s.preds = ctypes.cast(dp, ctypes.POINTER(Pred))
            s.npreds = ndp
            s.probe_col = js["probe_col"]
            s.max_load = float(js.get("max_load", 0.5))
        p.lo_src, p.lo_index = (_GSRC[self.lo[0]], self.lo[1])
        p.hi_src, p.hi_index = (G_NONE, 0) if self.hi is None else (_GSRC[self.hi[0]], self.hi[1])
        if self.value[0] == "col":
            p.vexpr, p.v0, p.v1, p.vconst = V_COL, self.value[1], 0, 0
        else:
            p.vexpr, p.v0, p.v1, p.vconst = V_COL_TIMES_C_MINUS, self.value[1], self.value[2], self.value[3]
        p.max_groups = int(self.max_groups)
        p.group_max_load = float(self.group_max_load)
        return p, keep


def query(ctx: Ctx, plan: QueryPlan, fact, out_cap=None, stream=None):
    """Fused filter + join + group-by: (keys int64, sums int64, count int64[1])."""
    fact = list(fact)
    cp, keep = plan.to_c()
    if out_cap is None:
        out_cap = plan.joins[0]["key"].numel() if plan.hi is None and plan.lo == ("join_key", 0) \
            and len(plan.joins) == 1 else fact[0].numel()
    ok = torch.empty(max(out_cap, 1), dtype=torch.int64, device=_dev(ctx))
    osum = torch.empty(max(out_cap, 1), dtype=torch.int64, device=_dev(ctx))
    ng = torch.empty(1, dtype=torch.int64, device=_dev(ctx))
    farr = (Col * len(fact))(*[col(t) for t in fact])
    _check(_lib.pyst_query(ctx.h, ctypes.byref(cp), farr, len(fact), _ptr(ok), _ptr(osum), int(out_cap), _ptr(ng),
                           _stream(stream)))
    del keep
    return ok, osum, ng


def host_col(t: torch.Tensor) -> Col:
    if t.is_cuda or not t.is_contiguous() or t.dtype not in (torch.int32, torch.int64):
        raise ValueError("streamed fact columns are contiguous int32/int64 host tensors")
    if not t.is_pinned():
        raise ValueError("streamed fact columns must be in pinned host memory")
    return Col(t.data_ptr(), t.numel(), I64 if t.dtype == torch.int64 else I32, 0)


def query_streamed(ctx: Ctx, plan: QueryPlan, host_fact, chunk_rows: int, nbuf: int = 2, out_cap=None,
                   stream=None):
    """pyst_query over pinned host fact columns, streamed in chunks: (keys, sums, count int64[1])."""
    host_fact = list(host_fact)
    cp, keep = plan.to_c()
    if out_cap is None:
        out_cap = plan.joins[0]["key"].numel() if plan.hi is None and plan.lo == ("join_key", 0) \
            and len(plan.joins) == 1 else max(plan.max_groups, 1)
    ok = torch.empty(max(out_cap, 1), dtype=torch.int64, device=_dev(ctx))
    osum = torch.empty(max(out_cap, 1), dtype=torch.int64, device=_dev(ctx))
    ng = torch.empty(1, dtype=torch.int64, device=_dev(ctx))
    farr = (Col * len(host_fact))(*[host_col(t) for t in host_fact])
    _check(_lib.pyst_query_streamed(ctx.h, ctypes.byref(cp), farr, len(host_fact), int(chunk_rows), int(nbuf),
                                    _ptr(ok), _ptr(osum), int(out_cap), _ptr(ng), _stream(stream)))
    del keep
    return ok, osum, ng


def pack(t: torch.Tensor, pinned: bool = True):
    """Bit-pack a contiguous int32/int64 host tensor: (blocks int64[nblocks + 1, 2] = (base, word_off),
    words int32[...] holding the 32-bit words), in pinned host memory unless pinned=False."""
    if t.is_cuda or not t.is_contiguous() or t.dtype not in (torch.int32, torch.int64):
        raise ValueError("pack takes a contiguous int32/int64 host tensor")
    c = Col(t.data_ptr(), t.numel(), I64 if t.dtype == torch.int64 else I32, 0)
    nw = _lib.pyst_pack_words(ctypes.byref(c))
    if nw < 0:
        raise PystError(ERR_ARG, "pyst_pack_words: bad column")
    nblk = (t.numel() + PACK_BLOCK - 1) // PACK_BLOCK
    blocks = torch.empty((nblk + 1, 2), dtype=torch.int64, pin_memory=pinned)
    words = torch.empty(max(nw, 1), dtype=torch.int32, pin_memory=pinned)
    _check(_lib.pyst_pack_encode(ctypes.byref(c), blocks.data_ptr(), words.data_ptr()))
    return blocks, words[:nw]


def packed_col(blocks: torch.Tensor, words: torch.Tensor, n: int, dtype) -> PackedCol:
    return PackedCol(blocks.data_ptr(), words.data_ptr() if words.numel() else blocks.data_ptr(), n,
                     I64 if dtype == torch.int64 else I32, 0)


def unpack(ctx: Ctx, blocks: torch.Tensor, words: torch.Tensor, n: int, dtype, stream=None):
    """Decode a packed column held in device tensors into a new device column of n values."""
    out = torch.empty(max(n, 1), dtype=dtype, device=_dev(ctx))
    _check(_lib.pyst_pack_decode(ctx.h, _ptr(blocks), _ptr(words) if words.numel() else None, words.numel(), n,
                                 I64 if dtype == torch.int64 else I32, _ptr(out), _stream(stream)))
    return out[:n]


def query_streamed_packed(ctx: Ctx, plan: QueryPlan, packed, chunk_rows: int, nbuf: int = 2, out_cap=None,
                          stream=None):
    """query_streamed over packed pinned host columns: packed = [(blocks, words, n, dtype), ...]."""
    packed = list(packed)
    cp, keep = plan.to_c()
    if out_cap is None:
        out_cap = plan.joins[0]["key"].numel() if plan.hi is None and plan.lo == ("join_key", 0) \
            and len(plan.joins) == 1 else max(plan.max_groups, 1)
    ok = torch.empty(max(out_cap, 1), dtype=torch.int64, device=_dev(ctx))
    osum = torch.empty(max(out_cap, 1), dtype=torch.int64, device=_dev(ctx))
    ng = torch.empty(1, dtype=torch.int64, device=_dev(ctx))
    farr = (PackedCol * len(packed))(*[packed_col(*x) for x in packed])
    _check(_lib.pyst_query_streamed_packed(ctx.h, ctypes.byref(cp), farr, len(packed), int(chunk_rows), int(nbuf),
                                           _ptr(ok), _ptr(osum), int(out_cap), _ptr(ng), _stream(stream)))
    del keep
    return ok, osum, ng


class Batch:
    """A batch of independent star fragments with preallocated outputs.

    fragments: list of (plan, fact columns); outputs get the dimension's row
    count as capacity.  run() enqueues pyst_query_batch; results() reads back.
    """

    def __init__(self, ctx: Ctx, fragments):
        self.ctx = ctx
        self._keep = []
        n = len(fragments)
        self.arr = (Fragment * max(n, 1))()
        self.outs = []
        for i, (plan, fact) in enumerate(fragments):
            cp, keep = plan.to_c()
            cp = ctypes.pointer(cp)
            farr = (Col * len(fact))(*[col(t) for t in fact])
            cap = plan.joins[0]["key"].numel()
            ok = torch.empty(max(cap, 1), dtype=torch.int64, device=_dev(ctx))
            osum = torch.empty(max(cap, 1), dtype=torch.int64, device=_dev(ctx))
            ng = torch.empty(1, dtype=torch.int64, device=_dev(ctx))
            self._keep += [cp, keep, farr, fact]
            self.outs.append((ok, osum, ng))
            self.arr[i] = Fragment(cp, ctypes.cast(farr, ctypes.POINTER(Col)), len(fact), 0, ok.data_ptr(),
                                   osum.data_ptr(), cap, ng.data_ptr())
        self.n = n

    def run(self, tuning=None, stream=None):
        t = ctypes.byref(Tuning(*tuning)) if tuning is not None else None
        _check(_lib.pyst_query_batch(self.ctx.h, self.arr, self.n, t, _stream(stream)))

    def autotune(self, reps=2):
        t, ms = Tuning(), ctypes.c_double()
        _check(_lib.pyst_autotune(self.ctx.h, self.arr, self.n, reps, ctypes.byref(t), ctypes.byref(ms)))
        return (t.fanout, t.block, t.max_load), ms.value

    def graph(self, tuning=None, stream=None):
        """Capture this batch as a HIP graph (BatchGraph); results() reads its replays."""
        return BatchGraph(self, tuning, stream)

    def results(self):
        out = []
        for ok, osum, ng in self.outs:
            m = int(ng.item())
            out.append((ok[:m], osum[:m]))
        return out


class BatchGraph:
    """pyst_batch_graph_*: a Batch captured once, replayed with launch()."""

    def __init__(self, batch: Batch, tuning=None, stream=None):
        self.batch = batch
        t = ctypes.byref(Tuning(*tuning)) if tuning is not None else None
        h = ctypes.c_void_p()
        _check(_lib.pyst_batch_graph_create(batch.ctx.h, batch.arr, batch.n, t, _stream(stream), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        _check(_lib.pyst_batch_graph_launch(self.h, _stream(stream)))

    def close(self):
        if self.h:
            _check(_lib.pyst_batch_graph_destroy(self.h))
            self.h = None


class Server:
    """pyst_server: continuous batching over a pinned host fact table.

    submit(plan, rows, out_cap) -> ticket (outputs allocated here);
    wait(ticket) -> (keys, sums, latency_ms).
    """

    def __init__(self, host_fact, budget=4 << 30, max_active=8, nbuf=3, chunk_rows=1 << 24, device=0,
                 packed=None):
        """packed: [(blocks, words, n, dtype), ...] from pack() instead of host_fact (pass host_fact=None)."""
        load()
        self.host_fact = list(host_fact) if host_fact is not None else []
        self.packed = list(packed) if packed is not None else None
        self.device = device
        cfg = ServerCfg(budget, max_active, nbuf, chunk_rows)
        h = ctypes.c_void_p()
        if self.packed is None:
            self._cols = (Col * len(self.host_fact))(*[host_col(t) for t in self.host_fact])
            _check(_lib.pyst_server_create(device, ctypes.byref(cfg), self._cols, len(self.host_fact),
                                           ctypes.byref(h)))
        else:
            self._cols = (PackedCol * len(self.packed))(*[packed_col(*x) for x in self.packed])
            _check(_lib.pyst_server_create_packed(device, ctypes.byref(cfg), self._cols, len(self.packed),
                                                  ctypes.byref(h)))
        self.h = h
        self._live = {}

    def submit(self, plan: QueryPlan, rows: int, out_cap: int):
        cp, keep = plan.to_c()
        d = torch.device("cuda", self.device)
        ok = torch.empty(max(out_cap, 1), dtype=torch.int64, device=d)
        osum = torch.empty(max(out_cap, 1), dtype=torch.int64, device=d)
        ng = torch.empty(1, dtype=torch.int64, device=d)
        req = Request(ctypes.pointer(cp), int(rows), ok.data_ptr(), osum.data_ptr(), int(out_cap), ng.data_ptr())
        t = ctypes.c_uint64()
        _check(_lib.pyst_server_submit(self.h, ctypes.byref(req), ctypes.byref(t)))
        self._live[t.value] = (ok, osum, ng, plan)  # plan holds the dimension tensors alive
        del keep
        return t.value

    def wait(self, ticket):
        lat = ctypes.c_double()
        st = _lib.pyst_server_wait(self.h, ticket, ctypes.byref(lat))
        ok, osum, ng, _ = self._live.pop(ticket)
        _check(st)
        m = int(ng.item())
        return ok[:m], osum[:m], lat.value

    def poll(self, ticket):
        """None while the request runs; then (keys, sums, latency_ms) as wait() returns them."""
        done, lat = ctypes.c_int(), ctypes.c_double()
        st = _lib.pyst_server_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(lat))
        if st == OK and not done.value:
            return None
        ok, osum, ng, _ = self._live.pop(ticket)
        _check(st)
        m = int(ng.item())
        return ok[:m], osum[:m], lat.value

    def forget_tables(self, dim_col=None):
        """Drop the resident tables built over dimension tensor `dim_col` (None: all)."""
        _check(_lib.pyst_server_forget_tables(self.h, None if dim_col is None else ctypes.c_void_p(dim_col.data_ptr())))

    def option(self, key, value):
        _check(_lib.pyst_server_option(self.h, int(key), int(value)))

    def stats(self):
        s = ServerStats()
        _check(_lib.pyst_server_get_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def check(self):
        _check(_lib.pyst_server_check(self.h))

    def close(self):
        if self.h:
            _lib.pyst_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ plans of the measured workloads

def star_plan(build, seg_eq=1, date_lt=1200, max_load=0.5):
    """SELECT key, SUM(price) ... WHERE segment == seg_eq AND date < date_lt GROUP BY key.

    build: {key, segment} device tensors; fact columns are [fk, date, price].
    """
    return QueryPlan(
        joins=[{"key": build["key"], "payload": None, "cols": [build["key"], build["segment"]],
                "preds": [(1, "==", seg_eq)], "probe_col": 0, "max_load": max_load}],
        preds=[(1, "<", date_lt)], lo=("join_key", 0), value=("col", 2))


def fact_star_plan(b, seg_eq=1, date_lt=1200, max_load=0.5):
    """The star query over the chain's fact columns [a_fk, b_fk, date, price, discount]:
    fact JOIN B ON b_fk = B.key WHERE B.segment == seg_eq AND date < date_lt GROUP BY B.key SUM(price)."""
    return QueryPlan(
        joins=[{"key": b["key"], "payload": None, "cols": [b["key"], b["segment"]], "preds": [(1, "==", seg_eq)],
                "probe_col": 1, "max_load": max_load}],
        preds=[(2, "<", date_lt)], lo=("join_key", 0), value=("col", 3))


def chain_plan(a, b, seg_eq=1, date_lt=1200, max_load=0.5, group_max_load=0.5, max_groups=0):
    """Two-join chain: fact JOIN B (filtered) JOIN A, GROUP BY (B.key, A.date) SUM(price*(100-discount)).

    Fact columns are [a_fk, b_fk, date, price, discount]; B is probed first (more selective).
    """
    return QueryPlan(
        joins=[{"key": b["key"], "payload": None, "cols": [b["key"], b["segment"]], "preds": [(1, "==", seg_eq)],
                "probe_col": 1, "max_load": max_load},
               {"key": a["key"], "payload": a["date"], "cols": [], "preds": [], "probe_col": 0,
                "max_load": max_load}],
        preds=[(2, "<", date_lt)], hi=("join_key", 0), lo=("join_payload", 1),
        value=("col_times_c_minus", 3, 4, 100), max_groups=max_groups, group_max_load=group_max_load)
