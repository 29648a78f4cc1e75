"""CPU-side checks of the C ABI: the library loads, exports every function that
include/*.h declares, and its host-side argument checks answer without a GPU."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2512_02862_amd", "libpyst.so")


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(pyst_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2512_02862_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ["pyst_filter", "pyst_partition", "pyst_join_build", "pyst_join_probe", "pyst_groupby_sum",
                 "pyst_query", "pyst_ctx_create", "pyst_ctx_check"]:
        assert must in names


def test_library_exports_every_declared_function(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_binding_signatures_cover_the_exports():
    from paper_2512_02862_amd import pyst
    assert set(pyst.EXPORTS) <= set(_declared_functions())


def test_null_arguments_are_rejected_synchronously(lib):
    lib.pyst_filter.restype = ctypes.c_int
    lib.pyst_filter.argtypes = [ctypes.c_void_p] * 8
    assert lib.pyst_filter(None, None, 0, None, 0, None, None, None) == 1  # PYST_ERR_ARG
    lib.pyst_ctx_create.restype = ctypes.c_int
    lib.pyst_ctx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p]
    assert lib.pyst_ctx_create(0, 1 << 20, None) == 1
    lib.pyst_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.pyst_last_error()


def test_context_creation_without_a_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib.pyst_ctx_create.restype = ctypes.c_int
    lib.pyst_ctx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    st = lib.pyst_ctx_create(0, 1 << 20, ctypes.byref(h))
    assert st != 0 and not h.value


def test_new_entry_points_reject_bad_arguments_synchronously(lib):
    from paper_2512_02862_amd import pyst
    pyst.load(LIB)
    L = pyst._lib
    assert L.pyst_gather(None, None, None, 0, None, 1, None, None) == pyst.ERR_ARG
    assert L.pyst_join_materialize(None, None, None, 0, None, None, 0, 0.5, 1, None, None, None, 0, None, None) == \
        pyst.ERR_ARG
    assert L.pyst_pack_words(None) == -1
    bad = pyst.Col(None, 5, pyst.I32, 0)  # data NULL with n > 0
    assert L.pyst_pack_words(ctypes.byref(bad)) == -1
    assert L.pyst_pack_encode(ctypes.byref(bad), None, None) == pyst.ERR_ARG
    assert L.pyst_pack_decode(None, None, None, 0, 10, pyst.I32, None, None) == pyst.ERR_ARG
    assert L.pyst_query_streamed_packed(None, None, None, 0, 1024, 2, None, None, 0, None, None) == pyst.ERR_ARG


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
