"""The C-ABI library loads on a CPU-only host and exports every symbol include/ials.h declares.

No compute call is made here; only argument validation that returns before
any device work.
"""
import ctypes as C
import os
import re

import pytest

from paper_2110_14044_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"IALS_API\s+[\w\s\*]+?\b(ials_\w+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libials.so is not built (run __graft_entry__.build())")
    return binding.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(binding.exported_symbols()) | set(names)
    assert set(binding.exported_symbols()) == set(names)


def test_version_string(lib):
    assert "gfx950" in binding.ials_version()


def test_create_rejects_bad_config_before_device_work(lib):
    S = binding.ials_coo(0, None, None, None, None, 0, 0)
    for cfg in [binding.make_config(0, 10, 16, 8, 0.1, 0.1), binding.make_config(10, 10, 16, 0, 0.1, 0.1),
                binding.make_config(10, 10, 16, 32, 0.1, 0.1), binding.make_config(10, 10, 16, 8, 0.1, 0.0),
                binding.make_config(10, 10, 512, 257, 0.1, 0.1), binding.make_config(10, 10, 16, 8, -1.0, 0.1),
                binding.make_config(10, 10, 16, 8, 0.1, 0.1, gram_split=100),
                binding.make_config(10, 10, 16, 8, 0.1, 0.1, gram_split=32),
                binding.make_config(10, 10, 16, 8, 0.1, 0.1, gram_split=4096)]:
        out = C.c_void_p()
        st = lib.ials_create(C.byref(cfg), C.byref(S), 1, 1, None, C.byref(out))
        assert st == binding.IALS_E_INVALID
        assert out.value is None
        assert binding.ials_last_error(None)
    out = C.c_void_p()
    cfg = binding.make_config(10, 10, 16, 8, 0.1, 0.1)
    assert lib.ials_create(None, C.byref(S), 1, 1, None, C.byref(out)) == binding.IALS_E_INVALID
    assert lib.ials_create(C.byref(cfg), C.byref(S), None, 1, None, C.byref(out)) == binding.IALS_E_INVALID
    bad = binding.ials_coo(-1, None, None, None, None, 0, 0)
    assert lib.ials_create(C.byref(cfg), C.byref(bad), 1, 1, None, C.byref(out)) == binding.IALS_E_INVALID


def test_null_context_calls_fail_cleanly(lib):
    assert lib.ials_epoch(None, 1) == binding.IALS_E_INVALID
    assert lib.ials_block_sweep(None, 0, 0) == binding.IALS_E_INVALID
    assert lib.ials_destroy(None) == binding.IALS_E_INVALID
    L = C.c_double()
    assert lib.ials_loss(None, C.byref(L), None) == binding.IALS_E_INVALID


def test_server_create_rejects_bad_config_before_device_work(lib):
    bad = [binding.make_server_config(0, 256, 64, 0.1, 0.05),          # no items
           binding.make_server_config(100, 256, 0, 0.1, 0.05),         # b = 0
           binding.make_server_config(100, 256, 65, 0.1, 0.05),        # b > 64
           binding.make_server_config(100, 16, 32, 0.1, 0.05),         # b > d
           binding.make_server_config(100, 256, 64, 0.1, 0.0),        # lambda = 0
           binding.make_server_config(100, 256, 64, -0.1, 0.05),       # alpha0 < 0
           binding.make_server_config(100, 256, 64, 0.1, 0.05, passes=-1),
           binding.make_server_config(100, 256, 64, 0.1, 0.05, max_slots=0),
           binding.make_server_config(100, 256, 64, 0.1, 0.05, streams=9),
           binding.make_server_config(100, 256, 64, 0.1, 0.05, hbm_budget=1000),
           binding.make_server_config(100, 256, 64, 0.1, 0.05, precision=binding.IALS_PREC_BF16)]
    for cfg in bad:
        out = C.c_void_p()
        assert lib.ials_server_create(C.byref(cfg), 1, C.byref(out)) == binding.IALS_E_INVALID
        assert out.value is None
        assert binding.ials_server_last_error(None)
    cfg = binding.make_server_config(100, 256, 64, 0.1, 0.05)
    out = C.c_void_p()
    assert lib.ials_server_create(C.byref(cfg), None, C.byref(out)) == binding.IALS_E_INVALID


def test_null_server_and_foldin_calls_fail_cleanly(lib):
    n = C.c_int32()
    assert lib.ials_server_submit(None, 0, None, None, 0) == binding.IALS_E_INVALID
    assert lib.ials_server_poll(None, 1, 0, None, None, None, C.byref(n)) == binding.IALS_E_INVALID
    assert lib.ials_server_destroy(None) == binding.IALS_E_INVALID
    assert lib.ials_foldin(None, 0, None, None, None, 3, None) == binding.IALS_E_INVALID


def test_rank_entry_points_reject_bad_arguments_before_device_work(lib):
    E = binding.IALS_E_INVALID
    f = lib.ials_rank_topk
    # d not a multiple of 4, k out of [1, 512], negative sizes, missing pointers, half of an exclusion CSR
    assert f(1, 4, 1, 5, 6, None, None, 3, 1, None, 0, None) == E
    assert f(1, 4, 1, 5, 8, None, None, 0, 1, None, 0, None) == E
    assert f(1, 4, 1, 5, 8, None, None, 513, 1, None, 0, None) == E
    assert f(1, -1, 1, 5, 8, None, None, 3, 1, None, 0, None) == E
    assert f(None, 4, 1, 5, 8, None, None, 3, 1, None, 0, None) == E
    assert f(16, 4, 16, 5, 8, 16, None, 3, 16, None, 0, None) == E
    assert f(3, 4, 16, 5, 8, None, None, 3, 16, None, 0, None) == E  # W not 16-byte aligned
    assert lib.ials_rank_last_error()
    # no users: nothing to do
    assert f(None, 0, None, 5, 8, None, None, 3, None, None, 0, None) == binding.IALS_OK
    g = lib.ials_rank_metrics
    sums = (C.c_double * 2)()
    counts = (C.c_int64 * 2)()
    kinds = (C.c_int32 * 2)(0, 2)  # kind 2 is neither recall nor ndcg
    ks = (C.c_int32 * 2)(5, 5)
    assert g(1, 4, 10, 1, 1, 2, kinds, ks, 1, sums, counts, None) == E
    kinds = (C.c_int32 * 2)(0, 1)
    ks = (C.c_int32 * 2)(5, 11)  # k_m above the list length
    assert g(1, 4, 10, 1, 1, 2, kinds, ks, 1, sums, counts, None) == E
    ks = (C.c_int32 * 2)(5, 10)
    assert g(None, 4, 10, None, None, 2, kinds, ks, None, sums, counts, None) == E
    assert g(None, 0, 10, None, None, 2, kinds, ks, None, sums, counts, None) == binding.IALS_OK
    assert list(sums) == [0.0, 0.0] and list(counts) == [0, 0]
