"""CPU-side checks of the C ABI: the library builds and exports every symbol
that include/mp.h declares; argument errors are rejected before any HIP call."""
import ctypes
import os
import re

import pytest

import paper_1901_05708_amd as mp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mp_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mp.LIB_PATH):
        from paper_1901_05708_amd import build
        build.build()
    return mp.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for f in ("mp_aamp", "mp_pnorm", "mp_acamp", "mp_batch", "mp_strerror", "mp_release"):
        assert f in names
    assert set(mp.EXPORTED) <= set(names)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"libmp.so does not export {name}"


def test_invalid_arguments_rejected_without_gpu(lib):
    vp = ctypes.c_void_p
    dummy = vp(16)   # never dereferenced: validation fails first
    # null pointers
    assert lib.mp_aamp(None, 100, 10, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    # bad m
    assert lib.mp_aamp(dummy, 100, 0, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_aamp(dummy, 100, 101, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    # bad n
    assert lib.mp_acamp(dummy, 0, 1, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_acamp(dummy, 1 << 31, 4, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    # bad precision / R
    assert lib.mp_aamp(dummy, 100, 10, 0, 7, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_aamp(dummy, 100, 10, 0, 0, -1, dummy, dummy, None) == mp.MP_EINVAL
    # bad p
    assert lib.mp_pnorm(dummy, 100, 10, 0.5, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_pnorm(dummy, 100, 10, float("inf"), 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_pnorm(dummy, 100, 10, float("nan"), 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    msg = lib.mp_strerror(mp.MP_EINVAL).decode()
    assert "invalid argument" in msg
    # batch: bad job table
    jobs = (mp.MpJob * 1)()
    jobs[0] = mp.MpJob(0, 100, 0, 10, 9, 0, 0, 2.0)
    assert lib.mp_batch(dummy, jobs, 1, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_batch(None, jobs, 1, 0, dummy, dummy, None) == mp.MP_EINVAL


def test_batch_table_errors_rejected_without_gpu(lib):
    dummy = ctypes.c_void_p(16)
    ok = mp.MpJob(0, 100, 0, 10, mp.KIND_AAMP, 0, 0, 2.0)
    # overlapping output ranges (91 outputs from 0, the second job starts at 50)
    jobs = (mp.MpJob * 2)(ok, mp.MpJob(100, 100, 50, 10, mp.KIND_ACAMP, 0, 0, 2.0))
    assert lib.mp_batch(dummy, jobs, 2, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert "overlap" in lib.mp_strerror(mp.MP_EINVAL).decode()
    # negative offsets, bad m, bad p, too many jobs, bad precision
    for bad in (mp.MpJob(-1, 100, 0, 10, 0, 0, 0, 2.0), mp.MpJob(0, 100, -5, 10, 0, 0, 0, 2.0),
                mp.MpJob(0, 100, 0, 101, 0, 0, 0, 2.0), mp.MpJob(0, 100, 0, 10, 1, 0, 0, 0.9),
                mp.MpJob(0, 100, 0, 10, 0, 0, -2, 2.0)):
        jobs = (mp.MpJob * 1)(bad)
        assert lib.mp_batch(dummy, jobs, 1, 0, dummy, dummy, None) == mp.MP_EINVAL
    jobs = (mp.MpJob * 1)(ok)
    assert lib.mp_batch(dummy, jobs, 65536, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_batch(dummy, jobs, -1, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_batch(dummy, jobs, 1, 3, dummy, dummy, None) == mp.MP_EINVAL
    # an empty batch is a no-op that needs no device
    assert lib.mp_batch(dummy, jobs, 0, 0, dummy, dummy, None) == mp.MP_OK


def test_stats_struct_matches_header():
    src = open(HEADER).read()
    body = src[src.index("typedef struct mp_stats {"):src.index("} mp_stats;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(double|int64_t|int32_t)\s+(\w+);", body)
    assert [f for _, f in fields] == [f for f, _ in mp.MpStats._fields_]
    sizes = {"double": 8, "int64_t": 8, "int32_t": 4}
    assert sum(sizes[t] for t, _ in fields) == ctypes.sizeof(mp.MpStats)


def test_topk_arguments_rejected_without_gpu(lib):
    d = ctypes.c_void_p(16)
    ok = (d, d, 100, 5, 3, mp.MP_MOTIFS, d, d, d, d, None)
    bad = [
        (None,) + ok[1:],                                   # null P
        ok[:2] + (-1,) + ok[3:],                            # N < 0
        ok[:2] + (1 << 31,) + ok[3:],                       # N too large
        ok[:3] + (-1,) + ok[4:],                            # k < 0
        ok[:3] + (65537,) + ok[4:],                         # k too large
        ok[:4] + (0,) + ok[5:],                             # excl < 1
        ok[:5] + (2,) + ok[6:],                             # bad mode
        ok[:9] + (None,) + ok[10:],                         # null count
    ]
    for args in bad:
        assert lib.mp_topk(*args) == mp.MP_EINVAL


def test_incremental_arguments_rejected_without_gpu(lib):
    h = ctypes.c_void_p()
    bad = [
        (0, mp.KIND_AAMP, 2.0, 0, 1000, 0),        # m < 1
        (16, 7, 2.0, 0, 1000, 0),                  # bad kind
        (16, mp.KIND_PNORM, 0.5, 0, 1000, 0),      # p < 1
        (16, mp.KIND_AAMP, 2.0, 0, 8, 0),          # capacity < m
        (16, mp.KIND_AAMP, 2.0, 0, 1 << 31, 0),    # capacity too large
        (16, mp.KIND_AAMP, 2.0, 0, 1000, -1),      # refresh < 0
    ]
    for args in bad:
        assert lib.mp_inc_create(*args, ctypes.byref(h)) == mp.MP_EINVAL
    assert lib.mp_inc_create(16, mp.KIND_AAMP, 2.0, 0, 1000, 0, None) == mp.MP_EINVAL
    assert lib.mp_inc_append(None, ctypes.c_void_p(16), 10, None) == mp.MP_EINVAL
    assert lib.mp_inc_read(None, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == mp.MP_EINVAL
    lib.mp_inc_destroy(None)                       # a no-op


def test_strerror_never_null(lib):
    for code in (0, -1, -2, -3, -4, 12345):
        assert isinstance(lib.mp_strerror(code), bytes)


def test_profile_read_rejects_null(lib):
    assert lib.mp_profile_read(None) == mp.MP_EINVAL
