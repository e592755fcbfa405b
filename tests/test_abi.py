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
    assert lib.mp_aamp(dummy, 100, 10, 0, 3, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_aamp(dummy, 100, 10, 0, 0, -1, dummy, dummy, None) == mp.MP_EINVAL
    # bad p
    assert lib.mp_pnorm(dummy, 100, 10, 0.5, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_pnorm(dummy, 100, 10, float("inf"), 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_pnorm(dummy, 100, 10, float("nan"), 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    # the F comparator variant: the same argument rules
    assert lib.mp_acamp_fcmp(None, 100, 10, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_acamp_fcmp(dummy, 100, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_acamp_fcmp(dummy, 100, 10, 0, -1, dummy, dummy, None) == mp.MP_EINVAL
    msg = lib.mp_strerror(mp.MP_EINVAL).decode()
    assert "invalid argument" in msg
    # the allocation-free variant: the same rules, plus its window limit
    lim = mp.NOALLOC_MAX_N
    assert lib.mp_profile_noalloc(0, None, 100, 10, 2.0, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_profile_noalloc(3, dummy, 100, 10, 2.0, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_profile_noalloc(1, dummy, 100, 10, 0.5, 0, 0, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_profile_noalloc(2, dummy, 100, 10, 2.0, 0, 5, 0, dummy, dummy, None) == mp.MP_EINVAL
    assert lib.mp_profile_noalloc(0, dummy, lim + 64, 64, 2.0, 0, 0, 0, dummy, dummy,
                                  None) == mp.MP_EINVAL
    assert "MP_NOALLOC_MAX_N" in lib.mp_strerror(mp.MP_EINVAL).decode()
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


def test_precision_constants_match_header():
    src = open(os.path.join(ROOT, "include", "mp.h")).read()
    for name in ("MP_FP64", "MP_FP32_REFRESH", "MP_FP32_AUTO"):
        got = re.search(r"#define %s (\d+)" % name, src)
        assert got and int(got.group(1)) == getattr(mp, name), name
    assert mp._prec("fp32_auto") == mp.MP_FP32_AUTO
    with pytest.raises(ValueError):
        mp._prec("fp16")


def test_strerror_never_null(lib):
    for code in (0, -1, -2, -3, -4, 12345):
        assert isinstance(lib.mp_strerror(code), bytes)


def test_profile_read_rejects_null(lib):
    assert lib.mp_profile_read(None) == mp.MP_EINVAL


def test_anytime_arguments_rejected_without_gpu(lib):
    dummy = ctypes.c_void_p(16)
    g = (ctypes.c_int32 * 2)(0, 1)
    n, m = 5000, 32                       # N = 4969, excl 8: 10 groups
    ok = [mp.KIND_AAMP, dummy, n, m, 2.0, 0, g, 2, 0, dummy, dummy, None]

    def call(**kw):
        a = list(ok)
        for k, v in kw.items():
            a[int(k[1:])] = v
        return lib.mp_anytime(*a)

    assert call(a1=None) == mp.MP_EINVAL                          # null T
    assert call(a3=0) == mp.MP_EINVAL                             # m < 1
    assert call(a0=9) == mp.MP_EINVAL                             # bad kind
    assert call(a0=mp.KIND_PNORM, a4=7.0) == mp.MP_EINVAL         # p > 6: no band kernel
    assert call(a7=-1) == mp.MP_EINVAL                            # ngroups < 0
    assert call(a6=None) == mp.MP_EINVAL                          # null groups
    assert call(a8=2) == mp.MP_EINVAL                             # resume not 0 / 1
    bad = (ctypes.c_int32 * 1)(10)
    assert call(a6=bad, a7=1) == mp.MP_EINVAL                     # group past the last
    neg = (ctypes.c_int32 * 1)(-1)
    assert call(a6=neg, a7=1) == mp.MP_EINVAL
    G = ctypes.c_int64()
    assert lib.mp_anytime_groups(n, m, 0, None) == mp.MP_EINVAL
    assert lib.mp_anytime_groups(n, 0, 0, ctypes.byref(G)) == mp.MP_EINVAL
    assert lib.mp_anytime_groups(10, 11, 0, ctypes.byref(G)) == mp.MP_EINVAL
    assert lib.mp_anytime_order(n, m, 0, 1, None, None) == mp.MP_EINVAL


def test_anytime_groups_and_order_on_host(lib):
    """Host-only helpers: the group count, the order is a permutation fixed by
    the seed, and the cumulative pairs count the admissible pairs of each
    prefix (checked by summing N - d over the prefix's diagonals)."""
    import numpy as np
    for n, m, excl in ((5000, 32, 0), (2000, 100, 1), (1100, 64, 0), (700, 64, 700)):
        N = n - m + 1
        e = excl or mp.default_excl(m)
        G = mp.anytime_groups(n, m, excl)
        assert G == (max(N - e, 0) + 511) // 512
        order, cum = mp.anytime_order(n, m, excl, seed=7)
        assert sorted(order.tolist()) == list(range(G))
        o2, c2 = mp.anytime_order(n, m, excl, seed=7)
        assert np.array_equal(order, o2) and np.array_equal(cum, c2)
        if G:
            assert cum[-1] == mp.pair_count(n, m, e)
            want, run = [], 0
            for g in order:
                d = np.arange(e + 512 * g, min(e + 512 * (g + 1), N))
                run += int((N - d).sum())
                want.append(run)
            assert cum.tolist() == want
    # different seeds give different orders; seed 0 is not the identity
    a, _ = mp.anytime_order(200000, 64, 0, seed=1)
    b, _ = mp.anytime_order(200000, 64, 0, seed=2)
    c, _ = mp.anytime_order(200000, 64, 0, seed=0)
    assert not np.array_equal(a, b)
    assert not np.array_equal(c, np.arange(c.size))
    # roughly uniform: each group lands in the first half about half the time
    first = np.zeros(a.size)
    for s in range(200):
        o, _ = mp.anytime_order(200000, 64, 0, seed=100 + s)
        first[o[: o.size // 2]] += 1
    assert 0.35 < first.mean() / 200 < 0.65 and first.min() > 50 and first.max() < 150


def _gpu_visible():
    """Whether a GPU device node exists (checked without initialising HIP)."""
    return os.path.exists("/dev/kfd")


@pytest.mark.skipif(_gpu_visible(), reason="the no-device error path needs a host without a GPU")
def test_hip_error_without_gpu(lib):
    """Valid arguments on a host without a GPU: the first HIP call fails and
    the call returns MP_EHIP with the HIP error text, never crashing."""
    dummy = ctypes.c_void_p(16)
    rc = lib.mp_aamp(dummy, 100, 10, 0, 0, 0, dummy, dummy, None)
    assert rc == mp.MP_EHIP
    msg = lib.mp_strerror(rc).decode()
    assert msg.startswith("HIP runtime error") and "hipGetDevice" in msg
    rc = lib.mp_profile_noalloc(2, dummy, 100, 10, 2.0, 0, 0, 0, dummy, dummy, None)
    assert rc == mp.MP_EHIP
    jobs = (mp.MpJob * 1)(mp.MpJob(0, 100, 0, 10, mp.KIND_AAMP, 0, 0, 2.0))
    assert lib.mp_batch(dummy, jobs, 1, 0, dummy, dummy, None) == mp.MP_EHIP
    h = ctypes.c_void_p()
    assert lib.mp_inc_create(16, mp.KIND_ACAMP, 2.0, 0, 1000, 0, ctypes.byref(h)) == mp.MP_EHIP
    assert h.value is None


def test_allocation_failure_hook(lib, monkeypatch):
    """MP_FAIL_ALLOC=1 makes every device allocation fail as out-of-memory:
    MP_ENOMEM, no handle returned, and the next call without the hook works
    as before (here: reaches the device query again)."""
    monkeypatch.setenv("MP_FAIL_ALLOC", "1")
    h = ctypes.c_void_p()
    rc = lib.mp_inc_create(16, mp.KIND_ACAMP, 2.0, 0, 1000, 0, ctypes.byref(h))
    assert rc == mp.MP_ENOMEM and h.value is None
    assert "incremental profile buffers" in lib.mp_strerror(rc).decode()
    monkeypatch.delenv("MP_FAIL_ALLOC")
    if not _gpu_visible():
        rc = lib.mp_inc_create(16, mp.KIND_ACAMP, 2.0, 0, 1000, 0, ctypes.byref(h))
        assert rc == mp.MP_EHIP and h.value is None


def test_every_error_code_has_a_message(lib):
    for code, word in ((mp.MP_OK, "success"), (mp.MP_EINVAL, "invalid argument"),
                       (mp.MP_ENOMEM, "allocation failed"), (mp.MP_EHIP, "HIP runtime error"),
                       (mp.MP_EUNSUPPORTED, "unsupported device"), (-99, "unknown error code")):
        assert word in lib.mp_strerror(code).decode()
