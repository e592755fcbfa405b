"""mp_profile_noalloc (the entry point that allocates no device memory)
against the entry points it is a variant of, through the C ABI.

For each distance, two calls in a row, the second on a smaller series, each
compared with mp_aamp / mp_pnorm / mp_acamp on the same input and refresh
interval: the same kernels run on slices of the static array instead of the
grow-only workspace, so P and I must agree exactly (and therefore meet the
oracle's tolerance wherever the existing entry point does). The small call is
also checked against the oracle directly, and one call runs at the window
limit.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import atol_for, check_profile

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_05708_amd as m
    m.load()
    return m


def _existing(mp, kind, Td, m, p, excl, precision, R):
    if kind == "aamp":
        return mp.aamp(Td, m, excl=excl, precision=precision, R=R)
    if kind == "pnorm":
        return mp.pnorm(Td, m, p=p, excl=excl, precision=precision, R=R)
    return mp.acamp(Td, m, excl=excl, precision=precision, R=R)


def _noalloc_abi(mp, kind, Td, m, p, excl, precision, R):
    """Direct ctypes call of mp_profile_noalloc with outputs allocated here."""
    import torch
    lib = mp.load()
    n = Td.numel()
    N = n - m + 1
    P = torch.full((N,), -7.0, dtype=torch.float64, device=Td.device)
    I = torch.full((N,), -7, dtype=torch.int64, device=Td.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.mp_profile_noalloc(mp._KIND_OF[kind], ctypes.c_void_p(Td.data_ptr()), n, m,
                                float(p), excl, mp._prec(precision), R,
                                ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(I.data_ptr()),
                                stream)
    assert rc == mp.MP_OK, lib.mp_strerror(rc).decode()
    return P, I


CASES = [
    # kind, p, m, precision, R, n of the first and of the second call
    ("acamp", 2.0, 100, "fp64", 700, 20000, 6003),
    ("aamp", 2.0, 64, "fp64", 1000, 16000, 5001),
    ("pnorm", 3.0, 48, "fp64", 800, 12000, 4100),
    ("acamp", 2.0, 128, "fp32", 512, 18000, 7000),
    ("pnorm", 1.0, 64, "fp32", 1024, 15000, 3333),
]


@pytest.mark.parametrize("kind,p,m,precision,R,n1,n2", CASES)
def test_noalloc_matches_existing_entry_point(mp, kind, p, m, precision, R, n1, n2):
    import torch
    rng = np.random.default_rng(1000 + m)
    excl = W.excl_default(m)
    for call, n in enumerate((n1, n2)):
        T = np.cumsum(rng.standard_normal(n))
        if kind == "acamp":
            T[n // 3:n // 3 + 2 * m] = T[n // 3]        # a constant run: +inf rows
        Td = torch.as_tensor(T, dtype=torch.float64, device="cuda")
        _note(f"noalloc call {call} kind={kind} p={p} n={n} m={m} prec={precision} R={R}")
        Pn, In = _noalloc_abi(mp, kind, Td, m, p, excl, precision, R)
        Pe, Ie = _existing(mp, kind, Td, m, p, excl, precision, R)
        torch.cuda.synchronize()
        Pn, In, Pe, Ie = Pn.cpu().numpy(), In.cpu().numpy(), Pe.cpu().numpy(), Ie.cpu().numpy()
        assert np.array_equal(In, Ie), f"call {call}: indices differ at {np.nonzero(In != Ie)[0][:10]}"
        assert np.array_equal(Pn, Pe), f"call {call}: values differ at {np.nonzero(Pn != Pe)[0][:10]}"
        if call == 1:
            Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl)
            rtol = 1e-9 if precision == "fp64" else 1e-4
            atol = 1e-6 if kind == "acamp" else 0.0
            check_profile(T, m, kind, p, excl, Pn, In, Pr, Ir, Qr, rtol, atol,
                          label=f"noalloc-{kind}-{precision}")


def test_noalloc_long_windows(mp):
    """m = 2048 (z-normalized): the window statistics keep each window's
    sums in the static array and the rescoring reads them back; bit for bit
    against the allocating call on two calls in a row, the second smaller,
    and against the oracle on sampled rows."""
    import torch
    m, excl = 2048, W.excl_default(2048)
    rng = np.random.default_rng(2048)
    for call, n in enumerate((14000, 9000)):
        T = np.cumsum(rng.standard_normal(n))
        T[n // 2:n // 2 + 600] = T[n // 2]
        Td = torch.as_tensor(T, dtype=torch.float64, device="cuda")
        _note(f"noalloc long windows call {call} n={n} m={m}")
        Pn, In = _noalloc_abi(mp, "acamp", Td, m, 2.0, excl, "fp64", 8192)
        Pe, Ie = _existing(mp, "acamp", Td, m, 2.0, excl, "fp64", 8192)
        torch.cuda.synchronize()
        assert torch.equal(In, Ie) and torch.equal(Pn, Pe), f"call {call}"
    rows = np.unique(np.concatenate([W.sample_rows(n - m + 1, 64, 9),
                                     np.arange(n // 2 - m - 2, n // 2 - m + 3)]))
    Pr, Ir, Qr = oracle.profile(T, m, "acamp", rows=rows, excl=excl)
    check_profile(T, m, "acamp", 2.0, excl, Pn.cpu().numpy()[rows], In.cpu().numpy()[rows],
                  Pr, Ir, Qr, 1e-9, atol_for("acamp", m), rows=rows, label="noalloc-long")


def test_noalloc_at_the_window_limit(mp):
    """A series of exactly MP_NOALLOC_MAX_N windows fits the static array;
    one more window is rejected before anything runs."""
    import torch
    m = 128
    n = mp.NOALLOC_MAX_N + m - 1
    rng = np.random.default_rng(77)
    T = np.cumsum(rng.standard_normal(n))
    Td = torch.as_tensor(T, dtype=torch.float64, device="cuda")
    excl = W.excl_default(m)
    _note(f"noalloc at the limit n={n} m={m}")
    Pn, In = _noalloc_abi(mp, "aamp", Td, m, 2.0, excl, "fp64", 16384)
    Pe, Ie = _existing(mp, "aamp", Td, m, 2.0, excl, "fp64", 16384)
    torch.cuda.synchronize()
    assert torch.equal(In, Ie) and torch.equal(Pn, Pe)
    rows = np.random.default_rng(5).choice(n - m + 1, size=48, replace=False)
    Pr, Ir, Qr = oracle.profile(T, m, "aamp", rows=rows, excl=excl)
    check_profile(T, m, "aamp", 2.0, excl, Pn.cpu().numpy()[rows], In.cpu().numpy()[rows],
                  Pr, Ir, Qr, 1e-9, 0.0, rows=rows, label="noalloc-limit")
    # one window too many: MP_EINVAL, outputs untouched
    lib = mp.load()
    Tl = torch.cat([Td, Td[:1]])
    P = torch.full((n - m + 2,), -7.0, dtype=torch.float64, device="cuda")
    I = torch.full((n - m + 2,), -7, dtype=torch.int64, device="cuda")
    rc = lib.mp_profile_noalloc(mp.KIND_AAMP, ctypes.c_void_p(Tl.data_ptr()), n + 1, m, 2.0,
                                excl, mp.MP_FP64, 0, ctypes.c_void_p(P.data_ptr()),
                                ctypes.c_void_p(I.data_ptr()), None)
    assert rc == mp.MP_EINVAL
    torch.cuda.synchronize()
    assert bool(torch.all(P == -7.0)) and bool(torch.all(I == -7))
