"""GPU parity of MP_FP32_AUTO: the FP32 tolerance served by whichever sweep
(FP32 with FP64 refresh, or FP64) the autotuner times faster, and the stats
that report which sweep ran. Every result is checked against the oracle at
1e-4, whatever the tuner picked."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import check_profile

pytestmark = pytest.mark.gpu

KINDS = {"aamp": 0, "pnorm": 1, "acamp": 2}


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


def _walk_with_motif(n, m, seed):
    rng = np.random.default_rng(seed)
    T = np.cumsum(rng.standard_normal(n))
    T[n // 2:n // 2 + m] = T[n // 5:n // 5 + m] + 0.01 * rng.standard_normal(m)
    return T


def _series(mp, kind, T, m, p, precision, R=0):
    import torch
    Td = torch.as_tensor(T, dtype=torch.float64, device="cuda")
    excl = W.excl_default(m)
    mp.set_profiling(True)
    if kind == "aamp":
        P, I = mp.aamp(Td, m, excl=excl, precision=precision, R=R)
    elif kind == "pnorm":
        P, I = mp.pnorm(Td, m, p=p, excl=excl, precision=precision, R=R)
    else:
        P, I = mp.acamp(Td, m, excl=excl, precision=precision, R=R)
    torch.cuda.synchronize()
    st = mp.profile_read()
    mp.set_profiling(False)
    return P.cpu().numpy(), I.cpu().numpy(), st


CASES = [("acamp", 2.0, 6000, 128, 1), ("pnorm", 1.0, 6000, 64, 2), ("aamp", 2.0, 5000, 64, 3)]


@pytest.mark.parametrize("kind,p,n,m,seed", CASES)
def test_auto_series_within_fp32_tolerance(mp, kind, p, n, m, seed):
    T = _walk_with_motif(n, m, seed)
    excl = W.excl_default(m)
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl)
    atol = 1e-6 if kind == "acamp" else 0.0
    # twice: the first call tunes, the second runs the cached choice
    for call in range(2):
        _note(f"fp32_auto {kind} p={p} n={n} m={m} call={call}")
        P, I, st = _series(mp, kind, T, m, p, "fp32_auto")
        check_profile(T, m, kind, p, excl, P, I, Pr, Ir, Qr, 1e-4, atol,
                      label=f"auto-{kind}-{call}")
        assert st["band_jobs"] == 1
        assert st["fp32_jobs"] in (0, 1)
        if kind == "aamp":
            assert st["fp32_jobs"] == 0       # AAMP has no FP32 sweep


@pytest.mark.parametrize("kind,p,expect32", [("acamp", 2.0, 1), ("pnorm", 1.0, 1),
                                             ("aamp", 2.0, 0), ("pnorm", 3.0, 0),
                                             ("pnorm", 2.5, 0)])
def test_stats_report_the_sweep_precision(mp, kind, p, expect32):
    T = _walk_with_motif(4000, 64, 7)
    _note(f"sweep precision report {kind} p={p}")
    _, _, st64 = _series(mp, kind, T, 64, p, "fp64")
    assert (st64["band_jobs"], st64["fp32_jobs"]) == (1, 0)
    _, _, st32 = _series(mp, kind, T, 64, p, "fp32")
    assert (st32["band_jobs"], st32["fp32_jobs"]) == (1, expect32)


@pytest.mark.parametrize("kind,p", [("acamp", 2.0), ("pnorm", 1.0)])
def test_auto_with_explicit_interval_runs_the_fp32_sweep(mp, kind, p):
    # no tuning with an explicit R: the mode then behaves as MP_FP32_REFRESH
    m, R = 64, 512
    T = _walk_with_motif(5000, m, 21)
    excl = W.excl_default(m)
    _note(f"fp32_auto explicit R={R} {kind} p={p}")
    P, I, st = _series(mp, kind, T, m, p, "fp32_auto", R=R)
    assert (st["band_jobs"], st["fp32_jobs"], st["refresh_rows"]) == (1, 1, R)
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl)
    atol = 1e-6 if kind == "acamp" else 0.0
    check_profile(T, m, kind, p, excl, P, I, Pr, Ir, Qr, 1e-4, atol, label=f"auto-R-{kind}")


def test_auto_batch_within_fp32_tolerance(mp):
    import torch
    rng = np.random.default_rng(11)
    specs = []
    for b, (kind, p, m) in enumerate([("acamp", 2.0, 64), ("aamp", 2.0, 32), ("pnorm", 1.0, 48),
                                      ("acamp", 2.0, 96), ("pnorm", 3.0, 40)]):
        n = int(rng.integers(2500, 5000))
        specs.append((_walk_with_motif(n, m, 100 + b), m, kind, p))
    jobs = [mp.Job(n=len(T), m=m, kind=KINDS[kind], excl=W.excl_default(m), p=p)
            for T, m, kind, p in specs]
    T_cat = torch.as_tensor(np.concatenate([sp[0] for sp in specs]), device="cuda")
    ref = [oracle.profile(T, m, kind, p=p, excl=W.excl_default(m)) for T, m, kind, p in specs]
    # the first call tunes and captures, the second replays the graph
    for call in range(2):
        _note(f"fp32_auto batch jobs={len(specs)} call={call}")
        P, I = mp.batch(T_cat, jobs, precision="fp32_auto")
        torch.cuda.synchronize()
        P, I = P.cpu().numpy(), I.cpu().numpy()
        off = 0
        for b, (T, m, kind, p) in enumerate(specs):
            N = len(T) - m + 1
            Pr, Ir, Qr = ref[b]
            atol = 1e-6 if kind == "acamp" else 0.0
            check_profile(T, m, kind, p, W.excl_default(m), P[off:off + N], I[off:off + N],
                          Pr, Ir, Qr, 1e-4, atol, label=f"auto-batch-{b}-{call}")
            off += N
