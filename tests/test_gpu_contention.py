"""Many waves on many XCDs flushing into the same packed keys (64-bit
atomicMin from every band a row or column crosses). In a constant series
every pair ties at distance 0 and every key receives a flush from every band
its row or column crosses: no key may be lost (P = +inf) or corrupted (an
inadmissible or out-of-range partner). Which tied partner wins is not fixed:
within a band the column keys prefer the nearest row, across bands the
smallest index. A periodic series gives every row about n / period
exact-period partners whose distances tie up to rounding: the winner must be
one of them."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_05708_amd as m
    m.load()
    return m


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


# A constant series ties every pair (all sums are zero): the packed keys of
# every row and column collide on the same atomics. Under the FP32 flag AAMP
# runs the FP64 sweep and p = 1 the FP32 one.
@pytest.mark.parametrize("kind,p,precision", [("aamp", 2.0, "fp64"), ("aamp", 2.0, "fp32"),
                                              ("pnorm", 1.0, "fp64"), ("pnorm", 1.0, "fp32"),
                                              ("pnorm", 2.5, "fp64")])
def test_constant_series_loses_no_key(mp, kind, p, precision):
    import torch
    n, m = 200000, 64
    excl = W.excl_default(m)
    _note(f"contention constant series {kind} p={p} {precision} n={n}")
    T = torch.full((n,), 3.25, dtype=torch.float64, device="cuda")
    if kind == "aamp":
        P, I = mp.aamp(T, m, excl=excl, precision=precision)
    else:
        P, I = mp.pnorm(T, m, p=p, excl=excl, precision=precision)
    P, I = P.cpu().numpy(), I.cpu().numpy()
    N = n - m + 1
    i = np.arange(N)
    assert np.all(P == 0.0)
    assert np.all((I >= 0) & (I < N))
    assert np.all(np.abs(I - i) >= excl)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_periodic_series_picks_a_whole_period(mp, precision):
    import torch
    n, m, period = 150000, 200, 100
    excl = W.excl_default(m)
    _note(f"contention periodic series acamp {precision} n={n}")
    t = np.arange(n, dtype=np.float64)
    T = torch.as_tensor(np.sin(2.0 * np.pi * t / period), device="cuda")
    P, I = mp.acamp(T, m, excl=excl, precision=precision)
    P, I = P.cpu().numpy(), I.cpu().numpy()
    i = np.arange(n - m + 1)
    assert np.all(I >= 0)
    assert np.all(np.abs(I - i) >= excl)
    # a shift by one sample already costs DZ ~ 0.9; whole periods cost rounding
    assert np.all((I - i) % period == 0)
    assert P.max() < (1e-5 if precision == "fp64" else 1e-3)
