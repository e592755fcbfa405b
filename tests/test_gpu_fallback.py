"""GPU parity of the exact search for queued rows. Every row is pushed through
it (test hook MP_FORCE_FALLBACK): seeded with the sweep's winner, so that the
triangle-inequality pruning over pivot windows is active, and unseeded, so that
every column is scored. Either way the result must be the oracle's at 1e-9."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import atol_for, check_profile

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_05708_amd as m
    m.load()
    return m


def _run(mp, kind, T, m, p, force, precision="fp64"):
    import torch
    print(f"[gpu-case] fallback force={force} kind={kind} p={p} n={len(T)} m={m} {precision}",
          flush=True)
    sys.stdout.flush()
    os.environ["MP_FORCE_FALLBACK"] = str(force)
    try:
        Td = torch.as_tensor(T, dtype=torch.float64, device="cuda")
        if kind == "aamp":
            P, I = mp.aamp(Td, m, precision=precision)
        elif kind == "pnorm":
            P, I = mp.pnorm(Td, m, p=p, precision=precision)
        else:
            P, I = mp.acamp(Td, m, precision=precision)
        torch.cuda.synchronize()
    finally:
        del os.environ["MP_FORCE_FALLBACK"]
    return P.cpu().numpy(), I.cpu().numpy()


CASES = [("aamp", 2.0), ("acamp", 2.0), ("pnorm", 1.0), ("pnorm", 3.0)]


@pytest.mark.parametrize("force", [1, 2])
@pytest.mark.parametrize("kind,p", CASES)
def test_fallback_every_row(mp, kind, p, force):
    rng = np.random.default_rng(70 + force)
    n, m = 2600 if force == 1 else 1500, 40
    T = np.cumsum(rng.standard_normal(n))
    excl = W.excl_default(m)
    P, I = _run(mp, kind, T, m, p, force)
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl)
    atol = atol_for(kind, m)
    check_profile(T, m, kind, p, excl, P, I, Pr, Ir, Qr, 1e-9, atol, label=f"fb{force}-{kind}")


def test_fallback_runs_and_motifs(mp):
    """Constant windows are never pivots' victims: rows inside runs stay
    +inf/-1 (they are never queued) and planted motifs are found."""
    T, m, planted = W.rw128k(n=6000, m=48, nruns=4, nmotifs=3, run_len=(100, 300))
    P, I = _run(mp, "acamp", T, m, 2.0, 1)
    Pr, Ir, Qr = oracle.profile(T, m, "acamp", excl=W.excl_default(m))
    check_profile(T, m, "acamp", 2.0, W.excl_default(m), P, I, Pr, Ir, Qr, 1e-9,
                  atol_for("acamp", m), label="fb-runs")
    for a, b in planted.motifs:
        assert I[a] == b and I[b] == a


def test_fallback_large_m_unstaged(mp):
    """Windows longer than the staged limit read the row window from T."""
    rng = np.random.default_rng(5)
    T = np.cumsum(rng.standard_normal(4000))
    m = 1100
    P, I = _run(mp, "aamp", T, m, 2.0, 1)
    Pr, Ir, Qr = oracle.profile(T, m, "aamp", excl=W.excl_default(m))
    check_profile(T, m, "aamp", 2.0, W.excl_default(m), P, I, Pr, Ir, Qr, 1e-9, 0.0,
                  label="fb-large-m")


def test_fallback_seeded_equals_unseeded(mp):
    """Pruning must not change the answer: seeded and unseeded searches agree
    bit for bit on a series with many near-ties (a noisy sine)."""
    T, m = W.noisy_sine(3000, np.random.default_rng(8)), 50
    for kind, p in CASES:
        P1, I1 = _run(mp, kind, T, m, p, 1)
        P2, I2 = _run(mp, kind, T, m, p, 2)
        assert np.array_equal(I1, I2), kind
        assert np.array_equal(P1, P2), kind
