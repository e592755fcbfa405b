"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Sizes are chosen so the oracle finishes in seconds while the GPU launch still
spans several bands / segments and ragged tails; the full-size workloads are
checked on sampled rows in test_gpu_fullsize.py.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import atol_for, check_profile

pytestmark = pytest.mark.gpu

RTOL64 = 1e-9


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


def _run(mp, fn, T, m, **kw):
    import torch
    Td = torch.as_tensor(T, dtype=torch.float64, device="cuda")
    P, I = fn(Td, m, **kw)
    torch.cuda.synchronize()
    return P.cpu().numpy(), I.cpu().numpy()


def _kind_of(name):
    return {"aamp": "aamp", "pnorm": "pnorm", "acamp": "acamp"}[name]


def _parity(mp, T, m, kind, p=2.0, excl=None, precision="fp64", R=0, label=""):
    excl = excl or W.excl_default(m)
    _note(f"{label} kind={kind} p={p} n={len(T)} m={m} excl={excl} prec={precision} R={R}")
    if kind == "aamp":
        P, I = _run(mp, mp.aamp, T, m, excl=excl, precision=precision, R=R)
    elif kind == "pnorm":
        P, I = _run(mp, mp.pnorm, T, m, p=p, excl=excl, precision=precision, R=R)
    else:
        P, I = _run(mp, mp.acamp, T, m, excl=excl, precision=precision, R=R)
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl)
    rtol = RTOL64 if precision == "fp64" else 1e-4
    atol = atol_for(kind, m, precision, R)
    return check_profile(T, m, kind, p, excl, P, I, Pr, Ir, Qr, rtol, atol, label=label), P, I


def test_rw8k_aamp_fp64_full(mp):
    T, m = W.rw8k()
    info, _, _ = _parity(mp, T, m, "aamp", label="rw8k")
    print(info)


@pytest.mark.parametrize("R", [1, 7, 64, 1000])
def test_refresh_interval_variants(mp, R):
    rng = np.random.default_rng(100 + R)
    T = np.cumsum(rng.standard_normal(1500))
    _parity(mp, T, 32, "aamp", R=R, label=f"R{R}")


@pytest.mark.parametrize("p", [1.0, 3.0, 2.5])
def test_pnorm_fp64(mp, p):
    T, _ = W.sines(n=3000, m=48)
    _parity(mp, T, 48, "pnorm", p=p, label=f"pnorm{p}")


def test_pnorm_p2_equals_aamp(mp):
    rng = np.random.default_rng(5)
    T = np.cumsum(rng.standard_normal(2000))
    P1, I1 = _run(mp, mp.aamp, T, 40)
    P2, I2 = _run(mp, mp.pnorm, T, 40, p=2.0)
    assert np.array_equal(P1, P2) and np.array_equal(I1, I2)


def test_acamp_fp64_runs_and_motifs(mp):
    T, m, planted = W.rw128k(n=6000, m=64, nruns=4, nmotifs=3, run_len=(100, 300))
    info, P, I = _parity(mp, T, m, "acamp", label="acamp-small")
    for s, L in planted.runs:
        inside = np.arange(s, s + L - m + 1)
        assert np.all(np.isinf(P[inside])) and np.all(I[inside] == -1)
    N = len(P)
    const = np.zeros(N, dtype=bool)
    for s, L in planted.runs:
        const[s:s + L - m + 1] = True
    assert not np.any(const[I[I >= 0]]), "a constant window was reported as a neighbour"
    for a, b in planted.motifs:
        assert I[a] == b and I[b] == a


def test_edge_no_admissible_pair(mp):
    T = np.arange(20, dtype=np.float64)
    P, I = _run(mp, mp.aamp, T, 15, excl=6)          # N = 6 <= excl
    assert np.all(np.isinf(P)) and np.all(I == -1)
    P, I = _run(mp, mp.aamp, T, 20)                  # m = n: a single window
    assert P.shape == (1,) and np.isinf(P[0]) and I[0] == -1


def test_edge_two_windows(mp):
    T = np.array([0.0, 1.0, 3.0, 2.5])
    P, I = _run(mp, mp.aamp, T, 3, excl=1)
    assert list(I) == [1, 0]
    np.testing.assert_allclose(P, [oracle.distance(T, 3, 0, 1)] * 2, rtol=1e-15)


def test_edge_constant_series(mp):
    T = np.full(500, -1.5)
    P, I = _run(mp, mp.aamp, T, 16)
    assert np.all(P == 0.0)
    assert np.all(np.abs(np.arange(len(I)) - I) >= W.excl_default(16))
    P, I = _run(mp, mp.acamp, T, 16)
    assert np.all(np.isinf(P)) and np.all(I == -1)


def test_edge_exact_copy_zero_distance(mp):
    rng = np.random.default_rng(9)
    T = np.cumsum(rng.standard_normal(3000))
    m, a, b = 50, 300, 2100
    T[b:b + m] = T[a:a + m]
    P, I = _run(mp, mp.aamp, T, m)
    assert P[a] == 0.0 and P[b] == 0.0 and I[a] == b and I[b] == a


def test_excl_one_is_paper_behaviour(mp):
    rng = np.random.default_rng(12)
    T = rng.uniform(0, 1, 700)
    _parity(mp, T, 8, "aamp", excl=1, label="excl1")
    _parity(mp, T, 8, "acamp", excl=1, label="excl1-z")


def test_repeat_calls_bitwise_identical(mp):
    T, m = W.rw8k()
    P1, I1 = _run(mp, mp.aamp, T, m)
    P2, I2 = _run(mp, mp.aamp, T, m)
    assert np.array_equal(P1, P2) and np.array_equal(I1, I2)
