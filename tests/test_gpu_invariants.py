"""Properties of the profile that hold at any size, checked on the GPU at the
full sizes of the workloads (no oracle needed): translation and scaling
(AAMP, p-norm), affine invariance (ACAMP), and time reversal (all three).
Values must agree within the tolerance; where the indices differ (exact
ties, e.g. inside constant runs), the reported pair is checked directly."""
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


def _run(mp, kind, T, m, p=2.0, precision="fp64"):
    import torch
    print(f"[gpu-case] invariants {kind} p={p} n={len(T)} m={m} {precision}", flush=True)
    sys.stdout.flush()
    Td = torch.as_tensor(T, device="cuda")
    if kind == "aamp":
        P, I = mp.aamp(Td, m, precision=precision)
    elif kind == "acamp":
        P, I = mp.acamp(Td, m, precision=precision)
    else:
        P, I = mp.pnorm(Td, m, p=p, precision=precision)
    torch.cuda.synchronize()
    return P.cpu().numpy(), I.cpu().numpy()


def _same(P1, I1, P2, I2, rtol, atol, label, T2=None, m=None, kind="aamp", p=2.0):
    """Values agree within the tolerance. Where the indices differ (ties:
    windows inside a constant run are exact copies of each other, and round-
    off picks among them), the second index must be admissible and its
    direct FP64 distance in the second series must equal P2 (checked on up
    to 200 such rows)."""
    import oracle
    fin = np.isfinite(P1)
    assert np.array_equal(fin, np.isfinite(P2)), label
    err = np.abs(P1[fin] - P2[fin])
    assert np.all(err <= rtol * P1[fin] + atol), f"{label}: worst {np.max(err):.3e}"
    rows = np.nonzero(fin & (I1 != I2))[0]
    if T2 is not None and rows.size:
        excl = W.excl_default(m)
        for i in np.random.default_rng(0).choice(rows, size=min(200, rows.size), replace=False):
            j = int(I2[i])
            assert abs(int(i) - j) >= excl, f"{label}: row {i} index {j} not admissible"
            d = oracle.distance(T2, m, int(i), j, kind, p)
            assert abs(d - P2[i]) <= 1e-9 * max(d, 1e-300) + 1e-9, f"{label}: row {i}"


@pytest.fixture(scope="module")
def rw(mp):
    T, m, _ = W.rw128k()
    return T, m


def test_aamp_translation_and_scaling(mp, rw):
    T, m = rw
    P, I = _run(mp, "aamp", T, m)
    P2, I2 = _run(mp, "aamp", T + 1234.5, m)
    _same(P, I, P2, I2, 1e-9, 1e-9, "aamp translation", T + 1234.5, m)
    P3, I3 = _run(mp, "aamp", -3.5 * T, m)
    _same(3.5 * P, I, P3, I3, 1e-9, 1e-9, "aamp scaling", -3.5 * T, m)


def test_acamp_affine_invariance(mp, rw):
    T, m = rw
    P, I = _run(mp, "acamp", T, m)
    for a, c in ((2.0, 5.0), (-3.0, -40.0), (1e-3, 1e3)):
        P2, I2 = _run(mp, "acamp", a * T + c, m)
        _same(P, I, P2, I2, 1e-8, 1e-6, f"acamp affine a={a} c={c}", a * T + c, m, "acamp")


@pytest.mark.parametrize("kind", ["aamp", "acamp"])
def test_time_reversal(mp, rw, kind):
    """Reversing the series reverses every window: D(i, j) of T equals
    D(N-1-i, N-1-j) of the reversed series."""
    T, m = rw
    N = len(T) - m + 1
    P, I = _run(mp, kind, T, m)
    Pr, Ir = _run(mp, kind, T[::-1].copy(), m)
    Pr, Ir = Pr[::-1], Ir[::-1]
    Ir = np.where(Ir >= 0, N - 1 - Ir, -1)
    _same(P, I, Pr, Ir, 1e-9, 1e-6 if kind == "acamp" else 0.0, f"{kind} reversal", T, m, kind)


@pytest.mark.parametrize("p", [1.0, 3.0])
def test_pnorm_translation_full_size(mp, p):
    T, m = W.sines()
    P, I = _run(mp, "pnorm", T, m, p=p)
    P2, I2 = _run(mp, "pnorm", T + 77.0, m, p=p)
    _same(P, I, P2, I2, 1e-9, 1e-9, f"p={p} translation", T + 77.0, m, "pnorm", p)


def test_fp32_translation_invariance(mp, rw):
    """The single-precision streams are recentred, so a large offset must not
    change the FP32 + refresh result beyond its bound."""
    T, m = rw
    P, I = _run(mp, "aamp", T, m, precision="fp32")
    P2, I2 = _run(mp, "aamp", T + 1e4, m, precision="fp32")
    _same(P, I, P2, I2, 2e-4, 0.0, "fp32 aamp translation", T + 1e4, m)
