"""GPU parity of the band sweep kernel (forced with MP_SWEEP=band) on shapes
that exercise its edges: partial last bands, segments of one row, the triangle
corner, exclusion zones of every size, constant runs, exact copies."""
import os
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


def _call(mp, kind, T, m, p=2.0, excl=None, R=0, sweep="band", precision="fp64"):
    import torch
    old = os.environ.get("MP_SWEEP")
    os.environ["MP_SWEEP"] = sweep
    try:
        Td = torch.as_tensor(T, dtype=torch.float64, device="cuda")
        if kind == "aamp":
            P, I = mp.aamp(Td, m, excl=excl, R=R, precision=precision)
        elif kind == "pnorm":
            P, I = mp.pnorm(Td, m, p=p, excl=excl, R=R, precision=precision)
        else:
            P, I = mp.acamp(Td, m, excl=excl, R=R, precision=precision)
        torch.cuda.synchronize()
    finally:
        if old is None:
            del os.environ["MP_SWEEP"]
        else:
            os.environ["MP_SWEEP"] = old
    return P.cpu().numpy(), I.cpu().numpy()


def _check(mp, kind, T, m, p=2.0, excl=None, R=0, label=""):
    excl = excl or W.excl_default(m)
    _note(f"{label}: band kind={kind} p={p} n={len(T)} m={m} excl={excl} R={R}")
    P, I = _call(mp, kind, T, m, p=p, excl=excl, R=R)
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl)
    atol = atol_for(kind, m, "fp64", R)
    return check_profile(T, m, kind, p, excl, P, I, Pr, Ir, Qr, 1e-9, atol, label=label), P, I


# N - excl relative to the band width 512 (8 diagonals x 64 lanes): below one
# band, exactly one, one plus a bit, several with a ragged last band
@pytest.mark.parametrize("n", [400, 560, 600, 1100, 2500])
@pytest.mark.parametrize("kind", ["aamp", "acamp"])
def test_band_ragged_sizes(mp, n, kind):
    rng = np.random.default_rng(n)
    T = np.cumsum(rng.standard_normal(n))
    _check(mp, kind, T, 24, label=f"ragged{n}")


# segment lengths that leave 1-row and partial-block segments
@pytest.mark.parametrize("R", [8, 16, 24, 64, 200])
def test_band_segment_lengths(mp, R):
    rng = np.random.default_rng(200 + R)
    T = np.cumsum(rng.standard_normal(1700))
    _check(mp, "aamp", T, 40, R=R, label=f"R{R}")
    _check(mp, "acamp", T, 40, R=R, label=f"R{R}z")


@pytest.mark.parametrize("excl", [1, 3, 100, 700])
def test_band_exclusion_zones(mp, excl):
    rng = np.random.default_rng(300 + excl)
    T = rng.uniform(-1, 1, 1500)
    _check(mp, "aamp", T, 16, excl=excl, label=f"excl{excl}")


@pytest.mark.parametrize("p", [1.0, 3.0])
def test_band_pnorm(mp, p):
    T, _ = W.sines(n=2600, m=32)
    _check(mp, "pnorm", T, 32, p=p, label=f"pnorm{p}")


def test_band_acamp_constant_runs_and_motifs(mp):
    T, m, planted = W.rw128k(n=5000, m=48, nruns=5, nmotifs=3, run_len=(80, 400))
    info, P, I = _check(mp, "acamp", T, m, label="runs")
    for s, L in planted.runs:
        inside = np.arange(s, s + L - m + 1)
        assert np.all(np.isinf(P[inside])) and np.all(I[inside] == -1)
    for a, b in planted.motifs:
        assert I[a] == b and I[b] == a


def test_band_exact_copy_and_zero_keys(mp):
    rng = np.random.default_rng(17)
    T = np.cumsum(rng.standard_normal(3000))
    m, a, b = 64, 100, 1900
    T[b:b + m] = T[a:a + m]
    P, I = _call(mp, "aamp", T, m)
    assert P[a] == 0.0 and P[b] == 0.0 and I[a] == b and I[b] == a
    T2 = np.full(900, 2.0)
    P, I = _call(mp, "aamp", T2, 16)
    assert np.all(P == 0.0)
    assert np.all(np.abs(np.arange(len(I)) - I) >= W.excl_default(16))


def test_band_matches_simple_kernel(mp):
    T, m = W.rw8k()
    Pb, Ib = _call(mp, "aamp", T, m, sweep="band")
    Ps, Is = _call(mp, "aamp", T, m, sweep="simple")
    same = Ib == Is
    assert same.mean() > 0.999
    assert np.array_equal(Pb[same], Ps[same])


def test_band_rw8k_full(mp):
    T, m = W.rw8k()
    info, _, _ = _check(mp, "aamp", T, m, label="rw8k-band")
    print(info)


def test_band_repeatable(mp):
    T, m = W.rw8k()
    P1, I1 = _call(mp, "acamp", T, m)
    P2, I2 = _call(mp, "acamp", T, m)
    assert np.array_equal(P1, P2) and np.array_equal(I1, I2)


# ---- FP32 sweep with FP64 restarts: profile values within 1e-4 relative ----

def _check32(mp, kind, T, m, p=2.0, excl=None, R=0, label=""):
    excl = excl or W.excl_default(m)
    _note(f"{label}: band fp32 kind={kind} p={p} n={len(T)} m={m} excl={excl} R={R}")
    P, I = _call(mp, kind, T, m, p=p, excl=excl, R=R, precision="fp32")
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl)
    atol = 1e-6 if kind == "acamp" else 0.0
    return check_profile(T, m, kind, p, excl, P, I, Pr, Ir, Qr, 1e-4, atol, label=label), P, I


@pytest.mark.parametrize("kind", ["aamp", "acamp"])
@pytest.mark.parametrize("n", [560, 2500])
def test_band_fp32_ragged(mp, kind, n):
    rng = np.random.default_rng(900 + n)
    T = np.cumsum(rng.standard_normal(n))
    _check32(mp, kind, T, 24, label=f"fp32-{kind}-{n}")


@pytest.mark.parametrize("R", [16, 200, 1024])
def test_band_fp32_refresh_intervals(mp, R):
    rng = np.random.default_rng(950 + R)
    T = np.cumsum(rng.standard_normal(3000))
    _check32(mp, "aamp", T, 48, R=R, label=f"fp32-R{R}")
    _check32(mp, "acamp", T, 48, R=R, label=f"fp32-R{R}z")


@pytest.mark.parametrize("p", [1.0, 3.0])
def test_band_fp32_pnorm(mp, p):
    T, _ = W.sines(n=2600, m=32)
    _check32(mp, "pnorm", T, 32, p=p, label=f"fp32-pnorm{p}")


def test_band_fp32_runs_motifs_offset(mp):
    T, m, planted = W.rw128k(n=5000, m=48, nruns=5, nmotifs=3, run_len=(80, 400))
    T = T + 1e4          # a large offset: the FP32 streams are recentred
    info, P, I = _check32(mp, "acamp", T, m, label="fp32-runs")
    for s, L in planted.runs:
        inside = np.arange(s, s + L - m + 1)
        assert np.all(np.isinf(P[inside])) and np.all(I[inside] == -1)
    info, P, I = _check32(mp, "aamp", T, m, label="fp32-offset-aamp")


# ---- long windows: the exact restarts and the rescoring run over m >= 2048 ----

@pytest.mark.parametrize("m", [2048, 4096])
@pytest.mark.parametrize("kind", ["aamp", "acamp"])
def test_band_long_windows(mp, kind, m):
    rng = np.random.default_rng(m + (kind == "acamp"))
    T = np.cumsum(rng.standard_normal(m + 3000))
    _check(mp, kind, T, m, label=f"long-{kind}-{m}")
    _check32(mp, kind, T, m, label=f"long-fp32-{kind}-{m}")


def test_band_long_windows_pnorm(mp):
    T, _ = W.sines(n=7000, m=2048)
    _check(mp, "pnorm", T, 2048, p=3.0, label="long-p3")
    _check(mp, "pnorm", T, 2048, p=1.0, label="long-p1")


def test_band_long_windows_pnorm_generic_fp32(mp):
    """The long-window rescoring of p-norms: a non-integer p (its terms are
    powers, rounded as in the direct sum) on an offset series, and p = 1 in
    FP32 + refresh, whose self-check compares the carried sums."""
    T, _ = W.sines(n=5000, m=2048)
    _check(mp, "pnorm", T + 300.0, 2048, p=2.5, label="long-pgen-offset")
    _check32(mp, "pnorm", T, 2048, p=1.0, label="long-fp32-p1")


@pytest.mark.parametrize("wps", [1, 2])
@pytest.mark.parametrize("kind,p,prec", [("aamp", 2.0, "fp64"), ("acamp", 2.0, "fp64"),
                                         ("acamp", 2.0, "fp32"), ("pnorm", 1.0, "fp32")])
def test_band_long_windows_long_refresh(mp, monkeypatch, kind, p, prec, wps):
    """m = 2048 over 20000 samples with the longest refresh interval the
    autotuner allows (16 m; m for the p = 1 sums in single precision) and
    grids capped at one and two waves per SIMD (the sweep then runs in blocks
    of four waves): many long items, one exact restart each. Checked on
    sampled rows."""
    monkeypatch.setenv("MP_WPS", str(wps))
    m = 2048
    R = m if kind == "pnorm" else 16 * m
    T, _, _ = W.rw128k(n=20000, m=m, nruns=0, nmotifs=2, seed=31)
    excl = W.excl_default(m)
    N = len(T) - m + 1
    rows = W.sample_rows(N, 192, 32)
    _note(f"long-refresh {kind} p={p} {prec}: n={len(T)} m={m} R={R} wps={wps}")
    P, I = _call(mp, kind, T, m, p=p, excl=excl, R=R, precision=prec)
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl, rows=rows)
    if prec == "fp64":
        rtol, atol = 1e-9, atol_for(kind, m, "fp64", R)
    else:
        rtol, atol = 1e-4, (1e-6 if kind == "acamp" else 0.0)
    check_profile(T, m, kind, p, excl, P[rows], I[rows], Pr, Ir, Qr, rtol, atol, rows=rows,
                  label=f"long-refresh-{kind}{p:g}-{prec}-wps{wps}")


def test_band_long_windows_runs_offset(mp):
    """Window statistics and rescoring of long windows (m >= 2048: one exact
    anchor per 256 windows and exact slides, constant flags from counts of
    sample changes; winners summed once per run of a common diagonal) on
    constant runs shorter than, exactly, just over and longer than m and a
    near-constant run; then on a walk offset by 1e4 with steps of 1e-2.
    Windows inside a run are constant (+inf, -1); rows at every run edge, at
    every edge minus m, and a sample are checked against the oracle. (The
    windows that end a run's approach hold one walk sample and m - 1 equal
    ones; pairs of them match exactly, DZ = 0, and on an offset series the
    oracle's FP64 means put its own value of such a pair microunits off, so
    the two cases are separate.)"""
    rng = np.random.default_rng(77)
    m, n = 2048, 16000
    T = np.cumsum(rng.standard_normal(n))
    runs = [(1500, 700), (5000, 3000), (9500, 2100), (12500, 2048)]
    for s0, L in runs:
        T[s0:s0 + L] = T[s0]
    T[14700:15600] = T[14700] + 1e-9 * rng.standard_normal(900)
    excl = W.excl_default(m)
    N = n - m + 1
    edges = [e for s0, L in runs for e in (s0, s0 + L)] + [14700, 15600]
    near = [r for e in edges for base in (e, e - m + 1) for r in range(base - 3, base + 4)]
    rows = np.unique(np.clip(np.concatenate([near, W.sample_rows(N, 96, 5)]), 0, N - 1))
    _note(f"long-window stats: acamp n={n} m={m} runs={runs} rows={len(rows)}")
    P, I = _call(mp, "acamp", T, m, excl=excl)
    assert np.all(np.isinf(P[5000:5953])) and np.all(I[5000:5953] == -1)
    assert np.isinf(P[12500]) and np.isfinite(P[12499]) and np.isfinite(P[12501])
    Pr, Ir, Qr = oracle.profile(T, m, "acamp", excl=excl, rows=rows)
    check_profile(T, m, "acamp", 2.0, excl, P[rows], I[rows], Pr, Ir, Qr, 1e-9,
                  atol_for("acamp", m), rows=rows, label="long-stats-runs")
    To = 1e4 + 1e-2 * np.cumsum(np.random.default_rng(78).standard_normal(n))
    rows = W.sample_rows(N, 128, 6)
    _note(f"long-window stats: acamp offset 1e4 n={n} m={m} rows={len(rows)}")
    for kind in ("acamp", "aamp"):
        P, I = _call(mp, kind, To, m, excl=excl)
        Pr, Ir, Qr = oracle.profile(To, m, kind, excl=excl, rows=rows)
        check_profile(To, m, kind, 2.0, excl, P[rows], I[rows], Pr, Ir, Qr, 1e-9,
                      atol_for(kind, m), rows=rows, label=f"long-offset-{kind}")


@pytest.mark.parametrize("kind", ["aamp", "acamp"])
def test_long_windows_many_runs(mp, kind):
    """m = 2048 on a pattern of period 97 repeated under strong noise: every
    multiple of the period is a near-tie, so neighbouring rows change winner
    diagonal more often than on a plain series (Euclidean: about 20 runs
    per 300 rows, more than the 16 anchor blocks per block of rows, so some
    anchor blocks take two runs; z-normalized: one long run). Sampled rows
    and a contiguous stretch of rows against the oracle."""
    m, n = 2048, 9000
    rng = np.random.default_rng(2049 + (kind == "acamp"))
    T = np.tile(rng.standard_normal(97), n // 97 + 1)[:n] + 0.7 * rng.standard_normal(n)
    excl = W.excl_default(m)
    N = n - m + 1
    rows = np.unique(np.concatenate([W.sample_rows(N, 96, 13), np.arange(3000, 3300)]))
    _note(f"long windows many runs {kind}: n={n} m={m}")
    P, I = _call(mp, kind, T, m, excl=excl, R=8 * m)
    d = I[3000:3300] - np.arange(3000, 3300)
    runs = 1 + np.count_nonzero(d[1:] != d[:-1])
    _note(f"runs over 300 rows: {runs}")
    Pr, Ir, Qr = oracle.profile(T, m, kind, excl=excl, rows=rows)
    check_profile(T, m, kind, 2.0, excl, P[rows], I[rows], Pr, Ir, Qr, 1e-9,
                  atol_for(kind, m, "fp64", 8 * m), rows=rows, label=f"long-many-runs-{kind}")


# ---- p-norms with other p (1 < p <= 6): a band kernel of their own ----

@pytest.mark.parametrize("p", [1.5, 2.5, 4.7, 6.0])
def test_band_generic_p(mp, p):
    """pow per term in the sweep and the restarts; sentinels sized per p."""
    rng = np.random.default_rng(1300 + int(10 * p))
    T = np.cumsum(rng.standard_normal(3000))
    _check(mp, "pnorm", T, 32, p=p, label=f"pgen-{p}")


def test_band_generic_p_long_and_offset(mp):
    T, _ = W.sines(n=7000, m=512)
    _check(mp, "pnorm", T + 500.0, 512, p=2.5, label="pgen-long-offset")


def test_generic_p_above_band_limit_uses_simple_kernel(mp):
    """p = 7 would let real terms approach the sentinel sums; it stays on the
    simple kernel and must still match the oracle."""
    rng = np.random.default_rng(1377)
    T = np.cumsum(rng.standard_normal(1500))
    excl = W.excl_default(24)
    P, I = _call(mp, "pnorm", T, 24, p=7.0, excl=excl, sweep="auto")
    Pr, Ir, Qr = oracle.profile(T, 24, "pnorm", p=7.0, excl=excl)
    check_profile(T, 24, "pnorm", 7.0, excl, P, I, Pr, Ir, Qr, 1e-9, 0.0, label="pgen-7")
