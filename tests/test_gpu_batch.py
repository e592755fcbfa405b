"""GPU parity of mp_batch: many series of uneven length, mixed window length
and distance, in one launch (the persistent band kernel over the job table,
the simple kernel for short or generic-p jobs), its captured-graph replay and
its autotuner. Every job is checked against the oracle run on that series
alone."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import atol_for, check_profile

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


def _jobs(mp, specs):
    return [mp.Job(n=len(T), m=m, kind=KINDS[kind], excl=excl, R=R, p=p)
            for T, m, kind, p, excl, R in specs]


def _run(mp, specs, precision="fp64", out=None, T_cat=None):
    import torch
    if T_cat is None:
        T_cat = torch.as_tensor(np.concatenate([sp[0] for sp in specs]), device="cuda")
    P, I = mp.batch(T_cat, _jobs(mp, specs), precision=precision, out=out)
    torch.cuda.synchronize()
    return P, I, T_cat


def _check(specs, P, I, rtol, label, rows_per_job=None):
    P, I = P.cpu().numpy(), I.cpu().numpy()
    off = 0
    for b, (T, m, kind, p, excl, R) in enumerate(specs):
        N = len(T) - m + 1
        e = excl or W.excl_default(m)
        atol = atol_for(kind, m, "fp64" if rtol <= 1e-9 else "fp32", R)
        if rows_per_job is None:
            rows = None
            Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=e)
            Pg, Ig = P[off:off + N], I[off:off + N]
        else:
            rows = W.sample_rows(N, min(N, rows_per_job), seed=b)
            Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=e, rows=rows)
            Pg, Ig = P[off:off + N][rows], I[off:off + N][rows]
        check_profile(T, m, kind, p, e, Pg, Ig, Pr, Ir, Qr, rtol, atol, rows=rows,
                      label=f"{label} job {b} ({kind} p={p} n={len(T)} m={m})")
        off += N


def _mixed_specs(seed, count, nmax, kinds, with_runs=True):
    rng = np.random.default_rng(seed)
    specs = []
    for b in range(count):
        kind, p = kinds[b % len(kinds)]
        m = int(rng.choice([4, 8, 16, 32, 64]))
        n = int(rng.integers(m, nmax))
        T = np.cumsum(rng.standard_normal(n)) if rng.random() < 0.6 else W.noisy_sine(n, rng)
        if with_runs and kind == "acamp" and n > 400:
            s = int(rng.integers(0, n - 150))
            T[s:s + 120] = T[s]                       # a constant run
        excl = int(rng.choice([0, 0, 1, 3]))
        specs.append((T, m, kind, p, excl, 0))
    return specs


ALL = [("aamp", 2.0), ("acamp", 2.0), ("pnorm", 1.0), ("pnorm", 3.0), ("pnorm", 1.5)]
BAND = [("aamp", 2.0), ("acamp", 2.0), ("pnorm", 1.0), ("pnorm", 3.0)]


def test_batch_mixed_fp64(mp):
    """Lengths from m (one window) to 4000, every distance incl. generic p
    (simple kernel), short jobs below half a band, exclusion zones 1..ceil(m/4)."""
    specs = _mixed_specs(1, 30, 4000, ALL)
    specs.append((np.linspace(0, 1, 50), 50, "aamp", 2.0, 0, 0))       # n == m: no pairs
    specs.append((np.cumsum(np.ones(40)), 8, "acamp", 2.0, 40, 0))     # N <= excl
    _note(f"batch mixed fp64 jobs={len(specs)}")
    P, I, _ = _run(mp, specs)
    _check(specs, P, I, 1e-9, "mixed")


def test_batch_fp32(mp):
    specs = _mixed_specs(2, 16, 5000, BAND)
    specs = [(T, m, k, p, e, R) for T, m, k, p, e, R in specs if len(T) > 1500]
    _note(f"batch fp32 jobs={len(specs)}")
    P, I, _ = _run(mp, specs, precision="fp32")
    _check(specs, P, I, 1e-4, "fp32")


def test_batch_single_kind_kernels(mp):
    """Batches of one distance use that distance's own kernel."""
    for kind, p in BAND:
        specs = [(np.cumsum(np.random.default_rng(40 + k).standard_normal(1200 + 300 * k)), 24,
                  kind, p, 0, 0) for k in range(4)]
        _note(f"batch single kind {kind} p={p}")
        P, I, _ = _run(mp, specs)
        _check(specs, P, I, 1e-9, f"single-{kind}{p}")


def test_batch_long_and_short_windows(mp):
    """One launch holding windows on both sides of the long-window limit
    (2048): the statistics and the rescoring take the anchored path for some
    jobs and the direct one for others, per job. Both precisions, sampled
    rows of every job against the oracle."""
    rng = np.random.default_rng(4242)
    specs = []
    for k, (m, kind, p) in enumerate([(2100, "acamp", 2.0), (64, "acamp", 2.0), (3000, "aamp", 2.0),
                                      (200, "aamp", 2.0), (2048, "pnorm", 3.0), (2500, "acamp", 2.0),
                                      (100, "pnorm", 1.0)]):
        n = m + int(rng.integers(3000, 7000))
        T = np.cumsum(rng.standard_normal(n))
        if k == 5:
            T[1000:1000 + 2600] = T[1000]   # a constant run longer than m
        specs.append((T, m, kind, p, 0, 0))
    for prec, rtol in (("fp64", 1e-9), ("fp32", 1e-4)):
        _note(f"batch long+short windows {prec}: " +
              ", ".join(f"{kd} m={m} n={len(T)}" for T, m, kd, p, e, R in specs))
        P, I, _ = _run(mp, specs, precision=prec)
        _check(specs, P, I, rtol, f"long-short-{prec}", rows_per_job=160)


def test_batch_matches_single_series_calls(mp):
    import torch
    specs = _mixed_specs(3, 8, 3000, BAND, with_runs=False)
    _note("batch vs single calls")
    P, I, _ = _run(mp, specs)
    P, I = P.cpu().numpy(), I.cpu().numpy()
    off = 0
    for T, m, kind, p, excl, R in specs:
        N = len(T) - m + 1
        Td = torch.as_tensor(T, device="cuda")
        e = excl or None
        if kind == "aamp":
            Ps, Is = mp.aamp(Td, m, excl=e)
        elif kind == "acamp":
            Ps, Is = mp.acamp(Td, m, excl=e)
        else:
            Ps, Is = mp.pnorm(Td, m, p=p, excl=e)
        torch.cuda.synchronize()
        Ps, Is = Ps.cpu().numpy(), Is.cpu().numpy()
        same = Is == I[off:off + N]
        assert same.mean() > 0.99
        assert np.allclose(P[off:off + N], Ps, rtol=1e-9, atol=1e-6 if kind == "acamp" else 0)
        off += N


def test_batch_graph_replay(mp):
    """The second identical call replays the captured graph and reproduces the
    first bit for bit; after new data is written into the same buffers, a
    replay computes the new profiles."""
    import torch
    specs = _mixed_specs(5, 10, 3000, BAND)
    _note("batch graph replay")
    mp.set_profiling(False)                  # clears the counters
    P1, I1, T_cat = _run(mp, specs)          # tunes, captures and launches
    assert mp.profile_read()["graph_replays"] == 0
    P1c, I1c = P1.cpu().numpy().copy(), I1.cpu().numpy().copy()
    P1.fill_(-1.0)
    I1.fill_(-7)
    P2, I2, _ = _run(mp, specs, out=(P1, I1), T_cat=T_cat)
    assert mp.profile_read()["graph_replays"] == 1
    assert np.array_equal(P2.cpu().numpy(), P1c) and np.array_equal(I2.cpu().numpy(), I1c)
    _check(specs, P2, I2, 1e-9, "replay")
    # new data, same pointers
    rng = np.random.default_rng(99)
    specs2 = [(np.cumsum(rng.standard_normal(len(T))), m, k, p, e, R)
              for T, m, k, p, e, R in specs]
    T_cat.copy_(torch.as_tensor(np.concatenate([sp[0] for sp in specs2]), device="cuda"))
    P4, I4, _ = _run(mp, specs, out=(P1, I1), T_cat=T_cat)
    assert mp.profile_read()["graph_replays"] == 2
    _check(specs2, P4, I4, 1e-9, "replay-new-data")


def test_batch_workload_shape_sampled(mp):
    """The batch workload's recipe (random walks and noisy sines, m in
    {32, 64, 128, 256}, AAMP / ACAMP) at reduced count and length, every job
    checked on sampled rows, in FP64 and FP32."""
    import torch
    jobs = W.batch(seed=4, count=48, nrange=(2048, 12000))
    specs = [(jb.T, jb.m, jb.kind, 2.0, 0, 0) for jb in jobs]
    for prec, rtol in (("fp64", 1e-9), ("fp32", 1e-4)):
        _note(f"batch workload shape {prec} jobs={len(specs)}")
        P, I, _ = _run(mp, specs, precision=prec)
        _check(specs, P, I, rtol, f"workload-{prec}", rows_per_job=24)
    st = mp.profile_read()
    assert st["ms_autotune"] >= 0.0


def test_batch_replays_between_eager_calls(mp):
    """Graph replays interleaved with the program's own eager work (single-
    series calls that share the workspace, device syncs): every replay must
    equal the eager result. A single call on a longer series grows the
    workspace, which invalidates the captured graph; the next batch call must
    rebuild it and still be right."""
    import torch
    specs = _mixed_specs(7, 6, 2500, BAND)
    _note("batch replays between eager calls")
    P0, I0, T_cat = _run(mp, specs)
    ref_P, ref_I = P0.cpu().numpy().copy(), I0.cpu().numpy().copy()
    _check(specs, P0, I0, 1e-9, "eager-replay-ref")
    rng = np.random.default_rng(3)
    for k in range(3):
        # eager work of the program between the replays
        Tx = torch.as_tensor(np.cumsum(rng.standard_normal(3000)), device="cuda")
        Px, Ix = mp.acamp(Tx, 32)
        torch.cuda.synchronize()
        P, I, _ = _run(mp, specs, out=(P0, I0), T_cat=T_cat)
        assert np.array_equal(P.cpu().numpy(), ref_P), f"replay {k}"
        assert np.array_equal(I.cpu().numpy(), ref_I), f"replay {k}"
    # grow the workspace with a long single series, then replay again
    big = np.cumsum(rng.standard_normal(int(T_cat.numel()) + 50000))
    Pb, Ib = mp.aamp(torch.as_tensor(big, device="cuda"), 64)
    torch.cuda.synchronize()
    P, I, _ = _run(mp, specs, out=(P0, I0), T_cat=T_cat)
    assert np.array_equal(P.cpu().numpy(), ref_P) and np.array_equal(I.cpu().numpy(), ref_I)


def test_batch_full_workload(mp):
    """The full 512-series batch workload (3.9e11 pairs) in one call, FP64 and
    FP32 + refresh, against the oracle's stored rows: 32 rows of every series
    and 256 of 64 series (tests/golden/fullsize/batch512.npz); FP32 also on
    every row against FP64."""
    from tests import fullsize_refs as R
    jobs = W.batch()
    ref = R.load("batch512", series=[jb.T for jb in jobs])
    specs = [(jb.T, jb.m, jb.kind, 2.0, 0, 0) for jb in jobs]
    out = {}
    for prec, rtol in (("fp64", 1e-9), ("fp32", 1e-4)):
        _note(f"batch full workload {prec} jobs={len(specs)}")
        P, I, _ = _run(mp, specs, precision=prec)
        P, I = P.cpu().numpy(), I.cpu().numpy()
        out[prec] = P
        off = 0
        for b, (T, m, kind, p, excl, R_) in enumerate(specs):
            N = len(T) - m + 1
            e = W.excl_default(m)
            sel = ref["job"] == b
            rows = ref["rows"][sel]
            assert len(rows) >= 32
            check_profile(T, m, kind, 2.0, e, P[off:off + N][rows], I[off:off + N][rows],
                          ref["P"][sel], ref["I"][sel], ref["Q"][sel], rtol,
                          atol_for(kind, m, prec), rows=rows, sample=8,
                          label=f"full-{prec} job {b}")
            off += N
        _note(f"batch {prec}: {len(ref['rows'])} oracle rows over {len(specs)} series match")
    kinds = np.concatenate([np.full(len(jb.T) - jb.m + 1, jb.kind == "acamp") for jb in jobs])
    P32, P64 = out["fp32"], out["fp64"]
    assert np.array_equal(np.isinf(P32), np.isinf(P64))
    fin = np.isfinite(P64)
    tol = 1e-4 * P64 + np.where(kinds, 1e-6, 0.0)
    bad = np.nonzero(fin & (np.abs(P32 - P64) > tol))[0]
    assert bad.size == 0, f"{bad.size} FP32 rows beyond 1e-4 of FP64, e.g. {bad[:10]}"


def test_fp32_wide_bands_with_short_windows(mp, monkeypatch):
    """Regression: with 16 diagonals per lane chosen for the FP32 sweep, jobs
    whose windows are too short for FP32 (m < 32) run the FP64 sweep, whose
    bands stay 512 wide; their band tables must use that width. Checked for a
    batch and for single-series calls."""
    import torch
    monkeypatch.setenv("MP_KD", "16")
    rng = np.random.default_rng(21)
    specs = []
    for k, m in enumerate([8, 16, 24, 48, 64, 24]):
        T = np.cumsum(rng.standard_normal(1500 + 400 * k))
        specs.append((T, m, "acamp" if k % 2 else "aamp", 2.0, 0, 0))
    _note("fp32 wide bands, short windows (batch)")
    P, I, _ = _run(mp, specs, precision="fp32")
    P, I = P.cpu().numpy(), I.cpu().numpy()
    off = 0
    for b, (T, m, kind, p, excl, R) in enumerate(specs):
        N, e = len(T) - m + 1, W.excl_default(m)
        Pr, Ir, Qr = oracle.profile(T, m, kind, excl=e)
        rtol = 1e-9 if m < 32 else 1e-4
        check_profile(T, m, kind, p, e, P[off:off + N], I[off:off + N], Pr, Ir, Qr, rtol,
                      atol_for(kind, m, "fp64" if m < 32 else "fp32"), label=f"wide-{b}")
        off += N
    _note("fp32 wide bands, short windows (single)")
    T, m = specs[2][0], 24
    Ps, Is = mp.acamp(torch.as_tensor(T, device="cuda"), m, precision="fp32")
    torch.cuda.synchronize()
    Pr, Ir, Qr = oracle.profile(T, m, "acamp", excl=W.excl_default(m))
    check_profile(T, m, "acamp", 2.0, W.excl_default(m), Ps.cpu().numpy(), Is.cpu().numpy(),
                  Pr, Ir, Qr, 1e-9, atol_for("acamp", m), label="wide-single")
