"""The sweeps' own pair-visit count (test mode MP_COUNT_PAIRS=1) equals the
number of admissible pairs, (N - excl)(N - excl + 1) / 2 per series: the
work split into bands, refresh segments, wave shares and jobs covers every
pair exactly once, for every kernel, precision, band width and batch mix."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

KINDS = {"aamp": 0, "pnorm": 1, "acamp": 2}


@pytest.fixture(scope="module")
def mp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1901_05708_amd as m
    m.load()
    return m


def _visits(mp, fn):
    import torch
    mp.set_profiling(True)
    fn()
    torch.cuda.synchronize()
    st = mp.profile_read()
    mp.set_profiling(False)
    return st["pairs_visited"], st["pairs"]


CASES = [
    # kind, p, n, m, excl, R, precision, sweep
    ("aamp", 2.0, 600, 24, 0, 0, "fp64", "auto"),
    ("aamp", 2.0, 2500, 24, 0, 37, "fp64", "auto"),       # short, ragged segments
    ("acamp", 2.0, 5000, 48, 700, 0, "fp64", "auto"),     # wide exclusion zone
    ("acamp", 2.0, 4000, 64, 1, 100, "fp32", "auto"),
    ("pnorm", 1.0, 3000, 32, 0, 0, "fp32", "auto"),
    ("pnorm", 3.0, 3000, 32, 0, 0, "fp64", "auto"),
    ("pnorm", 1.5, 1200, 16, 0, 0, "fp64", "auto"),       # generic p: its own band kernel
    ("pnorm", 2.5, 5000, 48, 0, 37, "fp64", "auto"),      # generic p, short segments
    ("pnorm", 7.0, 1200, 16, 0, 0, "fp64", "auto"),       # p > 6: simple kernel
    ("aamp", 2.0, 300, 16, 0, 0, "fp64", "auto"),         # below half a band: simple
    ("acamp", 2.0, 300, 16, 0, 0, "fp64", "band"),        # forced band, one partial band
    ("aamp", 2.0, 40, 40, 0, 0, "fp64", "auto"),          # one window, no pairs
    ("aamp", 2.0, 131072, 256, 0, 0, "fp64", "auto"),     # the headline shape
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}-n{c[2]}-m{c[3]}-{c[6]}-{c[7]}")
def test_single_series_visits_every_pair_once(mp, monkeypatch, case):
    import torch
    kind, p, n, m, excl, R, prec, sweep = case
    monkeypatch.setenv("MP_COUNT_PAIRS", "1")
    monkeypatch.setenv("MP_SWEEP", sweep)
    print(f"[gpu-case] counts {case}", flush=True)
    sys.stdout.flush()
    T = torch.as_tensor(np.cumsum(np.random.default_rng(n).standard_normal(n)), device="cuda")
    e = excl or None
    if kind == "aamp":
        fn = lambda: mp.aamp(T, m, excl=e, R=R, precision=prec)
    elif kind == "acamp":
        fn = lambda: mp.acamp(T, m, excl=e, R=R, precision=prec)
    else:
        fn = lambda: mp.pnorm(T, m, p=p, excl=e, R=R, precision=prec)
    visited, pairs = _visits(mp, fn)
    assert pairs == mp.pair_count(n, m, excl or W.excl_default(m))
    assert visited == pairs


def test_wide_fp32_bands_visit_every_pair_once(mp, monkeypatch):
    import torch
    monkeypatch.setenv("MP_COUNT_PAIRS", "1")
    monkeypatch.setenv("MP_KD", "16")
    T = torch.as_tensor(np.cumsum(np.random.default_rng(5).standard_normal(9000)), device="cuda")
    for kind in ("aamp", "acamp"):
        fn = (lambda: mp.aamp(T, 64, precision="fp32")) if kind == "aamp" else \
             (lambda: mp.acamp(T, 64, precision="fp32"))
        visited, pairs = _visits(mp, fn)
        assert visited == pairs == mp.pair_count(9000, 64, W.excl_default(64))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_visits_every_pair_once(mp, monkeypatch, prec):
    """Mixed jobs (every distance, lengths down to one window, m from 4 to
    128) in one launch: both band sweeps and the simple kernel together."""
    import torch
    monkeypatch.setenv("MP_COUNT_PAIRS", "1")
    rng = np.random.default_rng(77)
    jobs, series, expect = [], [], 0
    kinds = [("aamp", 2.0), ("acamp", 2.0), ("pnorm", 1.0), ("pnorm", 3.0), ("pnorm", 2.5)]
    for b in range(40):
        kind, p = kinds[b % len(kinds)]
        m = int(rng.choice([4, 16, 32, 64, 128]))
        n = int(rng.integers(m, 6000))
        excl = int(rng.choice([0, 1, 9]))
        series.append(np.cumsum(rng.standard_normal(n)))
        jobs.append(mp.Job(n=n, m=m, kind=KINDS[kind], excl=excl, p=p))
        expect += mp.pair_count(n, m, excl or W.excl_default(m))
    T_cat = torch.as_tensor(np.concatenate(series), device="cuda")
    print(f"[gpu-case] counts batch {prec}", flush=True)
    visited, pairs = _visits(mp, lambda: mp.batch(T_cat, jobs, precision=prec))
    assert pairs == expect
    assert visited == expect


@pytest.mark.parametrize("wps", [1, 2])
def test_capped_grids_visit_every_pair_once(mp, monkeypatch, wps):
    """Grids capped at one or two waves per SIMD (the long-window autotuner
    candidates) and refresh intervals of 16 m still split the band rows
    exactly."""
    import torch
    monkeypatch.setenv("MP_COUNT_PAIRS", "1")
    monkeypatch.setenv("MP_WPS", str(wps))
    for n, m, R in ((131072, 256, 4096), (60000, 2048, 32768)):
        T = torch.as_tensor(np.cumsum(np.random.default_rng(n + wps).standard_normal(n)), device="cuda")
        print(f"[gpu-case] counts wps={wps} n={n} m={m} R={R}", flush=True)
        for kind in ("aamp", "acamp"):
            fn = (lambda: mp.aamp(T, m, R=R)) if kind == "aamp" else (lambda: mp.acamp(T, m, R=R))
            visited, pairs = _visits(mp, fn)
            assert visited == pairs == mp.pair_count(n, m, W.excl_default(m))
