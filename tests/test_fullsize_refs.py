"""The stored oracle rows of the full-size workloads are the oracle's.

Every file under tests/golden/fullsize/ must (1) belong to the series the
seeded generator produces today (stored SHA-256), (2) report for each row a
P that is the distance of the pair (row, I) and no larger than the distance
to a sample of other admissible windows, and (3) reproduce exactly when the
oracle is run again on a few of its rows (skipped for the files whose rows
cost more than a few seconds each). CPU only."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import fullsize_refs as R

SERIES = {
    "rw128k_acamp": (lambda: W.rw128k()[:2], "acamp", 2.0, 8),
    "rw128k_aamp": (lambda: W.rw128k()[:2], "aamp", 2.0, 8),
    "sines_p1": (W.sines, "pnorm", 1.0, 8),
    "sines_p3": (W.sines, "pnorm", 3.0, 8),
    "ecg_aamp": (lambda: W.ecg()[:2], "aamp", 2.0, 8),
    "ecg_acamp": (lambda: W.ecg()[:2], "acamp", 2.0, 8),
    "uniform_m16384_aamp": (lambda: (W.uniform()[0], 16384), "aamp", 2.0, 0),
    "uniform_m16384_acamp": (lambda: (W.uniform()[0], 16384), "acamp", 2.0, 0),
    "uniform_m65536_aamp": (lambda: (W.uniform()[0], 65536), "aamp", 2.0, 0),
    "uniform_m65536_acamp": (lambda: (W.uniform()[0], 65536), "acamp", 2.0, 0),
}


@pytest.fixture(scope="module", autouse=True)
def _oracle():
    oracle.build(force=False)


def _pair_checks(T, m, kind, p, rows, P, I, rng, pick=16, cols=64):
    N = len(T) - m + 1
    excl = W.excl_default(m)
    for k in rng.choice(len(rows), size=min(pick, len(rows)), replace=False):
        r, j = int(rows[k]), int(I[k])
        if j < 0:
            assert np.isinf(P[k])
            continue
        assert abs(r - j) >= excl
        d = oracle.distance(T, m, r, j, kind, p)
        assert d == P[k], f"row {r}: stored P is not the distance of (row, I)"
        for c in rng.integers(0, N, size=cols):
            if abs(int(c) - r) >= excl:
                assert oracle.distance(T, m, r, int(c), kind, p) >= P[k]


@pytest.mark.parametrize("name", sorted(SERIES))
def test_stored_series_rows(name):
    factory, kind, p, recompute = SERIES[name]
    T, m = factory()
    ref = R.load(name, T=T)
    rows, P, I, Q = ref["rows"], ref["P"], ref["I"], ref["Q"]
    assert int(ref["m"]) == m and str(ref["kind"]) == kind and float(ref["p"]) == p
    assert len(P) == len(rows) == len(I) == len(Q) and len(rows) >= 64
    assert np.all((Q >= P) | np.isinf(P))
    rng = np.random.default_rng(len(rows))
    _pair_checks(T, m, kind, p, rows, P, I, rng, pick=8 if m > 4096 else 16,
                 cols=16 if m > 4096 else 64)
    if recompute:
        k = np.sort(rng.choice(len(rows), size=recompute, replace=False))
        Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=W.excl_default(m), rows=rows[k])
        assert np.array_equal(Pr, P[k]) and np.array_equal(Ir, I[k]) and np.array_equal(Qr, Q[k])


def test_stored_batch_rows():
    jobs = W.batch()
    ref = R.load("batch512", series=[jb.T for jb in jobs])
    job, rows = ref["job"], ref["rows"]
    counts = np.bincount(job, minlength=len(jobs))
    assert np.all(counts >= 32) and np.sum(counts >= 256) >= 64
    rng = np.random.default_rng(7)
    for b in rng.choice(len(jobs), size=6, replace=False):
        jb = jobs[b]
        sel = np.nonzero(job == b)[0][:4]
        Pr, Ir, Qr = oracle.profile(jb.T, jb.m, jb.kind, excl=W.excl_default(jb.m),
                                    rows=rows[sel])
        assert np.array_equal(Pr, ref["P"][sel]) and np.array_equal(Ir, ref["I"][sel])
        _pair_checks(jb.T, jb.m, jb.kind, 2.0, rows[job == b], ref["P"][job == b],
                     ref["I"][job == b], rng, pick=4, cols=32)
