"""Write the oracle's profile rows for the full-size parity tests.

The full-size workloads are too long for the brute-force oracle to finish
during a GPU test run (the 2M-sample ECG series costs about a second per
z-normalized row on 8 cores), so its answers on seeded row samples are
computed once here, on the CPU, and stored under tests/golden/fullsize/.
This script calls only oracle/ and the seeded generators of workloads.py;
nothing in it touches the GPU library. Each file holds the rows, the oracle's
(P, I, Q) for them, the workload's parameters and a SHA-256 of the series, so
that a test can tell when the generator no longer reproduces the series the
values belong to. tests/test_fullsize_refs.py re-derives a few rows of every
file with the oracle.

    python tests/golden/make_fullsize_refs.py [name ...]

With no names every file is (re)written; long ones are written in chunks and
a rerun continues a partial file.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "fullsize")
CHUNK = 512


def series_hash(T) -> str:
    return hashlib.sha256(np.ascontiguousarray(T, dtype=np.float64).tobytes()).hexdigest()


def _rows_rw128k(N, m, planted, count, seed, extra=()):
    rows = list(W.sample_rows(N, count, seed=seed))
    for a, b in planted.motifs:
        for d in (-2, -1, 0, 1, 2):
            rows += [a + d, b + d]
    for s, L in planted.runs:
        rows += [s - m, s - m // 2, s - 1, s, s + L - m, s + L - m + 1, s + L - 1, s + L]
    rows += list(extra)
    rows = np.unique(np.clip(np.asarray(rows, dtype=np.int64), 0, N - 1))
    return rows


def _rows_ecg(N, m, anomalies, count, seed):
    rows = list(W.sample_rows(N, count, seed=seed))
    for c in anomalies:
        for d in (-64, -16, 0, 16, 64):
            rows.append(c - m // 2 + d)
    return np.unique(np.clip(np.asarray(rows, dtype=np.int64), 0, N - 1))


def specs():
    """name -> (series factory, m, kind, p, row factory). Row sets:
    rw128k: 4096 random rows plus the motif rows and every constant run's
    boundary rows (ACAMP, the headline), 1024 + the same for AAMP with the
    row that an earlier FP32 sweep got wrong; sines: 4096 rows per p (p = 3
    with its earlier FP32 miss); ecg: 4096 random rows per kind plus the rows
    around each anomalous beat; uniform n = 2^18 (the paper's Fig. 4 shape)
    with long windows: 256 rows at m = 16384, 64 rows at m = 65536."""
    out = {}

    def rw128k():
        T, m, pl = W.rw128k()
        return T, m, pl

    def rows_c2(T, m, pl):
        return _rows_rw128k(len(T) - m + 1, m, pl, 4096, 21)

    def rows_c2_aamp(T, m, pl):
        return _rows_rw128k(len(T) - m + 1, m, pl, 1024, 22, extra=(113495,))

    out["rw128k_acamp"] = (rw128k, "acamp", 2.0, rows_c2)
    out["rw128k_aamp"] = (rw128k, "aamp", 2.0, rows_c2_aamp)

    def sines():
        T, m = W.sines()
        return T, m, None

    out["sines_p1"] = (sines, "pnorm", 1.0,
                       lambda T, m, _: W.sample_rows(len(T) - m + 1, 4096, seed=31))
    out["sines_p3"] = (sines, "pnorm", 3.0,
                       lambda T, m, _: np.unique(np.append(
                           W.sample_rows(len(T) - m + 1, 4096, seed=33), 30128)))

    def ecg():
        T, m, an = W.ecg()
        return T, m, an

    for kind, seed in (("aamp", 51), ("acamp", 52)):
        out[f"ecg_{kind}"] = (ecg, kind, 2.0,
                              lambda T, m, an, s=seed: _rows_ecg(len(T) - m + 1, m, an, 4096, s))

    for m_long, count in ((16384, 256), (65536, 64)):
        def uni(m_long=m_long):
            T, _ = W.uniform()
            return T, m_long, None
        for kind, seed in (("aamp", 61), ("acamp", 62)):
            out[f"uniform_m{m_long}_{kind}"] = (
                uni, kind, 2.0,
                lambda T, m, _, c=count, s=seed + m_long // 1024: W.sample_rows(len(T) - m + 1, c, s))
    return out


def batch_rows():
    """The 512-series batch: 32 rows of every series, and 256 rows of 64
    series chosen by seed."""
    jobs = W.batch()
    rng = np.random.default_rng(41)
    deep = set(rng.choice(len(jobs), size=64, replace=False).tolist())
    per = []
    for b, jb in enumerate(jobs):
        N = len(jb.T) - jb.m + 1
        per.append(W.sample_rows(N, 256 if b in deep else 32, seed=1000 + b))
    return jobs, per


def write_series(name, factory, kind, p, row_fn):
    path = os.path.join(OUT, name + ".npz")
    T, m, aux = factory()
    rows = np.asarray(row_fn(T, m, aux), dtype=np.int64)
    excl = W.excl_default(m)
    h = series_hash(T)
    done = {}
    if os.path.exists(path):
        z = np.load(path)
        if str(z["series_sha256"]) == h and np.array_equal(z["rows"], rows) and int(z["m"]) == m:
            done = {k: z[k] for k in ("P", "I", "Q")}
    have = len(done["P"]) if done else 0
    P = np.full(len(rows), np.nan)
    I = np.full(len(rows), -2, dtype=np.int64)
    Q = np.full(len(rows), np.nan)
    if have:
        P[:have], I[:have], Q[:have] = done["P"][:have], done["I"][:have], done["Q"][:have]
    for s in range(have, len(rows), CHUNK):
        e = min(s + CHUNK, len(rows))
        t0 = time.time()
        P[s:e], I[s:e], Q[s:e] = oracle.profile(T, m, kind, p=p, excl=excl, rows=rows[s:e])
        print(f"{name}: rows {s}..{e} of {len(rows)} in {time.time() - t0:.1f} s", flush=True)
        np.savez_compressed(path + ".tmp.npz", rows=rows, P=P[:e], I=I[:e], Q=Q[:e], m=m,
                            excl=excl, kind=kind, p=p, n=len(T), series_sha256=h)
        os.replace(path + ".tmp.npz", path)
    if have >= len(rows):
        print(f"{name}: complete", flush=True)


def write_batch():
    path = os.path.join(OUT, "batch512.npz")
    jobs, per = batch_rows()
    job_of, rows, P, I, Q = [], [], [], [], []
    t0 = time.time()
    for b, (jb, r) in enumerate(zip(jobs, per)):
        Pr, Ir, Qr = oracle.profile(jb.T, jb.m, jb.kind, excl=W.excl_default(jb.m), rows=r)
        job_of.append(np.full(len(r), b, dtype=np.int32))
        rows.append(r)
        P.append(Pr)
        I.append(Ir)
        Q.append(Qr)
    h = hashlib.sha256(b"".join(np.ascontiguousarray(jb.T).tobytes() for jb in jobs)).hexdigest()
    np.savez_compressed(path + ".tmp.npz", job=np.concatenate(job_of), rows=np.concatenate(rows),
                        P=np.concatenate(P), I=np.concatenate(I), Q=np.concatenate(Q),
                        series_sha256=h)
    os.replace(path + ".tmp.npz", path)
    print(f"batch512: {sum(len(r) for r in rows)} rows in {time.time() - t0:.1f} s", flush=True)


ORDER = ["rw128k_acamp", "rw128k_aamp", "sines_p1", "sines_p3", "batch512", "ecg_aamp",
         "uniform_m16384_aamp", "uniform_m65536_aamp", "ecg_acamp", "uniform_m16384_acamp",
         "uniform_m65536_acamp"]


def main(names):
    os.makedirs(OUT, exist_ok=True)
    oracle.build(force=False)
    sp = specs()
    for name in names or ORDER:
        if name == "batch512":
            write_batch()
        else:
            factory, kind, p, row_fn = sp[name]
            write_series(name, factory, kind, p, row_fn)


if __name__ == "__main__":
    main(sys.argv[1:])
