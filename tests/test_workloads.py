"""The seeded input generators (workloads.py) are the specification of the
synthetic inputs: they must be deterministic, produce the stated structure,
and keep producing the same samples (SHA-256 of the float64 bytes, first 16
hex digits, pinned when the generators were written)."""
import hashlib

import numpy as np

import workloads as W


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()[:16]


def test_generators_are_pinned():
    T, m = W.rw8k()
    assert (len(T), m, _digest(T)) == (8192, 64, "cc5ba52052c2b459")
    T, m, _ = W.rw128k()
    assert (len(T), m, _digest(T)) == (131072, 256, "75fede4e1872cec6")
    T, m = W.sines()
    assert (len(T), m, _digest(T)) == (262144, 128, "ff8e702f573bb3fd")
    jobs = W.batch()
    assert len(jobs) == 512
    assert _digest(np.concatenate([j.T for j in jobs])) == "12ad68dbc76ea16b"
    T, m, anomalies = W.ecg()
    assert (len(T), m, _digest(T)) == (2097152, 512, "04da8345fbc01885")
    assert anomalies == [125003, 356673, 438203, 1178555, 1365215]
    T, m = W.uniform()
    assert (len(T), m, _digest(T)) == (262144, 256, "55a6ec1ca0ee6386")


def test_generators_are_deterministic():
    a, _, pa = W.rw128k(n=20000, m=64, nruns=5, nmotifs=3)
    b, _, pb = W.rw128k(n=20000, m=64, nruns=5, nmotifs=3)
    assert np.array_equal(a, b) and pa.runs == pb.runs and pa.motifs == pb.motifs
    c, _, _ = W.rw128k(seed=3, n=20000, m=64, nruns=5, nmotifs=3)
    assert not np.array_equal(a, c)


def test_rw128k_structure():
    T, m, pl = W.rw128k()
    assert len(pl.runs) == 20 and len(pl.motifs) == 10
    for s, L in pl.runs:
        assert 300 <= L <= 2000
        assert np.all(T[s:s + L] == T[s])            # exactly constant
    for a, b in pl.motifs:
        assert abs(a - b) >= m
        d = T[b:b + m] - T[a:a + m]                  # the planted N(0, 0.01) noise
        assert 0.005 < d.std() < 0.02
    # runs and motifs do not overlap
    cover = np.zeros(len(T), dtype=int)
    for s, L in pl.runs:
        cover[s:s + L] += 1
    for a, b in pl.motifs:
        cover[a:a + m] += 1
        cover[b:b + m] += 1
    assert cover.max() == 1


def test_batch_structure():
    jobs = W.batch()
    assert all(2048 <= len(j.T) <= 65536 for j in jobs)
    assert {j.m for j in jobs} == {32, 64, 128, 256}
    kinds = [j.kind for j in jobs]
    assert set(kinds) == {"aamp", "acamp"} and 200 < kinds.count("aamp") < 312
