"""GPU motif / discord extraction (mp_topk) against the oracle's greedy
definition, bit for bit, and end to end on planted structure: the 10 motif
pairs of the random walk and an anomalous beat of the ECG-like series."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle.topk import topk as topk_ref

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


@pytest.mark.parametrize("mode", ["motifs", "discords"])
@pytest.mark.parametrize("seed", range(6))
def test_topk_matches_oracle(mp, mode, seed):
    import torch
    rng = np.random.default_rng(seed)
    N = int(rng.choice([1, 7, 300, 5000, 70000]))
    P = np.round(rng.uniform(0, 4, N), 2)            # many exact ties
    P[rng.random(N) < 0.05] = np.inf
    I = rng.integers(-1, N, N)
    I[np.isinf(P)] = -1
    k = int(rng.choice([0, 1, 5, 40, 300]))
    excl = int(rng.integers(1, 50))
    _note(f"topk {mode} N={N} k={k} excl={excl}")
    gi, gj, gd = mp.topk(torch.as_tensor(P, device="cuda"), torch.as_tensor(I, device="cuda"),
                         k, excl, mode)
    ri, rj, rd = topk_ref(P, I, k, excl, mode)
    assert np.array_equal(gi.cpu().numpy(), ri)
    assert np.array_equal(gj.cpu().numpy(), rj)
    assert np.array_equal(gd.cpu().numpy(), rd)


def test_topk_repeated_calls_and_exhaustion(mp):
    import torch
    P = torch.tensor([3.0, 1.0, 2.0, float("inf"), 0.5], device="cuda", dtype=torch.float64)
    I = torch.tensor([1, 0, 4, -1, 2], device="cuda", dtype=torch.int64)
    # motifs, excl 1: (4, 2) then (1, 0); window 3 is infinite, so two rounds
    # exhaust the candidates. Discords, excl 2: 0, then 2, then 4.
    for _ in range(3):
        i, j, d = mp.topk(P, I, 10, 1, "motifs")
        assert i.tolist() == [4, 1] and j.tolist() == [2, 0] and d.tolist() == [0.5, 1.0]
        i, j, d = mp.topk(P, I, 10, 2, "discords")
        assert i.tolist() == [0, 2, 4]


@pytest.mark.parametrize("kind", ["aamp", "acamp"])
def test_planted_motifs_are_the_top_motifs(mp, kind):
    """The random walk of the headline workload without its constant runs:
    windows inside a run (or, z-normalized, constant except for a short
    tail) are exact matches of each other and would legitimately outrank
    the planted pairs."""
    import torch
    T, m, planted = W.rw128k(nruns=0)
    _note(f"rw128k {kind} top motifs")
    fn = mp.acamp if kind == "acamp" else mp.aamp
    P, I = fn(torch.as_tensor(T, device="cuda"), m)
    i, j, d = mp.topk(P, I, len(planted.motifs), m, "motifs")
    got = {frozenset((int(a), int(b))) for a, b in zip(i.cpu().numpy(), j.cpu().numpy())}
    want = {frozenset((a, b)) for a, b in planted.motifs}
    assert got == want


@pytest.mark.parametrize("kind", ["aamp", "acamp"])
def test_ecg_anomaly_is_the_top_discord(mp, kind):
    """One anomalous beat (amplitude 2, width 18 instead of about 1 and 6) in
    an ECG-like series of 2^18 samples: the top discord's window overlaps
    it. (With several anomalies of the same shape each one's nearest
    neighbour is another anomaly, so the 1-NN profile need not rank them
    all first.)"""
    import torch
    T, m, centres = W.ecg(n=262144, nanom=1)
    c = centres[0]
    _note(f"ecg {kind} top discord")
    fn = mp.acamp if kind == "acamp" else mp.aamp
    P, I = fn(torch.as_tensor(T, device="cuda"), m)
    i, j, d = mp.topk(P, I, 1, m, "discords")
    s0 = int(i.cpu().numpy()[0])
    assert s0 < c + 3 * 18 and c - 3 * 18 < s0 + m, (c, s0)
