"""Pins of the motif / discord extraction oracle on hand-worked cases."""
import numpy as np

from oracle.topk import topk


def test_hand_worked_motifs():
    # P and I of 10 windows; excl = 2 removes the window and its direct neighbours
    P = np.array([5.0, 1.0, 4.0, 3.0, 1.0, 6.0, np.inf, 2.0, 2.0, 7.0])
    I = np.array([3, 4, 8, 0, 1, 9, -1, 2, 2, 5])
    i, j, d = topk(P, I, 10, 2, "motifs")
    # pick 1: min P = 1.0 at 1 and 4 -> 1 (smallest index), partner 4; excluded
    #         0..2 and 3..5
    # pick 2: left 7, 8, 9 (6 is inf): min 2.0 at 7, partner 2; excluded 6..8
    # pick 3: left 9: P = 7, partner 5
    assert i.tolist() == [1, 7, 9]
    assert j.tolist() == [4, 2, 5]
    assert d.tolist() == [1.0, 2.0, 7.0]


def test_hand_worked_discords():
    P = np.array([5.0, 1.0, 4.0, 3.0, 1.0, 6.0, np.inf, 2.0, 2.0, 7.0])
    I = np.array([3, 4, 8, 0, 1, 9, -1, 2, 2, 5])
    i, j, d = topk(P, I, 3, 3, "discords")
    # 7.0 at 9 (excl 7..9), then 6.0 at 5 (excl 3..7), then 5.0 at 0 (excl 0..2)
    assert i.tolist() == [9, 5, 0] and d.tolist() == [7.0, 6.0, 5.0]
    i, j, d = topk(P, I, 10, 3, "discords")
    assert i.tolist() == [9, 5, 0]          # nothing finite is left after three


def test_properties_on_random_profiles():
    rng = np.random.default_rng(0)
    for trial in range(20):
        N = int(rng.integers(1, 400))
        P = np.round(rng.uniform(0, 5, N), 1)          # many exact ties
        P[rng.random(N) < 0.1] = np.inf
        I = rng.integers(0, N, N)
        excl = int(rng.integers(1, 20))
        for mode in ("motifs", "discords"):
            i, j, d = topk(P, I, 50, excl, mode)
            assert np.all(np.isfinite(d))
            # values come out in order
            assert np.all(np.diff(d) >= 0) if mode == "motifs" else np.all(np.diff(d) <= 0)
            # every reported window is outside the zones of the earlier ones
            for a in range(len(i)):
                for b in range(a):
                    assert abs(i[a] - i[b]) >= excl
                    if mode == "motifs":
                        assert abs(i[a] - j[b]) >= excl
            # exhausted only when every finite window is covered by some zone
            if len(i) < 50:
                cover = np.zeros(N, bool)
                for a in range(len(i)):
                    cover[max(0, i[a] - excl + 1):i[a] + excl] = True
                    if mode == "motifs":
                        cover[max(0, j[a] - excl + 1):j[a] + excl] = True
                assert np.all(cover | ~np.isfinite(P))
