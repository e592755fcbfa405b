"""Motifs and discords from a matrix profile (test infrastructure only).

The two uses of a matrix profile that Sec. 1 gives for it: motifs, the most
similar pairs of subsequences (the smallest profile values), and discords,
the subsequences farthest from every other one (the largest profile
values). A profile reports every pair twice, (i, I[i]) and (I[i], i), and
neighbouring windows of a good match are good matches too, so the extraction
is greedy with an exclusion zone:

* motifs: k times, take the not yet excluded window i with the smallest
  finite P[i] (ties: the smallest i), report (i, I[i], P[i]) and exclude
  every window x with |x - i| < excl or |x - I[i]| < excl;
* discords: k times, take the not yet excluded window i with the largest
  finite P[i] (ties: the smallest i), report it and exclude every window x
  with |x - i| < excl.

It stops early when no finite candidate is left. Plain numpy, one round at a
time; it shares nothing with the GPU path.
"""
from __future__ import annotations

import numpy as np


def topk(P, I, k: int, excl: int, mode: str = "motifs"):
    """Returns (idx, partner, value) arrays of length <= k."""
    P = np.asarray(P, dtype=np.float64)
    I = np.asarray(I, dtype=np.int64)
    N = len(P)
    alive = np.isfinite(P)
    out_i, out_j, out_d = [], [], []
    for _ in range(k):
        cand = np.nonzero(alive)[0]
        if cand.size == 0:
            break
        vals = P[cand]
        best = vals.min() if mode == "motifs" else vals.max()
        i = int(cand[vals == best][0])          # smallest index among exact ties
        j = int(I[i])
        out_i.append(i)
        out_j.append(j)
        out_d.append(float(P[i]))
        alive[max(0, i - excl + 1):min(N, i + excl)] = False
        if mode == "motifs" and 0 <= j < N:
            alive[max(0, j - excl + 1):min(N, j + excl)] = False
    return (np.array(out_i, dtype=np.int64), np.array(out_j, dtype=np.int64),
            np.array(out_d, dtype=np.float64))
