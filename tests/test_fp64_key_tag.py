"""Why the FP64 Euclidean sweep tags a copy of its running sum (CPU only).

The band kernels compare packed keys whose low mantissa bits hold the
partner's diagonal within the band (9 bits for 512 diagonals). For the
Euclidean distance the key is the running sum S of Lemma 1 itself, so the tag
is written into a copy of S, which costs one register move per pair. Writing
it into S in place would save that move, but every step would then replace
S's low 9 bits with the same value: a perturbation of up to 2^-43 relative
whose sign does not average out. Replayed on the host at the oracle's winners
of the 131072-sample walk, from exact starts less than R = 4096 rows back,
that raises the error of S at the winner by orders of magnitude over plain
FP64 accumulation."""
import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

import workloads as W
from tests import fullsize_refs as R


def _tag(S, d):
    b = S.view(np.uint64)
    return ((b & ~np.uint64(511)) | d.astype(np.uint64)).view(np.float64)


def test_tag_in_place_breaks_the_fp64_sum():
    T, m, _ = W.rw128k()
    T = np.asarray(T, dtype=np.float64)
    n = len(T)
    N = n - m + 1
    ref = R.load("rw128k_aamp", T=T)
    ok = np.isfinite(ref["P"]) & (ref["I"] >= 0) & (ref["P"] > 0)
    rows, P, I = ref["rows"][ok], ref["P"][ok], ref["I"][ok]
    ii, jj = np.minimum(rows, I), np.maximum(rows, I)
    S_true = P ** 2
    # the recurrence's streams (Lemma 1): u = t[j+m-1] - t[j-1], v = t[j+m-1] + t[j-1]
    u = np.zeros(N)
    v = np.zeros(N)
    u[1:] = T[m:n] - T[:N - 1]
    v[1:] = T[m:n] + T[:N - 1]
    Wv = sliding_window_view(T, m)
    rng = np.random.default_rng(5)
    L = np.minimum(rng.integers(0, 4096, size=len(ii)), ii)
    i0, j0 = ii - L, jj - L
    c = T[i0][:, None]
    S0 = (((Wv[i0] - c) - (Wv[j0] - c)) ** 2).sum(axis=1)
    plain, tagged = S0.copy(), S0.copy()
    d = rng.integers(0, 512, size=len(ii))
    for t in range(1, int(L.max()) + 1):
        act = L >= t
        i = np.where(act, i0 + t, ii)
        j = np.where(act, j0 + t, jj)
        inc = (u[i] - u[j]) * (v[i] - v[j])
        plain = np.where(act, plain + inc, plain)
        tagged = np.where(act, _tag(tagged + inc, d), tagged)
    e_plain = np.percentile(np.abs(plain - S_true) / S_true, 99)
    e_tag = np.percentile(np.abs(tagged - S_true) / S_true, 99)
    print(f"99th percentile relative error of S: plain {e_plain:.2e}, tag in place {e_tag:.2e}")
    assert e_plain < 1e-6
    assert e_tag > 1e3 * e_plain
