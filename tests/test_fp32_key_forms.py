"""Why the FP32 z-normalized sweep carries the centred cross sum, not 1 - rho:
a host replay at the oracle's winners of the 131072-sample walk (CPU only).

Near a good match the key 1 - rho is small, and the sweep forms it next to 1
from the running cross sum S (Lemma 3's numerator), so its single-precision
error is absolute: about u |rho| per rounding plus the sum's drift, u |S| per
step. Carrying e = 1 - rho itself would make the rounding relative to e on a
clean diagonal:
    e' = e r + (1 - r) - P_i Q_j - P_j Q_i,
    r = (invn_i' / invn_i)(invn_j' / invn_j),  P = df invn,  Q = dg invn
(df, dg the streams of the centred update; one operation more per pair). On
this walk, though, the pairs that fail the single-precision self-check are
those whose diagonal crosses windows of very different norm (the planted
constant runs and the walk's own amplitude swings), where the ratios r and
the normalised increments are large; there the e form drifts as much or more.
Each winner pair is replayed from an exact FP64 start a random number of rows
back (less than the refresh interval), in both forms, and checked with the
sweep's own self-check tolerance. The e form certifies no more rows."""
import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

import workloads as W
from tests import fullsize_refs as R

SELF_CHECK, SELF_CHECK_ABS = 1.5e-4, 2.5e-7   # the FP32 self-check of the finalize step
f32 = np.float32


def _fma32(a, b, c):
    # product of two floats exact in float64, one rounding of the sum (up to
    # a rare double rounding), then to float
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def _streams(T, m):
    n = len(T)
    N = n - m + 1
    Wv = sliding_window_view(T, m)
    mu = Wv.mean(axis=1)
    ss = ((Wv - mu[:, None]) ** 2).sum(axis=1)
    const = (Wv == Wv[:, :1]).all(axis=1)
    invn = np.where(const, 0.0, 1.0 / np.sqrt(np.where(const, 1.0, ss)))
    df = np.zeros(N)
    dg = np.zeros(N)
    df[1:] = 0.5 * (T[m:n] - T[:N - 1])
    dg[1:] = (T[m:n] - mu[1:]) + (T[:N - 1] - mu[:-1])
    prev = np.concatenate([[0.0], invn[:-1]])
    ratio = np.where(prev > 0, invn / np.where(prev > 0, prev, 1.0), 1.0)
    return Wv, mu, invn, df, dg, ratio


def test_carrying_one_minus_rho_certifies_no_more_rows():
    T, m, _ = W.rw128k()
    T = np.asarray(T, dtype=np.float64)
    ref = R.load("rw128k_acamp", T=T)
    ok = np.isfinite(ref["P"]) & (ref["I"] >= 0)
    rows, P, I = ref["rows"][ok], ref["P"][ok], ref["I"][ok]
    ii, jj = np.minimum(rows, I), np.maximum(rows, I)
    e_true = P ** 2 / (2 * m)
    Wv, mu, invn, df, dg, ratio = _streams(T, m)
    s = 1.0 - ratio
    Pw, Qw = df * invn, dg * invn

    refresh = 2048
    L = np.minimum(np.random.default_rng(3).integers(0, refresh, size=len(ii)), ii)
    i0, j0 = ii - L, jj - L
    cov0 = np.einsum("ij,ij->i", Wv[i0] - mu[i0, None], Wv[j0] - mu[j0, None])
    S = cov0.astype(f32)
    both = (invn[i0] > 0) & (invn[j0] > 0)
    E = np.where(both, 1.0 - cov0 * invn[i0] * invn[j0], 1.0).astype(f32)
    c = lambda v: v.astype(f32)
    for t in range(1, int(L.max()) + 1):
        act = L >= t
        i = np.where(act, i0 + t, ii)
        j = np.where(act, j0 + t, jj)
        # covariance form: the sweep's two fused updates
        Sn = _fma32(c(df[i]), c(dg[j]), S)
        Sn = _fma32(c(df[j]), c(dg[i]), Sn)
        S = np.where(act, Sn, S)
        # 1 - rho form
        t1 = _fma32(c(ratio[i]), c(s[j]), c(s[i]))
        t2 = _fma32(c(-Pw[i]), c(Qw[j]), t1)
        t3 = _fma32(c(-Qw[i]), c(Pw[j]), t2)
        En = _fma32(E, (c(ratio[i]) * c(ratio[j])).astype(f32), t3)
        E = np.where(act, En, E)
    key_s = _fma32((S * c(invn[ii])).astype(f32), c(-invn[jj]), np.ones(len(S), dtype=f32))

    def failed(key):
        return ~(np.abs(key.astype(np.float64) - e_true) <= SELF_CHECK * e_true + SELF_CHECK_ABS)

    fail_s, fail_e = int(failed(key_s).sum()), int(failed(E).sum())
    print(f"winners {len(ii)}: self-check fails {fail_s} (covariance form), {fail_e} (1 - rho form)")
    # both forms fail a few percent of the winners at this interval ...
    assert 0.01 * len(ii) < fail_s < 0.1 * len(ii)
    # ... and carrying 1 - rho does not reduce that
    assert fail_e >= fail_s, (fail_e, fail_s)
