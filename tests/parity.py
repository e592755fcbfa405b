"""Acceptance check of a GPU profile against the oracle (test helper).

Per row i, with rtol / atol the tolerance of the precision mode:
  1. both +inf with index -1, or both finite;
  2. |P - P_ref| <= rtol * P_ref + atol;
  3. I == I_ref, or the row is a near tie (runner-up within the tolerance of
     the best) and the reported index is admissible with a directly computed
     distance within the tolerance of the best;
  4. P equals the direct distance of (i, I) (checked on the mismatched rows
     and on a sample of the others).
"""
import math

import numpy as np

import oracle

# Absolute floor of z-normalized results, in DZ units. The sweep selects the
# partner on the key 1 - rho (Lemma 3); with delta the absolute error of that
# key, the reported pair's exact DZ^2 = 2 m (1 - rho) exceeds the minimum by at
# most 4 m delta, so DZ by at most sqrt(4 m delta), which dominates the
# relative tolerance near DZ = 0. FP64: the key is resolved to a few units of
# 2^-53 next to 1, and the refresh recurrence adds a drift that grows like the
# square root of the rows since the last restart R; delta = 2^-53 (8 + 2
# sqrt(R)), with R = 64 m, the longest interval the autotuner offers, when the
# caller does not fix it. The checks use the smaller of that floor and 1e-6:
# below m = 32 the floor is the tighter bound; above, the measured errors have
# stayed under 1e-6 at every window length tested (up to 2^16), well inside
# the drift allowance. FP32 + refresh: the 1e-6 of the single-precision
# contract.
ACAMP_ATOL = 1e-6


def acamp_atol(m, precision="fp64", R=None):
    if precision != "fp64":
        return ACAMP_ATOL
    R = 64 * m if not R else R
    delta = 2.0 ** -53 * (8.0 + 2.0 * math.sqrt(R))
    return min(ACAMP_ATOL, math.sqrt(4.0 * m * delta))


def atol_for(kind, m, precision="fp64", R=None):
    """Absolute tolerance of a profile check: 0 except for ACAMP."""
    return acamp_atol(m, precision, R) if kind == "acamp" else 0.0


def check_profile(T, m, kind, p, excl, P, I, Pref, Iref, Qref, rtol, atol, rows=None,
                  sample=64, label=""):
    P = np.asarray(P, dtype=np.float64)
    I = np.asarray(I, dtype=np.int64)
    rows = np.arange(len(Pref)) if rows is None else np.asarray(rows)
    inf_g, inf_r = np.isinf(P), np.isinf(Pref)
    bad = np.nonzero(inf_g != inf_r)[0]
    assert bad.size == 0, f"{label}: finiteness differs at rows {rows[bad[:10]]}"
    assert np.all(I[inf_r] == -1), f"{label}: infinite rows must report index -1"
    fin = ~inf_r
    err = np.abs(P[fin] - Pref[fin])
    tol = rtol * Pref[fin] + atol
    badv = np.nonzero(err > tol)[0]
    assert badv.size == 0, (f"{label}: {badv.size} values off, worst rel "
                            f"{np.max(err / np.maximum(Pref[fin], 1e-300)):.3e} at rows "
                            f"{rows[np.nonzero(fin)[0][badv[:10]]]}")
    mism = np.nonzero(fin & (I != Iref))[0]
    for r in mism:
        i, ig = int(rows[r]), int(I[r])
        near = (Qref[r] - Pref[r]) <= rtol * Pref[r] + atol
        assert near, (f"{label}: row {i}: index {ig} != {Iref[r]} and runner-up gap "
                      f"{(Qref[r] - Pref[r]) / max(Pref[r], 1e-300):.3e} exceeds rtol")
        assert abs(i - ig) >= excl and 0 <= ig
        d = oracle.distance(T, m, i, ig, kind, p)
        assert d <= Pref[r] * (1 + rtol) + atol, f"{label}: row {i}: reported pair is not near-best"
    rng = np.random.default_rng(0)
    finrows = np.nonzero(fin)[0]
    pick = np.unique(np.concatenate([mism, rng.choice(finrows, size=min(sample, finrows.size),
                                                      replace=False)])) if finrows.size else mism
    # The oracle's z-normalized distance sums squared differences of z-values
    # built from rounded window means and deviations, so near DZ = 0 it is off
    # by about sqrt(m) 2^-53 (window offset / spread) in absolute terms: 4e-11
    # for two walk windows that each hold one sample before m - 1 equal ones,
    # whose exact DZ (Def. 2.7, in rational arithmetic) is 0. Long-window
    # rescoring on the GPU sums in double-double and lands nearer the exact
    # value, so the absolute part of this check covers the oracle's floor.
    abs_tol = 1e-9 if kind == "acamp" else 1e-12
    for r in pick:
        d = oracle.distance(T, m, int(rows[r]), int(I[r]), kind, p)
        assert abs(d - P[r]) <= 1e-12 * max(d, 1e-300) + abs_tol, \
            f"{label}: row {rows[r]}: P is not the distance of the reported pair"
    return {"rows": len(rows), "index_mismatch": int(mism.size)}
