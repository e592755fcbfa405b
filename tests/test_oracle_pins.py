"""Pins for the CPU oracle: checks against things other than the oracle itself.

Each test ties the oracle to something the paper or the mathematics fixes:
hand-derived worked examples (tests/golden), library routines (scipy cdist,
numpy corrcoef / mean / std), exact integer and rational brute force, the
paper's own incremental recurrences (Lemmas 1-3), the alternative comparator
identity of Sec. 4.4, invariants and special cases.
"""
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
from numpy.lib.stride_tricks import sliding_window_view
from scipy.spatial.distance import cdist

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# golden fixtures
# ----------------------------------------------------------------------------

def _parse_cases(path):
    series, m, cases, cur = None, None, [], None
    for raw in open(path):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "series":
            series = np.array([float(x) for x in tok[1:]])
        elif tok[0] == "m":
            m = int(tok[1])
        elif tok[0] == "case":
            kw = dict(t.split("=") for t in tok[2:])
            cur = dict(kind=tok[1], p=float(kw["p"]), excl=int(kw["excl"]), rows=[])
            cases.append(cur)
        else:
            cur["rows"].append((int(tok[0]), int(tok[1]), int(tok[2]), int(tok[3])))
    return series, m, cases


def test_golden_fig2_euclid_pnorm(oracle_mod):
    T, m, cases = _parse_cases(os.path.join(GOLDEN, "fig2_euclid_pnorm.txt"))
    assert len(cases) == 4
    for c in cases:
        P, I, Q = oracle_mod.profile(T, m, c["kind"], p=c["p"], excl=c["excl"])
        assert len(P) == len(c["rows"]) == len(T) - m + 1
        for (r, best, idx, second) in c["rows"]:
            assert I[r] == idx, (c, r)
            assert P[r] ** c["p"] == pytest.approx(best, rel=1e-12, abs=1e-12), (c, r)
            assert Q[r] ** c["p"] == pytest.approx(second, rel=1e-12, abs=1e-12), (c, r)


def _rho(tok):
    if tok == "none":
        return None
    neg = tok.startswith("-")
    t = tok[1:] if neg else tok
    if t.startswith("sqrt(") and t.endswith(")"):
        v = math.sqrt(float(Fraction(t[5:-1])))
    else:
        v = float(Fraction(t))
    return -v if neg else v


def test_golden_znorm_patterns(oracle_mod):
    path = os.path.join(GOLDEN, "znorm_patterns.txt")
    T, m, excl, rows = None, None, None, []
    for raw in open(path):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "series":
            T = np.array([float(x) for x in tok[1:]])
        elif tok[0] == "m":
            m = int(tok[1])
        elif tok[0] == "excl":
            excl = int(tok[1])
        else:
            rows.append((int(tok[0]), _rho(tok[1]), [int(x) for x in tok[2].split("|")], _rho(tok[3])))
    P, I, Q = oracle_mod.profile(T, m, "acamp", excl=excl)
    assert len(rows) == len(P)
    for r, rho_b, idx, rho_q in rows:
        if rho_b is None:
            assert math.isinf(P[r]) and I[r] == -1 and math.isinf(Q[r])
            continue
        assert I[r] in idx, r
        assert P[r] ** 2 == pytest.approx(2 * m * (1 - rho_b), abs=1e-12), r
        assert Q[r] ** 2 == pytest.approx(2 * m * (1 - rho_q), abs=1e-12), r


# ----------------------------------------------------------------------------
# library routines
# ----------------------------------------------------------------------------

def _lib_profile(S, excl, root):
    """Row minimum of a full pairwise matrix S with the exclusion band."""
    N = S.shape[0]
    idx = np.arange(N)
    S = S.copy()
    S[np.abs(idx[:, None] - idx[None, :]) < excl] = np.inf
    I = np.argmin(S, axis=1)             # first minimum = smallest j
    best = S[idx, I]
    S2 = S.copy()
    S2[idx, I] = np.inf
    second = S2.min(axis=1)
    I = np.where(np.isinf(best), -1, I)
    return root(best), I, root(second)


def _check_against(P, I, Q, Pr, Ir, Qr, rtol):
    np.testing.assert_allclose(P, Pr, rtol=rtol, atol=1e-12)
    np.testing.assert_allclose(Q, Qr, rtol=rtol, atol=1e-12)
    # indices must agree wherever the best is separated from the runner-up
    sep = (Qr - Pr) > 1e-9 * np.maximum(Pr, 1e-300)
    assert np.array_equal(I[sep], Ir[sep])


def test_diagonal_mask_matches_library(oracle_mod):
    """Partial profiles (the anytime reading of Sec. 1 / Sec. 7: stopping
    after a set of outer iterations k leaves the minimum over exactly those
    diagonals): the oracle's masked profile equals the row minimum of a
    library pairwise matrix with the unmarked diagonals removed."""
    rng = np.random.default_rng(12)
    T = np.cumsum(rng.standard_normal(300))
    m, excl = 16, 4
    W = sliding_window_view(T, m)
    N = W.shape[0]
    mask = rng.random(N) < 0.3
    idx = np.arange(N)
    off = ~mask[np.abs(idx[:, None] - idx[None, :])]

    def lib(S, root):
        S = S.copy()
        S[off] = np.inf
        return _lib_profile(S, excl, root)

    P, I, Q = oracle_mod.profile(T, m, "aamp", excl=excl, diagonals=mask)
    _check_against(P, I, Q, *lib(cdist(W, W, "sqeuclidean"), np.sqrt), 1e-11)
    P, I, Q = oracle_mod.profile(T, m, "pnorm", p=3.0, excl=excl, diagonals=mask)
    _check_against(P, I, Q, *lib(cdist(W, W, "minkowski", p=3.0), lambda x: x), 1e-10)
    P, I, Q = oracle_mod.profile(T, m, "acamp", excl=excl, diagonals=mask)
    r = np.corrcoef(W)
    _check_against(P, I, Q, *lib(2.0 * m * (1.0 - r), lambda x: np.sqrt(np.maximum(x, 0))),
                   1e-8)


def test_diagonal_mask_union_and_extremes(oracle_mod):
    rng = np.random.default_rng(13)
    T = np.cumsum(rng.standard_normal(260))
    m, excl = 12, 3
    N = len(T) - m + 1
    full = oracle_mod.profile(T, m, "acamp", excl=excl)
    every = oracle_mod.profile(T, m, "acamp", excl=excl, diagonals=np.ones(N, bool))
    for a, b in zip(full, every):
        assert np.array_equal(a, b)
    P0, I0, _ = oracle_mod.profile(T, m, "aamp", excl=excl, diagonals=np.zeros(N, bool))
    assert np.all(np.isinf(P0)) and np.all(I0 == -1)
    # one diagonal k: the partner of row i is i - k or i + k
    k = 37
    one = np.zeros(N, bool)
    one[k] = True
    P1, I1, _ = oracle_mod.profile(T, m, "aamp", excl=excl, diagonals=one)
    i = np.arange(N)
    assert np.all((I1 == i - k) | (I1 == i + k))
    for r in (0, 5, N - 1, N // 2):
        assert P1[r] == pytest.approx(np.linalg.norm(T[r:r + m] - T[I1[r]:I1[r] + m]), rel=1e-12)
    # the union of two masks takes the smaller of the two profiles
    A = rng.random(N) < 0.2
    B = rng.random(N) < 0.2
    PA, _, _ = oracle_mod.profile(T, m, "aamp", excl=excl, diagonals=A)
    PB, _, _ = oracle_mod.profile(T, m, "aamp", excl=excl, diagonals=B)
    PU, _, _ = oracle_mod.profile(T, m, "aamp", excl=excl, diagonals=A | B)
    assert np.array_equal(PU, np.minimum(PA, PB))


@pytest.mark.parametrize("seed", [0, 1])
def test_scipy_cdist_euclid_and_pnorm(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    T = np.cumsum(rng.standard_normal(300))
    m, excl = 16, 4
    W = sliding_window_view(T, m)
    P, I, Q = oracle_mod.profile(T, m, "aamp", excl=excl)
    _check_against(P, I, Q, *_lib_profile(cdist(W, W, "sqeuclidean"), excl, np.sqrt), 1e-11)
    P, I, Q = oracle_mod.profile(T, m, "pnorm", p=1.0, excl=excl)
    _check_against(P, I, Q, *_lib_profile(cdist(W, W, "cityblock"), excl, lambda x: x), 1e-11)
    P, I, Q = oracle_mod.profile(T, m, "pnorm", p=3.0, excl=excl)
    _check_against(P, I, Q, *_lib_profile(cdist(W, W, "minkowski", p=3.0), excl, lambda x: x), 1e-10)
    # p = 2 is the Euclidean special case (Sec. 3.4)
    P, I, Q = oracle_mod.profile(T, m, "pnorm", p=2.0, excl=excl)
    _check_against(P, I, Q, *_lib_profile(cdist(W, W, "euclidean"), excl, lambda x: x), 1e-11)
    P, I, Q = oracle_mod.profile(T, m, "pnorm", p=2.5, excl=excl)
    _check_against(P, I, Q, *_lib_profile(cdist(W, W, "minkowski", p=2.5), excl, lambda x: x), 1e-10)


def test_numpy_corrcoef_znorm(oracle_mod):
    """Lemma 3 closed form: DZ^2 = 2m(1 - r), r = Pearson correlation."""
    rng = np.random.default_rng(7)
    T = np.cumsum(rng.standard_normal(400))
    T[100:160] = T[100]                  # a constant run (zero std windows)
    m, excl = 20, 5
    W = sliding_window_view(T, m)
    isconst = np.all(W == W[:, :1], axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        R = np.corrcoef(W)
    S = 2 * m * (1 - R)
    S[isconst, :] = np.inf
    S[:, isconst] = np.inf
    Pr, Ir, Qr = _lib_profile(S, excl, lambda x: np.sqrt(np.maximum(x, 0)))
    P, I, Q = oracle_mod.profile(T, m, "acamp", excl=excl)
    assert np.array_equal(np.isinf(P), np.isinf(Pr))
    fin = ~np.isinf(P)
    np.testing.assert_allclose(P[fin] ** 2, Pr[fin] ** 2, atol=1e-9)
    assert np.all(I[~fin] == -1)
    sep = fin & ((Qr ** 2 - Pr ** 2) > 1e-8)
    assert np.array_equal(I[sep], Ir[sep])


def test_numpy_window_stats(oracle_mod):
    rng = np.random.default_rng(8)
    T = rng.normal(3.0, 2.0, 500)
    T[200:260] = 1.25
    m = 32
    mu, sg, c = oracle_mod.window_stats(T, m)
    W = sliding_window_view(T, m)
    np.testing.assert_allclose(mu, W.mean(axis=1), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(sg, W.std(axis=1, ddof=0), rtol=1e-12, atol=1e-13)
    assert np.array_equal(c, np.all(W == W[:, :1], axis=1))


# ----------------------------------------------------------------------------
# exact integer / rational brute force
# ----------------------------------------------------------------------------

def _exact_rows(vals, m, excl, pair):
    N = len(vals) - m + 1
    out = []
    for i in range(N):
        cands = [(pair(i, j), j) for j in range(N) if abs(i - j) >= excl]
        cands = [c for c in cands if c[0] is not None]
        if not cands:
            out.append((None, -1, None, []))
            continue
        best = min(c[0] for c in cands)
        ties = [j for s, j in cands if s == best]
        rest = [s for s, j in cands if j != ties[0]]
        out.append((best, ties[0], min(rest) if rest else None, ties))
    return out


@pytest.mark.parametrize("excl", [1, 2, 3])
def test_exact_integer_euclid_pnorm(oracle_mod, excl):
    rng = np.random.default_rng(11 + excl)
    vals = [int(v) for v in rng.integers(-4, 5, 40)]
    T = np.array(vals, dtype=np.float64)
    m = 5
    for kind, p in (("aamp", 2), ("pnorm", 1), ("pnorm", 3)):
        def pair(i, j, p=p):
            return sum(abs(vals[i + l] - vals[j + l]) ** p for l in range(m))
        exact = _exact_rows(vals, m, excl, pair)
        P, I, Q = oracle_mod.profile(T, m, kind, p=float(p), excl=excl)
        for r, (best, j, second, _) in enumerate(exact):
            assert I[r] == j, (kind, p, r)          # smallest j among exact ties
            if p == 2:
                assert P[r] == math.sqrt(best)     # integer sum, correctly rounded root
                assert Q[r] == math.sqrt(second)
            else:
                assert P[r] ** p == pytest.approx(best, rel=1e-13, abs=0)
                assert Q[r] ** p == pytest.approx(second, rel=1e-13, abs=0)


def test_exact_rational_znorm(oracle_mod):
    getcontext().prec = 50
    rng = np.random.default_rng(21)
    vals = [int(v) for v in rng.integers(-3, 4, 36)]
    vals[10:18] = [2] * 8                    # a constant stretch
    T = np.array(vals, dtype=np.float64)
    m, excl = 4, 2
    N = len(vals) - m + 1

    def centred(i):
        w = [Fraction(v) for v in vals[i:i + m]]
        mu = sum(w) / m
        return [x - mu for x in w]

    C = [centred(i) for i in range(N)]
    SS = [sum(x * x for x in c) for c in C]

    def dz2(i, j):
        if SS[i] == 0 or SS[j] == 0:
            return None
        cov = sum(a * b for a, b in zip(C[i], C[j]))
        rho = Decimal(cov.numerator) / Decimal(cov.denominator) / (
            Decimal((SS[i] * SS[j]).numerator) / Decimal((SS[i] * SS[j]).denominator)).sqrt()
        return 2 * m * (1 - rho)

    exact = _exact_rows(vals, m, excl, dz2)
    P, I, Q = oracle_mod.profile(T, m, "acamp", excl=excl)
    for r, (best, j, second, ties) in enumerate(exact):
        if best is None:
            assert math.isinf(P[r]) and I[r] == -1
            continue
        assert P[r] ** 2 == pytest.approx(float(best), abs=1e-12)
        # exact rational ties may be split by rounding: any tied index is valid
        near = [jj for jj in range(N) if abs(r - jj) >= excl and dz2(r, jj) is not None
                and abs(dz2(r, jj) - best) < Decimal("1e-12")]
        assert I[r] in near, r


# ----------------------------------------------------------------------------
# the paper's incremental recurrences (a different computation of the same
# quantities) must agree with the brute force
# ----------------------------------------------------------------------------

def _diagonal_sweep(T, m, excl, kind, p=2.0):
    """Diagonal-wise incremental profile written from Lemmas 1-3 and the
    description of AAMP / ACAMP (Secs. 3.2, 3.4, 4.2): for each diagonal
    k = j - i the first pair is summed directly, every later pair on the
    diagonal is updated in O(1), and each pair updates both its row and its
    column. ACAMP uses the five running sums of Sec. 4.1."""
    n = len(T)
    N = n - m + 1
    best = np.full(N, np.inf)
    arg = np.full(N, -1, dtype=np.int64)

    def upd(i, v, j):
        if v < best[i] or (v == best[i] and j < arg[i]):
            best[i], arg[i] = v, j

    for k in range(excl, N):
        if kind == "znorm":
            A = T[0:m].sum(); B = T[k:k + m].sum()
            AA = (T[0:m] ** 2).sum(); BB = (T[k:k + m] ** 2).sum()
            C = (T[0:m] * T[k:k + m]).sum()
        else:
            d = np.abs(T[0:m] - T[k:k + m])
            S = (d ** p).sum()
        for i in range(0, N - k):
            j = i + k
            if i > 0:
                if kind == "znorm":
                    a_out, a_in = T[i - 1], T[i + m - 1]
                    b_out, b_in = T[j - 1], T[j + m - 1]
                    A += a_in - a_out; B += b_in - b_out
                    AA += a_in ** 2 - a_out ** 2; BB += b_in ** 2 - b_out ** 2
                    C += a_in * b_in - a_out * b_out
                else:
                    S += abs(T[i + m - 1] - T[j + m - 1]) ** p - abs(T[i - 1] - T[j - 1]) ** p
            if kind == "znorm":
                den = (AA - A * A / m) * (BB - B * B / m)
                v = 2 * m * (1 - (C - A * B / m) / math.sqrt(den))
            else:
                v = S
            upd(i, v, j)
            upd(j, v, i)
    root = (lambda s: s ** (1.0 / p)) if kind != "znorm" else (lambda s: math.sqrt(max(s, 0.0)))
    return np.array([root(b) if np.isfinite(b) else np.inf for b in best]), arg


@pytest.mark.parametrize("kind,p", [("aamp", 2.0), ("pnorm", 1.0), ("pnorm", 3.0), ("znorm", 2.0)])
def test_incremental_recurrences_match(oracle_mod, kind, p):
    rng = np.random.default_rng(31)
    T = rng.normal(0.0, 1.0, 160)
    m, excl = 12, 3
    Pi, Ii = _diagonal_sweep(T, m, excl, kind if kind != "aamp" else "pnorm", p)
    P, I, Q = oracle_mod.profile(T, m, "acamp" if kind == "znorm" else kind, p=p, excl=excl)
    np.testing.assert_allclose(Pi, P, rtol=1e-9, atol=1e-9)
    sep = (Q - P) > 1e-7 * P
    assert np.array_equal(Ii[sep], I[sep])


def test_alternative_comparator_identity(oracle_mod):
    """Sec. 4.4: with F built from the five sums (its denominator's B_j read as
    B_j^2), 2m + 2 sign(F) sqrt|F| equals the squared z-normalized distance."""
    rng = np.random.default_rng(41)
    T = np.cumsum(rng.standard_normal(200))
    m, excl = 16, 4
    P, I, Q = oracle_mod.profile(T, m, "acamp", excl=excl)
    for i in range(0, len(P), 7):
        j = int(I[i])
        a, b = T[i:i + m], T[j:j + m]
        A, B, AA, BB, C = a.sum(), b.sum(), (a * a).sum(), (b * b).sum(), (a * b).sum()
        X = A * B - m * C
        F = X * abs(X) / ((AA - A * A / m) * (BB - B * B / m))
        dz2 = 2 * m + 2 * np.sign(F) * math.sqrt(abs(F))
        assert dz2 == pytest.approx(P[i] ** 2, rel=1e-7, abs=1e-7)


# ----------------------------------------------------------------------------
# invariants and special cases
# ----------------------------------------------------------------------------

def test_translation_scaling_invariance(oracle_mod):
    rng = np.random.default_rng(51)
    T = rng.uniform(-1, 1, 300)
    m, excl = 10, 3
    for kind, p in (("aamp", 2.0), ("pnorm", 1.0), ("pnorm", 3.0)):
        P, I, Q = oracle_mod.profile(T, m, kind, p=p, excl=excl)
        P2, I2, _ = oracle_mod.profile(T + 7.5, m, kind, p=p, excl=excl)
        P3, I3, _ = oracle_mod.profile(-2.0 * T, m, kind, p=p, excl=excl)
        np.testing.assert_allclose(P2, P, rtol=1e-10)
        np.testing.assert_allclose(P3, 2.0 * P, rtol=1e-12)
        sep = (Q - P) > 1e-8 * P
        assert np.array_equal(I2[sep], I[sep]) and np.array_equal(I3[sep], I[sep])
    P, I, Q = oracle_mod.profile(T, m, "acamp", excl=excl)
    P2, I2, _ = oracle_mod.profile(3.0 * T - 11.0, m, "acamp", excl=excl)
    np.testing.assert_allclose(P2, P, rtol=1e-8, atol=1e-8)
    sep = (Q - P) > 1e-6 * P
    assert np.array_equal(I2[sep], I[sep])


def test_reversal(oracle_mod):
    rng = np.random.default_rng(52)
    T = np.cumsum(rng.standard_normal(250))
    m, excl = 9, 3
    for kind in ("aamp", "acamp"):
        P, I, Q = oracle_mod.profile(T, m, kind, excl=excl)
        Pr, Ir, _ = oracle_mod.profile(T[::-1].copy(), m, kind, excl=excl)
        N = len(P)
        np.testing.assert_allclose(Pr[::-1], P, rtol=1e-9, atol=1e-12)
        sep = (Q - P) > 1e-7 * P
        assert np.array_equal((N - 1 - Ir[::-1])[sep], I[sep])


def test_constant_series(oracle_mod):
    T = np.full(60, 3.25)
    m, excl = 8, 2
    P, I, Q = oracle_mod.profile(T, m, "aamp", excl=excl)
    N = len(P)
    assert np.all(P == 0.0)
    expect = np.array([0 if i >= excl else i + excl for i in range(N)])
    assert np.array_equal(I, expect)
    P, I, Q = oracle_mod.profile(T, m, "acamp", excl=excl)
    assert np.all(np.isinf(P)) and np.all(I == -1)


def test_no_admissible_pair(oracle_mod):
    T = np.arange(10, dtype=np.float64)
    P, I, Q = oracle_mod.profile(T, 6, "aamp", excl=5)   # N = 5 <= excl
    assert np.all(np.isinf(P)) and np.all(I == -1) and np.all(np.isinf(Q))
    P, I, Q = oracle_mod.profile(T, 10, "aamp", excl=1)  # a single window
    assert len(P) == 1 and np.isinf(P[0]) and I[0] == -1


def test_planted_copies(oracle_mod):
    rng = np.random.default_rng(61)
    T = np.cumsum(rng.standard_normal(500))
    m, a, b = 24, 60, 340
    T[b:b + m] = T[a:a + m]
    P, I, Q = oracle_mod.profile(T, m, "aamp", excl=6)
    assert P[a] == 0.0 and I[a] == b and P[b] == 0.0 and I[b] == a
    T2 = T.copy()
    T2[b:b + m] = 0.5 * T[a:a + m] - 3.0     # exact affine copy
    P, I, Q = oracle_mod.profile(T2, m, "acamp", excl=6)
    assert P[a] < 1e-6 and I[a] == b and I[b] == a


def test_sampled_rows_match_full(oracle_mod):
    rng = np.random.default_rng(71)
    T = np.cumsum(rng.standard_normal(300))
    m = 16
    P, I, Q = oracle_mod.profile(T, m, "acamp", excl=4)
    rows = np.array([0, 5, 77, 200, len(P) - 1])
    Ps, Is, Qs = oracle_mod.profile(T, m, "acamp", excl=4, rows=rows)
    assert np.array_equal(Ps, P[rows]) and np.array_equal(Is, I[rows]) and np.array_equal(Qs, Q[rows])
    for r in rows:
        assert oracle_mod.distance(T, m, r, I[r], "acamp") == pytest.approx(P[r], rel=1e-12)


def test_rejects_bad_arguments(oracle_mod):
    T = np.arange(20, dtype=np.float64)
    with pytest.raises(ValueError):
        oracle_mod.profile(T, 0, "aamp")
    with pytest.raises(ValueError):
        oracle_mod.profile(T, 5, "pnorm", p=0.5)
    with pytest.raises(ValueError):
        oracle_mod.profile(T, 5, "aamp", excl=0)
    with pytest.raises(ValueError):
        oracle_mod.profile(T, 5, "aamp", rows=[100])


def test_znorm_affine_invariance_far_from_zero(oracle_mod):
    """DZ is invariant under t -> a t + c (Def. 2.7). With c large against the
    window deviations (c = 1e5, a = 1e-3, m = 128), windows at the edges of
    constant runs are near-constant; their distances survive only if the
    window mean is evaluated without offset-scale rounding. (A plain running
    sum of the samples gives differences of 4.5e-6 here; the shifted sum,
    4.7e-8.)"""
    rng = np.random.default_rng(44)
    T = np.cumsum(rng.standard_normal(900))
    T[200:430] = T[200]
    T[550:780] = T[550]
    m, excl = 128, 32
    P, I, Q = oracle_mod.profile(T, m, "acamp", excl=excl)
    P2, I2, Q2 = oracle_mod.profile(1e-3 * T + 1e5, m, "acamp", excl=excl)
    fin = np.isfinite(P)
    assert np.array_equal(fin, np.isfinite(P2))
    assert np.max(np.abs(P[fin] - P2[fin])) < 1e-6
