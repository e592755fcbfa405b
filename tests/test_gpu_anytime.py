"""GPU parity of partial (anytime) sweeps (mp_anytime): the profile over a set
of diagonal groups equals the oracle's profile restricted to those diagonals
(1e-9 relative; for ACAMP the absolute floor of tests/parity.py; ties
allowed), resumed calls give the profile over the union, and all groups give
the full profile."""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import atol_for, check_profile

pytestmark = pytest.mark.gpu

G_W = 512


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


def _mask(N, excl, groups):
    """Diagonals d of the listed groups: d >= excl, (d - excl) // 512 listed."""
    mask = np.zeros(N, dtype=bool)
    for g in groups:
        lo = excl + G_W * int(g)
        mask[lo:min(lo + G_W, N)] = True
    return mask


def _series(seed, n, kind):
    rng = np.random.default_rng(seed)
    T = np.cumsum(rng.standard_normal(n))
    if kind == "acamp":
        T[n // 3:n // 3 + 120] = T[n // 3]          # a constant run
        T[2 * n // 3:2 * n // 3 + 90] = T[2 * n // 3]
    return T


def _check(T, m, kind, p, excl, P, I, groups, label, rows=None):
    N = len(T) - m + 1
    mask = _mask(N, excl, groups)
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl, diagonals=mask, rows=rows)
    P = P.cpu().numpy()
    I = I.cpu().numpy()
    if rows is not None:
        P, I = P[rows], I[rows]
    check_profile(T, m, kind, p, excl, P, I, Pr, Ir, Qr, 1e-9, atol_for(kind, m), rows=rows,
                  label=label)
    # every reported partner lies on a swept diagonal
    fin = I >= 0
    r = np.arange(N) if rows is None else np.asarray(rows)
    assert np.all(mask[np.abs(r[fin] - I[fin])]), f"{label}: partner off the swept diagonals"


CASES = [("aamp", 2.0), ("acamp", 2.0), ("pnorm", 1.0), ("pnorm", 3.0), ("pnorm", 2.5)]


@pytest.mark.parametrize("kind,p", CASES)
def test_groups_match_oracle(mp, kind, p):
    import torch
    n, m = 6000, 32
    excl = W.excl_default(m)
    T = _series(3, n, kind)
    G = mp.anytime_groups(n, m, excl)
    assert G == 12
    rng = np.random.default_rng(5)
    groups = rng.choice(G, size=5, replace=False)
    groups = np.append(groups, G - 1) if G - 1 not in groups else groups   # the ragged last group
    _note(f"anytime {kind} p={p} groups={sorted(groups.tolist())}")
    Td = torch.as_tensor(T, device="cuda")
    P, I = mp.anytime(Td, m, groups, kind=kind, p=p, excl=excl)
    _check(T, m, kind, p, excl, P, I, groups, f"any-{kind}{p}")


@pytest.mark.parametrize("force", [1, 2])
@pytest.mark.parametrize("kind", ["acamp", "aamp"])
def test_exact_search_keeps_to_the_groups(mp, kind, force):
    """Every row through the exact search (test hook MP_FORCE_FALLBACK): the
    search scores only columns on the call's diagonal groups."""
    import torch
    n, m = 5000, 24
    excl = W.excl_default(m)
    T = _series(9, n, kind)
    groups = [1, 4, 6]
    _note(f"anytime exact search {kind} force={force}")
    os.environ["MP_FORCE_FALLBACK"] = str(force)
    try:
        P, I = mp.anytime(torch.as_tensor(T, device="cuda"), m, groups, kind=kind, excl=excl)
        torch.cuda.synchronize()
    finally:
        del os.environ["MP_FORCE_FALLBACK"]
    _check(T, m, kind, 2.0, excl, P, I, groups, f"any-fb{force}-{kind}")


@pytest.mark.parametrize("kind", ["aamp", "acamp"])
def test_resume_gives_the_union(mp, kind):
    import torch
    n, m = 6500, 40
    excl = W.excl_default(m)
    T = _series(11, n, kind)
    Td = torch.as_tensor(T, device="cuda")
    A, B = [0, 3, 7], [2, 3, 10, 11]
    _note(f"anytime resume {kind}")
    P, I = mp.anytime(Td, m, A, kind=kind, excl=excl)
    _check(T, m, kind, 2.0, excl, P, I, A, f"any-A-{kind}")
    P_a = P.clone()
    mp.anytime(Td, m, B, kind=kind, excl=excl, P=P, I=I)
    _check(T, m, kind, 2.0, excl, P, I, sorted(set(A) | set(B)), f"any-AB-{kind}")
    assert torch.all(P <= P_a).item(), "a resumed profile never gets worse"
    # nothing more: resuming with no groups leaves P, I as they are
    P_ab, I_ab = P.clone(), I.clone()
    mp.anytime(Td, m, [], kind=kind, excl=excl, P=P, I=I)
    assert torch.equal(P, P_ab) and torch.equal(I, I_ab)


@pytest.mark.parametrize("kind", ["acamp", "aamp"])
def test_long_windows_groups_and_resume(mp, kind):
    """m = 2048: the partial sweep's rows go through the long-window
    statistics and rescoring (anchors per run of a common winner diagonal);
    rows with no candidate on the called groups stay +inf. Two calls, then
    the union, on sampled rows and on the rows around the constant runs."""
    import torch
    n, m = 12000, 2048
    excl = W.excl_default(m)
    T = _series(21, n, kind)
    N = n - m + 1
    G = mp.anytime_groups(n, m, excl)
    A, B = [0, 2, G - 1], [1, 5]
    rows = np.unique(np.concatenate([W.sample_rows(N, 96, 8),
                                     np.arange(n // 3 - m - 3, n // 3 + 5),
                                     np.arange(2 * n // 3 - 5, 2 * n // 3 + 5)]))
    rows = rows[(rows >= 0) & (rows < N)]
    Td = torch.as_tensor(T, device="cuda")
    _note(f"anytime long windows {kind} n={n} m={m} groups A={A} B={B}")
    P, I = mp.anytime(Td, m, A, kind=kind, excl=excl)
    _check(T, m, kind, 2.0, excl, P, I, A, f"any-long-A-{kind}", rows=rows)
    mp.anytime(Td, m, B, kind=kind, excl=excl, P=P, I=I)
    _check(T, m, kind, 2.0, excl, P, I, sorted(set(A) | set(B)), f"any-long-AB-{kind}",
           rows=rows)


def test_all_groups_give_the_full_profile(mp):
    import torch
    n, m = 7000, 50
    excl = W.excl_default(m)
    T = _series(21, n, "acamp")
    Td = torch.as_tensor(T, device="cuda")
    order, cum = mp.anytime_order(n, m, excl, seed=3)
    assert cum[-1] == mp.pair_count(n, m, excl)
    _note("anytime all groups in random order, three calls")
    P, I = mp.anytime(Td, m, order[:2], kind="acamp", excl=excl)
    mp.anytime(Td, m, order[2:5], kind="acamp", excl=excl, P=P, I=I)
    mp.anytime(Td, m, order[5:], kind="acamp", excl=excl, P=P, I=I)
    Pr, Ir, Qr = oracle.profile(T, m, "acamp", excl=excl)
    check_profile(T, m, "acamp", 2.0, excl, P.cpu().numpy(), I.cpu().numpy(), Pr, Ir, Qr, 1e-9,
                  atol_for("acamp", m), label="any-all")
    # resuming from a full profile changes nothing but near ties
    Pf, If = mp.acamp(Td, m, excl=excl)
    P2, I2 = Pf.clone(), If.clone()
    mp.anytime(Td, m, order[:4], kind="acamp", excl=excl, P=P2, I=I2)
    fin = torch.isfinite(Pf)
    assert torch.all(P2[fin] <= Pf[fin]).item()
    assert torch.all(P2[fin] >= Pf[fin] * (1 - 1e-9) - atol_for("acamp", m)).item()


def test_empty_and_degenerate(mp):
    import torch
    T = _series(2, 3000, "aamp")
    Td = torch.as_tensor(T, device="cuda")
    m = 20
    _note("anytime empty group list")
    P, I = mp.anytime(Td, m, [], kind="aamp")
    assert torch.all(torch.isinf(P)).item() and torch.all(I == -1).item()
    # no admissible diagonal at all: no groups exist
    short = Td[:40]
    assert mp.anytime_groups(40, 32, 20) == 0
    P, I = mp.anytime(short, 32, [], kind="acamp", excl=20)
    assert P.numel() == 9 and torch.all(torch.isinf(P)).item() and torch.all(I == -1).item()
    with pytest.raises(mp.MpError):
        mp.anytime(short, 32, [0], kind="acamp", excl=20)
    # a single group shorter than 512 diagonals (N - excl < 512)
    n, m = 600, 16
    T2 = _series(4, n, "aamp")
    assert mp.anytime_groups(n, m, 0) == 2
    for g in ([0], [1], [1, 0]):
        P, I = mp.anytime(torch.as_tensor(T2, device="cuda"), m, g, kind="aamp")
        _check(T2, m, "aamp", 2.0, W.excl_default(m), P, I, g, f"any-small-{g}")
    # p > 6 has no band kernel
    with pytest.raises(mp.MpError):
        mp.anytime(Td, m, [0], kind="pnorm", p=7.0)


def test_anytime_class_converges(mp):
    import torch
    n, m = 8000, 64
    excl = W.excl_default(m)
    T = _series(31, n, "acamp")
    Td = torch.as_tensor(T, device="cuda")
    a = mp.Anytime(Td, m, kind="acamp", excl=excl, seed=12)
    prev = None
    for f in (0.05, 0.3, 0.3, 1.0):
        _note(f"anytime class fraction {f}")
        P, I = a.advance(f)
        assert a.covered >= f
        cur = P.clone()
        if prev is not None:
            assert torch.all(cur <= prev).item()
        prev = cur
        done = a.order[:a.done]
        _check(T, m, "acamp", 2.0, excl, P, I, done, f"any-class-{f}")
    assert a.covered == 1.0 and a.done == a.order.size


def test_large_series_sampled_rows(mp):
    """n = 100000, m = 128, ACAMP on a random walk with constant runs: a
    quarter of the groups in random order, then another quarter resumed;
    600 sampled rows against the oracle's restricted profile."""
    import torch
    n, m = 100000, 128
    excl = W.excl_default(m)
    T = _series(41, n, "acamp")
    Td = torch.as_tensor(T, device="cuda")
    order, cum = mp.anytime_order(n, m, excl, seed=8)
    q = order.size // 4
    rows = np.random.default_rng(1).choice(n - m + 1, size=600, replace=False)
    _note(f"anytime large n={n} m={m} groups={q}")
    P, I = mp.anytime(Td, m, order[:q], kind="acamp", excl=excl)
    _check(T, m, "acamp", 2.0, excl, P, I, order[:q], "any-large-1", rows=rows)
    mp.anytime(Td, m, order[q:2 * q], kind="acamp", excl=excl, P=P, I=I)
    _check(T, m, "acamp", 2.0, excl, P, I, order[:2 * q], "any-large-2", rows=rows)
