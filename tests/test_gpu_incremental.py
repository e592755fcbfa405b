"""GPU parity of incremental profiles (mp_inc_*): after any sequence of
appends the profile equals the oracle's profile of everything appended so
far (1e-9 relative; for ACAMP the absolute floor of tests/parity.py; ties
allowed)."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import atol_for, check_profile

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


def _verify(inc, T, m, kind, p, excl, label):
    n, N = inc.size()
    assert n == len(T) and N == max(0, len(T) - m + 1)
    P, I = inc.profile()
    if N == 0:
        return
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=excl)
    check_profile(T, m, kind, p, excl, P.cpu().numpy(), I.cpu().numpy(), Pr, Ir, Qr, 1e-9,
                  atol_for(kind, m), label=label)


CASES = [("aamp", 2.0), ("acamp", 2.0), ("pnorm", 1.0), ("pnorm", 3.0), ("pnorm", 2.5)]


@pytest.mark.parametrize("kind,p", CASES)
def test_grow_from_empty_in_random_chunks(mp, kind, p):
    import torch
    rng = np.random.default_rng(31)
    full = np.cumsum(rng.standard_normal(4000))
    if kind == "acamp":
        full[1500:1650] = full[1500]            # a constant run, crossed by chunk boundaries
    m, excl = 40, W.excl_default(40)
    inc = mp.Incremental(m, kind=kind, p=p, capacity=len(full))
    pos, step = 0, 0
    while pos < len(full):
        c = int(rng.choice([1, 1, 3, 17, 64, 250, 700]))
        c = min(c, len(full) - pos)
        inc.append(torch.as_tensor(full[pos:pos + c], device="cuda"))
        pos += c
        step += 1
        if step % 9 == 0 or pos == len(full):
            _note(f"incremental {kind} p={p} n={pos}")
            _verify(inc, full[:pos], m, kind, p, excl, f"inc-{kind}{p}-n{pos}")
    inc.close()


@pytest.mark.parametrize("kind", ["aamp", "acamp"])
def test_single_sample_appends_cross_refreshes(mp, kind):
    """300 one-sample appends with an exact restart every 64 windows."""
    import torch
    rng = np.random.default_rng(5)
    full = np.cumsum(rng.standard_normal(3300))
    m, excl = 64, W.excl_default(64)
    inc = mp.Incremental(m, kind=kind, capacity=len(full), refresh=64)
    inc.append(torch.as_tensor(full[:3000], device="cuda"))      # one-shot path
    _verify(inc, full[:3000], m, kind, 2.0, excl, f"inc1-{kind}-start")
    for t in range(3000, 3300):
        inc.append(torch.as_tensor(full[t:t + 1], device="cuda"))
        if t in (3000, 3063, 3064, 3150, 3299):
            _note(f"single appends {kind} n={t + 1}")
            _verify(inc, full[:t + 1], m, kind, 2.0, excl, f"inc1-{kind}-n{t + 1}")
    inc.close()


def test_large_append_rebuilds(mp):
    import torch
    rng = np.random.default_rng(8)
    full = np.cumsum(rng.standard_normal(9000))
    m = 32
    inc = mp.Incremental(m, kind="acamp", capacity=len(full))
    inc.append(torch.as_tensor(full[:3000], device="cuda"))
    inc.append(torch.as_tensor(full[3000:3100], device="cuda"))   # incremental
    inc.append(torch.as_tensor(full[3100:9000], device="cuda"))   # one-shot rebuild
    _verify(inc, full, m, "acamp", 2.0, W.excl_default(m), "inc-rebuild")
    inc.append(torch.as_tensor(np.zeros(0), device="cuda"))        # empty append
    assert inc.size() == (9000, 9000 - m + 1)
    inc.close()


def test_short_series_and_capacity(mp):
    import torch
    m = 50
    inc = mp.Incremental(m, kind="aamp", capacity=200)
    inc.append(torch.as_tensor(np.arange(30, dtype=np.float64), device="cuda"))
    assert inc.size() == (30, 0)                 # no window yet
    P, I = inc.profile()
    assert P.numel() == 0
    rng = np.random.default_rng(2)
    rest = np.cumsum(rng.standard_normal(170))
    inc.append(torch.as_tensor(rest, device="cuda"))
    full = np.concatenate([np.arange(30, dtype=np.float64), rest])
    _verify(inc, full, m, "aamp", 2.0, W.excl_default(m), "inc-short")
    with pytest.raises(mp.MpError):
        inc.append(torch.as_tensor(np.ones(1), device="cuda"))     # capacity reached
    inc.close()


def test_pnorm_two_equals_aamp(mp):
    import torch
    rng = np.random.default_rng(4)
    full = np.cumsum(rng.standard_normal(2600))
    a = mp.Incremental(24, kind="aamp", capacity=2600)
    b = mp.Incremental(24, kind="pnorm", p=2.0, capacity=2600)
    for lo, hi in ((0, 2000), (2000, 2001), (2001, 2400), (2400, 2600)):
        chunk = torch.as_tensor(full[lo:hi], device="cuda")
        a.append(chunk)
        b.append(chunk)
    Pa, Ia = a.profile()
    Pb, Ib = b.profile()
    assert np.array_equal(Pa.cpu().numpy(), Pb.cpu().numpy())
    assert np.array_equal(Ia.cpu().numpy(), Ib.cpu().numpy())


@pytest.mark.parametrize("kind", ["aamp", "acamp"])
def test_widest_column_launches(mp, kind):
    """Appends of 2048 and 2049 windows to 20000: the first fills one column
    launch (2048 new columns, the most one launch takes), the second runs
    2048 more up to the restart and one after it. All new windows and a
    sample of old rows are checked against the oracle."""
    import torch
    rng = np.random.default_rng(17)
    m = 16
    n0 = 20000 + m - 1
    full = np.cumsum(rng.standard_normal(n0 + 2048 + 2049))
    if kind == "acamp":
        full[n0 + 700:n0 + 760] = full[n0 + 700]     # a constant run inside the launch
    excl = W.excl_default(m)
    inc = mp.Incremental(m, kind=kind, capacity=len(full), refresh=4096)
    inc.append(torch.as_tensor(full[:n0], device="cuda"))          # one-shot path
    for lo, hi in ((n0, n0 + 2048), (n0 + 2048, len(full))):
        inc.append(torch.as_tensor(full[lo:hi], device="cuda"))
        _note(f"widest column launch {kind} n={hi}")
        T = full[:hi]
        N = hi - m + 1
        rows = np.unique(np.concatenate([rng.choice(20000, size=600, replace=False),
                                         np.arange(20000, N)]))
        P, I = inc.profile()
        P = P.cpu().numpy()[rows]
        I = I.cpu().numpy()[rows]
        Pr, Ir, Qr = oracle.profile(T, m, kind, excl=excl, rows=rows)
        check_profile(T, m, kind, 2.0, excl, P, I, Pr, Ir, Qr, 1e-9,
                      atol_for(kind, m), rows=rows, label=f"inc-wide-{kind}-n{hi}")
    inc.close()
