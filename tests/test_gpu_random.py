"""GPU parity on a seeded random grid of shapes: series length, window length
(1 to 250), exclusion zone (default, 1, or anywhere up to past N), distance
(p in {1, 1.5, 2, 3, 4.2, 7}), precision, refresh interval and series type
(random walk, uniform noise, noisy sine, integer steps with exact ties,
constant runs), each against the oracle; then random small batches of such
series. Every case prints its parameters before the GPU call."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import atol_for, check_profile

pytestmark = pytest.mark.gpu

KINDS = {"aamp": 0, "pnorm": 1, "acamp": 2}


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


def _series(rng, n, shape):
    if shape == "walk":
        return np.cumsum(rng.standard_normal(n))
    if shape == "uniform":
        return rng.uniform(0.0, 1.0, n)
    if shape == "sine":
        t = np.arange(n)
        return np.sin(2 * np.pi * t / rng.uniform(20, 300)) + 0.05 * rng.standard_normal(n)
    if shape == "steps":                           # integers: exact ties and constant windows
        return np.cumsum(rng.integers(-2, 3, n)).astype(np.float64)
    T = np.cumsum(rng.standard_normal(n))          # walk with constant runs
    for _ in range(3):
        a = int(rng.integers(0, n))
        T[a:a + int(rng.integers(5, 200))] = T[a]
    return T


def _draw(seed):
    rng = np.random.default_rng(1000 + seed)
    kind = str(rng.choice(["aamp", "acamp", "pnorm"]))
    p = 2.0 if kind != "pnorm" else float(rng.choice([1.0, 1.5, 2.0, 3.0, 4.2, 7.0]))
    n = int(np.exp(rng.uniform(np.log(30), np.log(4000))))
    m = min(n, int(rng.choice([1, 2, 3, 5, 8, 17, 32, 64, 100, 250])))
    N = n - m + 1
    u = rng.uniform()
    excl = 0 if u < 0.5 else (1 if u < 0.7 else int(rng.integers(1, N + 3)))
    precision = "fp32" if rng.uniform() < 0.3 else "fp64"
    R = 0 if rng.uniform() < 0.5 else int(np.exp(rng.uniform(0, np.log(5000))))
    shape = str(rng.choice(["walk", "uniform", "sine", "steps", "runs"]))
    return rng, kind, p, n, m, excl, precision, R, shape


def _tols(kind, precision, m, R=0):
    return (1e-9 if precision == "fp64" else 1e-4), atol_for(kind, m, precision, R)


@pytest.mark.parametrize("seed", range(48))
def test_random_single_series(mp, seed):
    import torch
    rng, kind, p, n, m, excl, precision, R, shape = _draw(seed)
    T = _series(rng, n, shape)
    e = excl or W.excl_default(m)
    label = f"random{seed} {kind} p={p} n={n} m={m} excl={e} {precision} R={R} {shape}"
    _note(label)
    Td = torch.as_tensor(T, device="cuda")
    if kind == "aamp":
        P, I = mp.aamp(Td, m, excl=e, precision=precision, R=R)
    elif kind == "acamp":
        P, I = mp.acamp(Td, m, excl=e, precision=precision, R=R)
    else:
        P, I = mp.pnorm(Td, m, p=p, excl=e, precision=precision, R=R)
    torch.cuda.synchronize()
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=e)
    rtol, atol = _tols(kind, precision, m, R)
    check_profile(T, m, kind, p, e, P.cpu().numpy(), I.cpu().numpy(), Pr, Ir, Qr, rtol, atol,
                  label=label)


@pytest.mark.parametrize("seed", range(6))
def test_random_batches(mp, seed):
    import torch
    rng = np.random.default_rng(5000 + seed)
    precision = "fp32" if seed % 3 == 2 else "fp64"
    specs = []
    for b in range(int(rng.integers(2, 6))):
        _, kind, p, n, m, excl, _, R, shape = _draw(100 * seed + b)
        if p == 7.0:
            p = 3.0
        specs.append((_series(rng, n, shape), m, kind, p, excl, R))
    jobs = [mp.Job(n=len(T), m=m, kind=KINDS[kind], excl=excl, R=R, p=p)
            for T, m, kind, p, excl, R in specs]
    _note(f"random batch {seed} {precision}: " +
          ", ".join(f"{k} p={p} n={len(T)} m={m} excl={x} R={R}" for T, m, k, p, x, R in specs))
    T_cat = torch.as_tensor(np.concatenate([sp[0] for sp in specs]), device="cuda")
    P, I = mp.batch(T_cat, jobs, precision=precision)
    torch.cuda.synchronize()
    P, I = P.cpu().numpy(), I.cpu().numpy()
    off = 0
    for b, (T, m, kind, p, excl, R) in enumerate(specs):
        N = len(T) - m + 1
        e = excl or W.excl_default(m)
        Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=e)
        rtol, atol = _tols(kind, precision, m, R)
        check_profile(T, m, kind, p, e, P[off:off + N], I[off:off + N], Pr, Ir, Qr, rtol, atol,
                      label=f"random batch {seed} job {b}")
        off += N


def _mask(N, excl, groups):
    mask = np.zeros(max(N, 0), dtype=bool)
    for g in groups:
        lo = excl + 512 * int(g)
        mask[lo:min(lo + 512, N)] = True
    return mask


@pytest.mark.parametrize("seed", range(12))
def test_random_anytime(mp, seed):
    """Random series and group subsets (half of the cases resumed from a
    first subset) against the oracle's diagonal-restricted profile."""
    import torch
    rng = np.random.default_rng(7000 + seed)
    kind = str(rng.choice(["aamp", "acamp", "pnorm"]))
    p = 2.0 if kind != "pnorm" else float(rng.choice([1.0, 3.0, 2.5, 6.0]))
    n = int(rng.integers(300, 6000))
    m = int(rng.choice([1, 4, 16, 40, 128]))
    excl = 0 if rng.uniform() < 0.6 else int(rng.integers(1, 200))
    shape = str(rng.choice(["walk", "uniform", "sine", "steps", "runs"]))
    T = _series(rng, n, shape)
    e = excl or W.excl_default(m)
    G = mp.anytime_groups(n, m, e)
    A = rng.choice(G, size=int(rng.integers(0, G + 1)), replace=False) if G else np.zeros(0, int)
    B = rng.choice(G, size=int(rng.integers(0, G + 1)), replace=False) if G else np.zeros(0, int)
    resume = seed % 2 == 1
    label = (f"random anytime {seed} {kind} p={p} n={n} m={m} excl={e} {shape} G={G} "
             f"A={sorted(A.tolist())} B={sorted(B.tolist()) if resume else '-'}")
    _note(label)
    Td = torch.as_tensor(T, device="cuda")
    P, I = mp.anytime(Td, m, A, kind=kind, p=p, excl=e)
    groups = set(A.tolist())
    if resume:
        mp.anytime(Td, m, B, kind=kind, p=p, excl=e, P=P, I=I)
        groups |= set(B.tolist())
    torch.cuda.synchronize()
    N = n - m + 1
    Pr, Ir, Qr = oracle.profile(T, m, kind, p=p, excl=e, diagonals=_mask(N, e, groups))
    rtol, atol = _tols(kind, "fp64", m)
    check_profile(T, m, kind, p, e, P.cpu().numpy(), I.cpu().numpy(), Pr, Ir, Qr, rtol, atol,
                  label=label)


@pytest.mark.parametrize("seed", range(8))
def test_random_fcmp(mp, seed):
    import torch
    rng = np.random.default_rng(9000 + seed)
    n = int(np.exp(rng.uniform(np.log(40), np.log(5000))))
    m = min(n, int(rng.choice([2, 3, 8, 33, 100, 256])))
    e = W.excl_default(m) if rng.uniform() < 0.7 else int(rng.integers(1, n))
    R = 0 if rng.uniform() < 0.5 else int(rng.integers(1, 3000))
    shape = str(rng.choice(["walk", "uniform", "sine", "steps", "runs"]))
    T = _series(rng, n, shape)
    label = f"random fcmp {seed} n={n} m={m} excl={e} R={R} {shape}"
    _note(label)
    P, I = mp.acamp_fcmp(torch.as_tensor(T, device="cuda"), m, excl=e, R=R)
    torch.cuda.synchronize()
    Pr, Ir, Qr = oracle.profile(T, m, "acamp", excl=e)
    check_profile(T, m, "acamp", 2.0, e, P.cpu().numpy(), I.cpu().numpy(), Pr, Ir, Qr, 1e-9,
                  atol_for("acamp", m, "fp64", R), label=label)
