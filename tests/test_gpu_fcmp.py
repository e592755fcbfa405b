"""GPU parity of mp_acamp_fcmp: the z-normalized profile with the band sweep
comparing pairs on the F of Sec. 4.4 (Eq. 9). F orders pairs as the distance
does, so the profile equals the oracle's (1e-9 relative, the absolute floor
of tests/parity.py; ties allowed) and agrees with mp_acamp wherever both pick
the same index."""
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


def _walk(seed, n, runs=True, motifs=True):
    rng = np.random.default_rng(seed)
    T = np.cumsum(rng.standard_normal(n))
    if runs:
        for a in (n // 5, n // 2, 4 * n // 5):
            T[a:a + 70] = T[a]
    if motifs:
        src = T[n // 10:n // 10 + 60].copy()
        T[3 * n // 5:3 * n // 5 + 60] = 2.0 * src + 5.0 + 1e-3 * rng.standard_normal(60)
    return T


CASES = [(3001, 37, None, 0), (20000, 100, None, 0), (9000, 64, 1, 0), (12000, 256, None, 1000),
         (700, 32, None, 0), (250, 32, None, 0)]


@pytest.mark.parametrize("n,m,excl,R", CASES)
def test_fcmp_matches_oracle(mp, n, m, excl, R):
    import torch
    T = _walk(n + m, n)
    e = excl or W.excl_default(m)
    _note(f"acamp_fcmp n={n} m={m} excl={e} R={R}")
    Td = torch.as_tensor(T, device="cuda")
    P, I = mp.acamp_fcmp(Td, m, excl=e, R=R)
    Pr, Ir, Qr = oracle.profile(T, m, "acamp", excl=e)
    check_profile(T, m, "acamp", 2.0, e, P.cpu().numpy(), I.cpu().numpy(), Pr, Ir, Qr, 1e-9,
                  atol_for("acamp", m, "fp64", R), label=f"fcmp-{n}-{m}")
    # same exact rescoring as mp_acamp: equal indices give equal values
    P2, I2 = mp.acamp(Td, m, excl=e, R=R)
    same = I == I2
    assert torch.equal(P[same], P2[same])
    assert same.float().mean().item() > 0.99


def test_fcmp_affine_offset(mp):
    """Offset 1e4, scale 1e-2: the key 1 - rho|rho| is formed next to 1 like
    1 - rho, so near-constant windows stay within the bound."""
    import torch
    n, m = 15000, 128
    T = 1e4 + 1e-2 * _walk(77, n)
    e = W.excl_default(m)
    _note("acamp_fcmp offset series")
    P, I = mp.acamp_fcmp(torch.as_tensor(T, device="cuda"), m, excl=e)
    Pr, Ir, Qr = oracle.profile(T, m, "acamp", excl=e)
    check_profile(T, m, "acamp", 2.0, e, P.cpu().numpy(), I.cpu().numpy(), Pr, Ir, Qr, 1e-9,
                  atol_for("acamp", m), label="fcmp-offset")


def test_fcmp_full_size_sampled(mp):
    """The headline shape (n = 131072, m = 256): sampled rows against the oracle."""
    import torch
    n, m = 131072, 256
    T = _walk(5, n)
    e = W.excl_default(m)
    rows = np.random.default_rng(3).choice(n - m + 1, size=400, replace=False)
    _note("acamp_fcmp full size")
    P, I = mp.acamp_fcmp(torch.as_tensor(T, device="cuda"), m, excl=e)
    Pr, Ir, Qr = oracle.profile(T, m, "acamp", excl=e, rows=rows)
    check_profile(T, m, "acamp", 2.0, e, P.cpu().numpy()[rows], I.cpu().numpy()[rows], Pr, Ir, Qr,
                  1e-9, atol_for("acamp", m), rows=rows, label="fcmp-full")
