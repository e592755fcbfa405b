"""Seeded synthetic time series for the matrix-profile workloads.

This module only draws numbers. It holds none of the distance or profile
arithmetic, so both the CPU oracle tests and the GPU path may use it.

The paper's own evaluation (Sec. 5.1) used uniformly random series with
n = 2^18 and m = 2^8; it names no public dataset. The configurations below
are synthetic stand-ins with the shapes, sizes and structure of the
workloads this project measures:

* ``rw8k``   random walk, n = 8192, m = 64 (pure Euclidean)
* ``rw128k`` random walk, n = 131072, with 20 constant runs and 10 planted
  motif pairs, m = 256 (z-normalized)
* ``sines``  sum of three sinusoids plus noise, n = 262144, m = 128 (p-norm)
* ``batch``  512 series of uneven length and mixed m / kind
* ``ecg``    ECG-like pulse train, n = 2^21, m = 512
* ``uniform`` the paper's own default shape: uniform(0, 1), n = 2^18

Noise written N(0, s) means a normal draw with standard deviation s.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def excl_default(m: int) -> int:
    """Exclusion half-width used by every workload: pairs with |i-j| < m/4
    are skipped, i.e. excl = ceil(m/4)."""
    return (m + 3) // 4


def random_walk(n: int, rng: np.random.Generator) -> np.ndarray:
    return np.cumsum(rng.standard_normal(n)).astype(np.float64)


def rw8k(seed: int = 0):
    """Random walk n=8192 (cumsum of N(0,1), seed 0), m=64."""
    rng = np.random.default_rng(seed)
    return random_walk(8192, rng), 64


@dataclass
class Planted:
    runs: list = field(default_factory=list)     # (start, length)
    motifs: list = field(default_factory=list)   # (a, b): T[b:b+m] ~ T[a:a+m]


def rw128k(seed: int = 2, n: int = 131072, m: int = 256, nruns: int = 20,
           nmotifs: int = 10, run_len=(300, 2000), motif_noise: float = 0.01):
    """Random walk with constant runs and planted motif pairs.

    Runs: ``nruns`` non-overlapping stretches of length U{run_len}, each set
    to the value at its first sample (so every window fully inside a run has
    zero standard deviation). Motifs: ``nmotifs`` pairs (a, b) with
    |a - b| >= m, disjoint from the runs and from each other, where
    T[b:b+m] = T[a:a+m] + N(0, motif_noise).
    Returns (T, m, Planted).
    """
    rng = np.random.default_rng(seed)
    T = random_walk(n, rng)
    taken = np.zeros(n, dtype=bool)
    planted = Planted()
    tries = 0
    while len(planted.runs) < nruns:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place constant runs")
        L = int(rng.integers(run_len[0], run_len[1] + 1))
        s = int(rng.integers(0, n - L))
        if taken[max(0, s - m):s + L + m].any():
            continue
        T[s:s + L] = T[s]
        taken[s:s + L] = True
        planted.runs.append((s, L))
    tries = 0
    while len(planted.motifs) < nmotifs:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place motifs")
        a = int(rng.integers(1, n - m - 1))
        b = int(rng.integers(1, n - m - 1))
        if abs(a - b) < m:
            continue
        if taken[max(0, a - m):a + 2 * m].any() or taken[max(0, b - m):b + 2 * m].any():
            continue
        T[b:b + m] = T[a:a + m] + rng.normal(0.0, motif_noise, m)
        taken[a:a + m] = True
        taken[b:b + m] = True
        planted.motifs.append((a, b))
    planted.runs.sort()
    return T, m, planted


def sines(seed: int = 3, n: int = 262144, m: int = 128, noise: float = 0.1):
    """Sum of 3 unit-amplitude sinusoids, periods U[50, 2000] samples,
    phases U[0, 2pi), plus N(0, noise). Returns (T, m)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n, dtype=np.float64)
    T = np.zeros(n)
    for _ in range(3):
        period = rng.uniform(50.0, 2000.0)
        phase = rng.uniform(0.0, 2.0 * math.pi)
        T += np.sin(2.0 * math.pi * x / period + phase)
    T += rng.normal(0.0, noise, n)
    return T, m


def noisy_sine(n: int, rng: np.random.Generator) -> np.ndarray:
    x = np.arange(n, dtype=np.float64)
    period = rng.uniform(50.0, 2000.0)
    phase = rng.uniform(0.0, 2.0 * math.pi)
    return np.sin(2.0 * math.pi * x / period + phase) + rng.normal(0.0, 0.1, n)


@dataclass
class BatchJob:
    T: np.ndarray
    m: int
    kind: str      # "aamp" or "acamp"


def batch(seed: int = 4, count: int = 512, nrange=(2048, 65536), ms=(32, 64, 128, 256)):
    """``count`` series, n ~ U{nrange}, m uniform over ``ms``, kind AAMP/ACAMP
    50/50, generator random walk / noisy sine 50/50."""
    rng = np.random.default_rng(seed)
    jobs = []
    for _ in range(count):
        n = int(rng.integers(nrange[0], nrange[1] + 1))
        m = int(ms[int(rng.integers(0, len(ms)))])
        kind = "aamp" if rng.random() < 0.5 else "acamp"
        T = random_walk(n, rng) if rng.random() < 0.5 else noisy_sine(n, rng)
        jobs.append(BatchJob(T=T, m=m, kind=kind))
    return jobs


def ecg(seed: int = 5, n: int = 2097152, m: int = 512, nanom: int = 5):
    """ECG-like pulse train: Gaussian beats (width 6 samples, amplitude
    U[0.8, 1.2]) every U{200..300} samples, baseline wander
    0.3 sin(2 pi x / 2000 + phi), N(0, 0.05) noise, and ``nanom`` anomalous
    beats (amplitude 2.0, width 18). Returns (T, m, anomaly_centres)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n, dtype=np.float64)
    T = 0.3 * np.sin(2.0 * math.pi * x / 2000.0 + rng.uniform(0.0, 2.0 * math.pi))
    centres = []
    c = int(rng.integers(0, 200))
    while c < n:
        centres.append(c)
        c += int(rng.integers(200, 301))
    centres = np.array(centres)
    anom = set(int(v) for v in rng.choice(np.arange(5, len(centres) - 5), size=nanom, replace=False))
    amps = rng.uniform(0.8, 1.2, len(centres))
    for idx, c in enumerate(centres):
        width, amp = (18.0, 2.0) if idx in anom else (6.0, amps[idx])
        lo, hi = max(0, c - int(5 * width)), min(n, c + int(5 * width) + 1)
        xx = np.arange(lo, hi, dtype=np.float64)
        T[lo:hi] += amp * np.exp(-0.5 * ((xx - c) / width) ** 2)
    T += rng.normal(0.0, 0.05, n)
    return T, m, sorted(int(centres[i]) for i in anom)


def uniform(seed: int = 6, n: int = 262144, m: int = 256):
    """The paper's default evaluation shape (Sec. 5.1): uniform values."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, n), m


def sample_rows(N: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct row indices in [0, N) for sampled checks."""
    rng = np.random.default_rng(seed)
    count = min(count, N)
    return np.sort(rng.choice(N, size=count, replace=False)).astype(np.int64)
