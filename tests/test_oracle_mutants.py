"""The pins must be strong enough to catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of oracle.c (a flipped sign, a dropped
term, an off-by-one bound, a transposed operand, a wrong normalisation, a
broken tie rule), builds it on the CPU, swaps it in for the real oracle and
checks that at least one pin test fails.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "euclid_sign": ("double d = T[i + l] - T[j + l];", "double d = T[i + l] + T[j + l];"),
    "excl_off_by_one": ("if (gap < excl) continue;", "if (gap <= excl) continue;"),
    "tie_rule": ("if (s < best) {", "if (s <= best) {"),
    "dropped_term": ("        for (int32_t l = 0; l < m; ++l) {\n            double d = T[i + l] - T[j + l];",
                     "        for (int32_t l = 0; l < m - 1; ++l) {\n            double d = T[i + l] - T[j + l];"),
    "transposed_sigma": ("(T[j + l] - mu[j]) / sigma[j];", "(T[j + l] - mu[j]) / sigma[i];"),
    "sample_std": ("sigma[i] = sqrt(v / (double)m);", "sigma[i] = sqrt(v / (double)(m - 1));"),
    "runner_up_lost": ("            second = best;\n", ""),
    "pnorm_no_abs": ("double a = fabs(x);", "double a = x;"),
    "wrong_mean": ("double mean = T[i] + s / (double)m;", "double mean = T[i] + s / (double)(m + 1);"),
    "root_dropped": ("        if (p == 2.0) return sqrt(s);\n", "        if (p == 2.0) return s;\n"),
    "mask_ignored": ("            if (diag_ok && !diag_ok[gap]) continue;\n", ""),
    "mask_off_by_one": ("!diag_ok[gap]", "!diag_ok[gap - 1]"),
}

PIN_TESTS = [
    lambda o: pins.test_golden_fig2_euclid_pnorm(o),
    lambda o: pins.test_golden_znorm_patterns(o),
    lambda o: pins.test_scipy_cdist_euclid_and_pnorm(o, 0),
    lambda o: pins.test_numpy_corrcoef_znorm(o),
    lambda o: pins.test_numpy_window_stats(o),
    lambda o: pins.test_exact_integer_euclid_pnorm(o, 2),
    lambda o: pins.test_exact_rational_znorm(o),
    lambda o: pins.test_constant_series(o),
    lambda o: pins.test_diagonal_mask_matches_library(o),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, monkeypatch, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    cpath = tmp_path / "oracle_mut.c"
    cpath.write_text(mutated)
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", str(so),
                    str(cpath), "-lm"], check=True, capture_output=True)
    monkeypatch.setattr(oracle, "_lib", oracle._bind(ctypes.CDLL(str(so))))
    failures = 0
    for t in PIN_TESTS:
        try:
            t(oracle)
        except (AssertionError, ValueError):
            failures += 1
    assert failures >= 1, f"no pin caught mutant {name}"
