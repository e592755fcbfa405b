"""Why the Euclidean FP32 sweep is not offered: single-precision drift of the
running sum, replayed on the host (CPU only).

Row 113495 of the 131072-sample walk (m = 256) is the row an FP32 + refresh
AAMP sweep left 2.79e-4 above its minimum. Its true best pair (from the
stored oracle rows) is replayed along its diagonal from an exact FP64 start
at many possible item starts, with the sweep's update
S <- S + (u_i - u_j)(v_i - v_j) in two single-precision models:
  * operands rounded to float, the sum kept exact: the drift stays far inside
    the 2e-4 the 1e-4 profile contract allows on S;
  * operands exact, the sum rounded to float after every step (a fused
    multiply-add): the drift exceeds it.
So the running sum's rounding (u |S| per step while the diagonal passes
through large sums), not the operands, breaks the contract, which is why
per-item recentring of the operands cannot fix it."""
import numpy as np

import workloads as W
from tests import fullsize_refs as R


def _replay(T, m, i, j, s0, round_ops, round_sum):
    N = len(T) - m + 1
    a0, b0 = i - s0, j - s0
    c = T[a0]

    def exact(a, b):
        d = T[a:a + m] - T[b:b + m]
        return float(np.dot(d, d))

    def f32(x):
        return float(np.float32(x))

    S = exact(a0, b0)
    if round_sum:
        S = f32(S)
    for t in range(1, s0 + 1):
        a, b = a0 + t, b0 + t
        ua, ub = T[a + m - 1] - T[a - 1], T[b + m - 1] - T[b - 1]
        va, vb = T[a + m - 1] + T[a - 1] - 2 * c, T[b + m - 1] + T[b - 1] - 2 * c
        if round_ops:
            x = f32(f32(ua) - f32(ub))
            y = f32(f32(va) - f32(vb))
        else:
            x, y = ua - ub, va - vb
        S = S + x * y          # the float64 product of two floats is exact
        if round_sum:
            S = f32(S)
    assert b0 + s0 < N
    return S


def test_running_sum_rounding_not_operands_breaks_fp32_aamp():
    T, m, _ = W.rw128k()
    ref = R.load("rw128k_aamp", T=T)
    k = int(np.nonzero(ref["rows"] == 113495)[0][0])
    i, j = 113495, int(ref["I"][k])
    S_true = float(ref["P"][k]) ** 2
    starts = range(16, 2048, 61)
    ops = np.array([_replay(T, m, i, j, s0, True, False) for s0 in starts])
    acc = np.array([_replay(T, m, i, j, s0, False, True) for s0 in starts])
    rms_ops = np.sqrt(np.mean(((ops - S_true) / S_true) ** 2))
    rms_acc = np.sqrt(np.mean(((acc - S_true) / S_true) ** 2))
    assert rms_ops < 5e-5          # rounded operands alone: well inside 2e-4
    assert rms_acc > 1e-3          # the single-precision running sum: far beyond
