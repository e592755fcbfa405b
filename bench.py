#!/usr/bin/env python3
"""Benchmark of the matrix-profile hot path on one MI355X.

Headline workload (one step = one full call of the hot path: window
statistics and difference streams, the diagonal sweep, FP64 rescoring,
certification and exact search): z-normalized profile (ACAMP) of a random
walk of n = 131072 samples with 20 constant runs and 10 planted motif pairs,
m = 256, exclusion |i - j| < m/4. Timed in FP64 (``value``), in
FP32 + FP64 refresh (``fp32_refresh``) and in MP_FP32_AUTO (``fp32_auto``: the
same tolerance, the faster sweep), with the gains over FP64.

Batch workload (``batch``): 512 random-walk / noisy-sine series of length
U{2048..65536}, m in {32, 64, 128, 256}, AAMP / ACAMP mixed, one mp_batch call
per step (autotuned, captured once, then replayed as a HIP graph), in the
same three precision modes.

The other workloads (``configs``): the 8192-sample random walk (AAMP), the
262144-sample sines (p = 1 and p = 3) and the 2,097,152-sample ECG-like series
(ACAMP and AAMP), each in FP64 and FP32 + refresh. Long windows
(``long_windows``, the paper's Fig. 4 shape): n = 2^18 uniform values,
m = 256 .. 65536, AAMP and ACAMP, both precisions.

Every sweep figure carries its VALU roofline fraction: algorithmic lane
operations (the O(1) update plus one row and one column minimum per pair)
over the sweep phase's time, measured with the library's HIP events on the
calling stream, against 256 CUs x 64 lanes x 2.4 GHz.

Inputs are resident in HBM before timing starts. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only LIST] [--no-batch]
                    [--no-configs] [--no-long] [--no-cpu] [--no-fp32] [--no-auto]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "subsequence-pair distances/s (G pairs/s) FP32+refresh vs FP64, at stated error"

# VALU issue rate of one MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# lane-operations per second (FP64 FMA, add, mul and min are all full rate).
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# algorithmic lane-operations per pair (O(1) update + row min + column min):
# AAMP 2 sub + 2 FMA + 2 min (the update is (u_i - u_j)(v_i - v_j) + S, one
# FMA, but the count follows the update's two-product form), ACAMP 2 FMA +
# 2 mul + 2 min, p = 1 2 sub + 2 add + 2 min, p = 3 2 sub + 2 mul + 2 FMA +
# 2 min. The FP32 sweep is counted the same way: packed FP32 is not used, so
# single precision issues at the FP64 lane rate.
OPS_PER_PAIR = {"aamp": 6, "acamp": 6, "pnorm1": 6, "pnorm3": 8}
WORKLOADS = ("headline", "extras", "batch", "configs", "long")


def ops_per_pair(kind, p=2.0):
    if kind == "pnorm":
        return OPS_PER_PAIR["pnorm1"] if p == 1.0 else OPS_PER_PAIR["pnorm3"]
    return OPS_PER_PAIR[kind]


def roofline_frac(ops, sweep_ms):
    """Fraction of the VALU peak reached by `ops` lane-operations in sweep_ms."""
    return round(ops / (sweep_ms * 1e-3) / PEAK_LANE_OPS, 4) if sweep_ms > 0 else None
# HBM traffic of the sweep kernel, from rocprofv3 counters (see that file)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_band_acamp_rw128k_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1901_05708_amd", "csrc", "k_sweep_band.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--only", default="",
                    help="comma-separated subset of " + ",".join(WORKLOADS) +
                         " (headline runs whenever extras does); default: all")
    ap.add_argument("--names", default="",
                    help="comma-separated subset of the configs / long-window workload names "
                         "(e.g. ecg_acamp,uniform_m65536_aamp); default: all")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch workload")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other single-series workloads (rw8k, sines p = 1 and 3, "
                         "ecg ACAMP and AAMP)")
    ap.add_argument("--configs", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-long", action="store_true",
                    help="skip the long-window (Fig. 4) workloads")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32 + refresh and MP_FP32_AUTO runs")
    ap.add_argument("--no-auto", action="store_true", help="skip the MP_FP32_AUTO runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle sample rows (0: auto)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(T, m, excl, kind, P_gpu, I_gpu, rows_hint=0):
    """The oracle (FP64 brute force), timed on this host on a bounded sample of
    rows of the same workload; scaled to whole-workload pairs/s."""
    import numpy as np
    import oracle
    import workloads as W
    oracle.build(force=False)
    n = len(T)
    N = n - m + 1
    threads = oracle.num_threads()
    # one row costs about N*m*4 operations; ~300 rows per thread is 10-30 s
    rows = rows_hint or max(threads, min(N, int(threads * 300)))
    sample = W.sample_rows(N, rows, seed=123)
    t0 = time.perf_counter()
    Pr, Ir, Qr = oracle.profile(T, m, kind, excl=excl, rows=sample, nthreads=threads)
    dt = time.perf_counter() - t0
    # single-thread figure on a small slice of the same sample
    one = sample[:max(4, len(sample) // (threads * 25))]
    t1 = time.perf_counter()
    oracle.profile(T, m, kind, excl=excl, rows=one, nthreads=1)
    dt1 = time.perf_counter() - t1
    total_pairs = (N - excl) * (N - excl + 1) // 2
    extrapolated = dt * N / len(sample)
    # rows whose GPU result agrees with the oracle (same index, or a tie
    # within 1e-9 / 1e-6 absolute for the z-normalized distance)
    Pg, Ig = P_gpu[sample], I_gpu[sample]
    fin = np.isfinite(Pr)
    with np.errstate(invalid="ignore"):
        okv = np.where(fin, np.abs(Pg - Pr) <= 1e-9 * Pr + 1e-6, np.isinf(Pg))
        oki = (Ig == Ir) | ((Qr - Pr) <= 1e-9 * Pr + 1e-6)
    return {
        "value": total_pairs / extrapolated / 1e9,
        "unit": "Gpairs/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{len(sample)} random rows of the same workload (seed 123), brute force "
                   f"FP64 over every admissible column; {dt:.2f} s measured, whole-workload "
                   f"time extrapolated as N/rows x measured = {extrapolated:.1f} s"),
        "rows_checked": int(len(sample)),
        "rows_matching_gpu": int(np.sum(okv & oki)),
        "single_thread_value": total_pairs / (dt1 * N / len(one)) / 1e9,
        "single_thread_sample": f"{len(one)} rows, {dt1:.2f} s",
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
    }


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def sweep_traffic(refresh_rows):
    """HBM bytes per launch of the FP64 ACAMP sweep at this refresh interval,
    from the committed rocprofv3 counter summary; None when the summary has
    no entry for it or the kernel source changed since the counters were
    taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    want = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    got = re.search(r"traffic_bytes_per_launch\[R=%d\]:\s*([0-9]+)" % int(refresh_rows), text)
    if not want or not got:
        return None
    have = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    return int(got.group(1)) if have == want.group(1) else None


def timed(fn, steps, warmup, stream):
    """(mean, median) ms per call of fn over `steps` calls after `warmup`
    untimed ones. Every call is bracketed by events on the stream; the whole
    run by device synchronisation."""
    import statistics
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return ev[0].elapsed_time(ev[steps]) / steps, statistics.median(per)


def _lower_precisions(args):
    if args.no_fp32:
        return ()
    return ("fp32",) if args.no_auto else ("fp32", "fp32_auto")


def headline(args, mp, W, torch):
    T, m, planted = W.rw128k()
    n = len(T)
    excl = W.excl_default(m)
    pairs = mp.pair_count(n, m, excl)
    Td = torch.as_tensor(T, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    res = {"T": T, "m": m, "excl": excl, "pairs": pairs, "n": n}
    for prec in ("fp64",) + _lower_precisions(args):
        out = {}

        def step():
            out["PI"] = mp.acamp(Td, m, excl=excl, precision=prec, stream=stream, validate=False)

        # first call: input check and the refresh-interval autotuner (timed apart)
        mp.set_profiling(False)
        mp.acamp(Td, m, excl=excl, precision=prec, stream=stream)
        torch.cuda.synchronize()
        tune_ms = mp.profile_read()["ms_autotune"]
        # timed region with the library's phase events on (no host syncs)
        mp.set_profiling(True)
        t0 = time.perf_counter()
        ms, med = timed(step, args.steps, args.warmup, stream)
        wall = time.perf_counter() - t0
        prof = mp.profile_read()
        mp.set_profiling(False)
        calls = max(1, prof["calls"])
        res[prec] = {
            "ms_per_step": ms,
            "ms_median": med,
            "autotune_ms": tune_ms,
            "value": pairs / (ms * 1e-3) / 1e9,
            "sweep_ms": prof["ms_sweep"] / calls,
            "prep_ms": prof["ms_prep"] / calls,
            "finalize_ms": prof["ms_finalize"] / calls,
            "fallback_rows": prof["fallback_rows"] / calls,
            "refresh_rows": prof["refresh_rows"],
            "diags_per_lane": prof["diags_per_lane"],
            "items": prof["items"],
            "fp32_jobs": prof["fp32_jobs"],
            "wall_s": wall,
            "P": out["PI"][0].cpu().numpy(),
            "I": out["PI"][1].cpu().numpy(),
        }
    return res


def _time_single(mp, torch, Td, m, kind, p, excl, prec, steps, stream, label):
    """Autotune (first call), then `steps` timed calls with the library's
    phase events on: ms per call end to end, the sweep phase's ms, and the
    shape the autotuner chose."""
    def step():
        if kind == "aamp":
            mp.aamp(Td, m, excl=excl, precision=prec, stream=stream, validate=False)
        elif kind == "acamp":
            mp.acamp(Td, m, excl=excl, precision=prec, stream=stream, validate=False)
        else:
            mp.pnorm(Td, m, p=p, excl=excl, precision=prec, stream=stream, validate=False)
    print(f"[bench] {label} {prec}: autotune and timing", file=sys.stderr, flush=True)
    mp.set_profiling(False)
    step()                          # autotuner
    torch.cuda.synchronize()
    tune = mp.profile_read()["ms_autotune"]
    mp.set_profiling(True)
    ms, med = timed(step, steps, 1, stream)
    prof = mp.profile_read()
    mp.set_profiling(False)
    calls = max(1, prof["calls"])
    return {"ms_per_step": round(ms, 4), "ms_median": round(med, 4),
            "sweep_ms": round(prof["ms_sweep"] / calls, 4),
            "finalize_ms": round(prof["ms_finalize"] / calls, 4),
            "refresh_rows": prof["refresh_rows"], "diags_per_lane": prof["diags_per_lane"],
            "fp32_jobs": prof["fp32_jobs"], "autotune_ms": round(tune, 1),
            "fallback_rows_per_step": round(prof["fallback_rows"] / calls, 1)}


def _single_row(mp, torch, T, m, kind, p, steps, stream, label, precisions=("fp64", "fp32")):
    import workloads as W
    Td = torch.as_tensor(T, dtype=torch.float64, device="cuda")
    excl = W.excl_default(m)
    pairs = mp.pair_count(len(T), m, excl)
    ops = ops_per_pair(kind, p) * pairs
    row = {"n": len(T), "m": m, "kind": kind, "p": p, "pairs": pairs,
           "ops_per_pair": ops_per_pair(kind, p)}
    for prec in precisions:
        r = _time_single(mp, torch, Td, m, kind, p, excl, prec, steps, stream, label)
        r["value"] = round(pairs / (r["ms_per_step"] * 1e-3) / 1e9, 1)
        r["sweep_frac"] = roofline_frac(ops, r["sweep_ms"])
        row[prec] = r
    if "fp32" in row:
        row["fp32_gain"] = round(row["fp32"]["value"] / row["fp64"]["value"], 3)
        row["fp32_sweep_gain"] = round(row["fp64"]["sweep_ms"] / row["fp32"]["sweep_ms"], 3)
    print(f"[bench] {label}: " + ", ".join(f"{k} {row[k]['value']} Gpairs/s (sweep frac "
                                            f"{row[k]['sweep_frac']})" for k in precisions),
          file=sys.stderr, flush=True)
    return row


def other_configs(args, mp, W, torch):
    """The other single-series workloads, each autotuned and then timed over a
    few calls in FP64 and FP32 + refresh: pairs/s end to end, the sweep's VALU
    roofline fraction, the FP32 gain and the exact-search rows. Returns a dict
    keyed by workload."""
    runs = []
    T, m = W.rw8k()
    runs.append(("rw8k_aamp", T, m, "aamp", 2.0, 20))
    T, m = W.sines()
    runs.append(("sines_p1", T, m, "pnorm", 1.0, 5))
    runs.append(("sines_p3", T, m, "pnorm", 3.0, 5))
    T, m, _ = W.ecg()
    runs.append(("ecg_acamp", T, m, "acamp", 2.0, 2))
    runs.append(("ecg_aamp", T, m, "aamp", 2.0, 2))
    stream = torch.cuda.current_stream()
    names = set(x for x in args.names.split(",") if x)
    res = {}
    for name, T, m, kind, p, steps in runs:
        if names and name not in names:
            continue
        res[name] = _single_row(mp, torch, T, m, kind, p, steps, stream, name,
                                ("fp64",) if args.no_fp32 else ("fp64", "fp32"))
    return res


def long_windows(args, mp, W, torch):
    """The paper's second experiment (Sec. 5.2, Fig. 4): n = 2^18 uniform
    values, the window length doubled from 256 to 65536 (every other power of
    two), AAMP and ACAMP, both precisions."""
    T, _ = W.uniform()
    stream = torch.cuda.current_stream()
    names = set(x for x in args.names.split(",") if x)
    res = {}
    for m in (256, 1024, 4096, 16384, 65536):
        for kind in ("aamp", "acamp"):
            name = f"uniform_m{m}_{kind}"
            if names and name not in names:
                continue
            res[name] = _single_row(mp, torch, T, m, kind, 2.0, 3, stream, name,
                                    ("fp64",) if args.no_fp32 else ("fp64", "fp32"))
    res["workload"] = ("uniform U[0,1) n=262144 (seed 6), m in {256, 1024, 4096, 16384, 65536}, "
                       "excl = ceil(m/4)")
    return res


def batch_workload(args, mp, W, torch):
    import numpy as np
    jobs_np = W.batch()
    jobs = [mp.Job(n=len(jb.T), m=jb.m, kind=mp.KIND_AAMP if jb.kind == "aamp" else mp.KIND_ACAMP)
            for jb in jobs_np]
    T_cat = torch.as_tensor(np.concatenate([jb.T for jb in jobs_np]), device="cuda")
    table, total_n, total_out = mp.batch_layout(jobs)
    pairs = sum(mp.pair_count(jb.n, jb.m, mp.default_excl(jb.m)) for jb in jobs)
    ops = sum(mp.pair_count(jb.n, jb.m, mp.default_excl(jb.m)) *
              ops_per_pair("aamp" if jb.kind == mp.KIND_AAMP else "acamp") for jb in jobs)
    stream = torch.cuda.current_stream()
    res = {"jobs": len(jobs), "pairs": pairs, "samples": int(total_n), "ops_per_pair": 6}
    for prec in ("fp64",) + _lower_precisions(args):
        P = torch.empty(total_out, dtype=torch.float64, device="cuda")
        I = torch.empty(total_out, dtype=torch.int64, device="cuda")
        mp.set_profiling(False)       # clears autotune time and replay counters
        t0 = time.perf_counter()
        mp.batch(T_cat, jobs, precision=prec, out=(P, I), table=table, stream=stream)
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        tune = mp.profile_read()["ms_autotune"]

        def step():
            mp.batch(T_cat, jobs, precision=prec, out=(P, I), table=table, stream=stream,
                     validate=False)

        ms, med = timed(step, args.batch_steps, 1, stream)
        replays = mp.profile_read()["graph_replays"]
        # one profiled call (launched directly) for the phase split
        mp.set_profiling(True)
        step()
        prof = mp.profile_read()
        mp.set_profiling(False)
        res[prec] = {
            "ms_per_step": round(ms, 3),
            "ms_median": round(med, 3),
            "value": round(pairs / (ms * 1e-3) / 1e9, 3),
            "graph_replays": replays,
            "first_call_s": round(first, 3),
            "autotune_ms": round(tune, 1),
            "refresh_rows": prof["refresh_rows"],
            "diags_per_lane": prof["diags_per_lane"],
            "fallback_rows_per_step": prof["fallback_rows"],
            "band_jobs": prof["band_jobs"],
            "fp32_jobs": prof["fp32_jobs"],
            "phases_ms": {"prep": round(prof["ms_prep"], 3), "sweep": round(prof["ms_sweep"], 3),
                          "finalize": round(prof["ms_finalize"], 3)},
            # the sweep launches of one directly launched (profiled) call
            "sweep_frac": roofline_frac(ops, prof["ms_sweep"]),
        }
    if "fp32" in res:
        res["fp32_gain"] = round(res["fp32"]["value"] / res["fp64"]["value"], 4)
    if "fp32_auto" in res:
        res["fp32_auto_gain"] = round(res["fp32_auto"]["value"] / res["fp64"]["value"], 4)
    res["workload"] = ("512 series (seed 4): random walk or noisy sine, n ~ U{2048..65536}, "
                       "m in {32,64,128,256}, AAMP/ACAMP 50/50, excl = ceil(m/4); one mp_batch "
                       "call per step, graph replay")
    return res


def incremental(mp, h, torch):
    """Appending to the headline series (ACAMP, m = 256): the first 131072
    samples load through the one-shot path, then single samples and chunks
    of 256 are appended. Each new window is one new column of N pairs."""
    import numpy as np
    T = h["T"]
    m = h["m"]
    rng = np.random.default_rng(99)
    more = T[-1] + np.cumsum(rng.standard_normal(4096 + 200))
    inc = mp.Incremental(m, kind="acamp", capacity=len(T) + len(more))
    inc.append(torch.as_tensor(T, device="cuda"))
    torch.cuda.synchronize()
    ones = [torch.as_tensor(more[k:k + 1], device="cuda") for k in range(200)]
    chunks = [torch.as_tensor(more[200 + 256 * k:200 + 256 * (k + 1)], device="cuda")
              for k in range(16)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in ones:
        inc.append(c)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for c in chunks:
        inc.append(c)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    N = inc.size()[1]
    inc.close()
    single = (t1 - t0) / len(ones)
    chunk = (t2 - t1) / len(chunks)
    return {"single_append_us": round(single * 1e6, 1),
            "chunk256_append_ms": round(chunk * 1e3, 3),
            "chunk256_pairs_per_s": round(256 * N / chunk / 1e9, 2),
            "unit_note": "host wall time per append; pairs/s in G (N pairs per new window)",
            "N": N}


def anytime_curve(mp, h, torch):
    """Anytime sweep of the headline series: the diagonal groups in a seeded
    random order, advanced to 1 %, 5 %, 25 % and 100 % of the pairs. Reports
    the host wall time of each advance, and the share of rows whose value
    already equals the full profile's (relative 1e-9) at each point."""
    import numpy as np
    T = torch.as_tensor(h["T"], device="cuda")
    m, excl = h["m"], h["excl"]
    Pf = torch.as_tensor(h["fp64"]["P"], device="cuda")
    fin = torch.isfinite(Pf)
    mp.Anytime(T, m, kind="acamp", excl=excl, seed=1).advance(0.02)     # warm
    torch.cuda.synchronize()
    a = mp.Anytime(T, m, kind="acamp", excl=excl, seed=1)
    torch.cuda.synchronize()
    points, total_ms, prev_pairs = [], 0.0, 0
    total = int(a.cum[-1])
    for f in (0.01, 0.05, 0.25, 1.0):
        t0 = time.perf_counter()
        P, _ = a.advance(f)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        total_ms += ms
        pairs = int(a.cum[a.done - 1])
        # the parity tests' tolerance: 1e-9 relative, 1e-6 absolute (ACAMP)
        exact = torch.isfinite(P) & (P <= Pf * (1 + 1e-9) + 1e-6)
        both = fin & torch.isfinite(P) & (Pf > 0)
        ratio = (P[both] / Pf[both]).cpu().numpy()
        points.append({"fraction": round(pairs / total, 4), "groups": int(a.done),
                       "step_ms": round(ms, 3), "step_gpairs_per_s":
                       round((pairs - prev_pairs) / ms / 1e6, 1),
                       "rows_exact": round(float((exact & fin).sum()) / float(fin.sum()), 4),
                       "p_ratio_median": round(float(np.median(ratio)), 4) if ratio.size else None,
                       "p_ratio_p90": round(float(np.quantile(ratio, 0.9)), 4) if ratio.size
                       else None})
        prev_pairs = pairs
    return {"groups": int(a.order.size), "seed": 1, "points": points,
            "total_ms": round(total_ms, 3),
            "note": "host wall time per advance (one mp_anytime call each, resumed); rows_exact: "
                    "share of rows whose P already equals the full profile's; p_ratio: P over "
                    "the full profile's P (median, 90th percentile)"}


def fcmp_variant(args, mp, h, torch):
    """The headline series with the sweep comparing pairs on the F of
    Sec. 4.4 (mp_acamp_fcmp), timed like the headline at the refresh interval
    the headline run chose, against the headline's own FP64 figures (pairs
    compared on rho): ms per call, sweep ms, and index agreement."""
    Td = torch.as_tensor(h["T"], device="cuda")
    m, excl, rho = h["m"], h["excl"], h["fp64"]
    R = rho["refresh_rows"]
    stream = torch.cuda.current_stream()
    out = {}

    def step():
        out["PI"] = mp.acamp_fcmp(Td, m, excl=excl, R=R, stream=stream, validate=False)

    mp.acamp_fcmp(Td, m, excl=excl, R=R, stream=stream)
    torch.cuda.synchronize()
    mp.set_profiling(True)
    ms, med = timed(step, max(3, args.steps // 3), args.warmup, stream)
    prof = mp.profile_read()
    mp.set_profiling(False)
    calls = max(1, prof["calls"])
    sweep = prof["ms_sweep"] / calls
    agree = float((out["PI"][1].cpu().numpy() == rho["I"]).mean())
    return {"value": round(h["pairs"] / (ms * 1e-3) / 1e9, 3), "ms_per_step": round(ms, 4),
            "sweep_ms": round(sweep, 4), "rho_value": round(rho["value"], 3),
            "rho_sweep_ms": round(rho["sweep_ms"], 4),
            "sweep_ratio_vs_rho": round(sweep / rho["sweep_ms"], 4), "refresh_rows": R,
            "index_agreement": round(agree, 6)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1901_05708_amd as mp
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a HIP GPU", file=sys.stderr)
        sys.exit(1)
    mp.load()
    only = set(x for x in args.only.split(",") if x)
    bad = only - set(WORKLOADS)
    if bad:
        print(f"unknown workloads {sorted(bad)}; choose from {WORKLOADS}", file=sys.stderr)
        sys.exit(2)
    run = set(only or WORKLOADS)
    if args.no_batch:
        run.discard("batch")
    if args.no_configs:
        run.discard("configs")
    if args.no_long:
        run.discard("long")
    if "extras" in run:
        run.add("headline")
    if "headline" not in run:
        out = {"metric": METRIC, "value": None, "unit": "Gpairs/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": "subset: " + ",".join(sorted(run))}}
        if "batch" in run:
            out["batch"] = batch_workload(args, mp, W, torch)
        if "configs" in run:
            out["configs"] = other_configs(args, mp, W, torch)
        if "long" in run:
            out["long_windows"] = long_windows(args, mp, W, torch)
        print(json.dumps(out), flush=True)
        return
    h = headline(args, mp, W, torch)
    f64 = h["fp64"]
    pairs = h["pairs"]
    ops = OPS_PER_PAIR["acamp"] * pairs
    achieved = ops / (f64["sweep_ms"] * 1e-3) / 1e12
    peak = PEAK_LANE_OPS / 1e12
    out = {
        "metric": METRIC,
        "value": round(f64["value"], 3),
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f64["ms_per_step"], 4),
        "ms_median": round(f64["ms_median"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "acamp_rw128k: z-normalized matrix profile, random walk n=131072 with 20 "
                        "constant runs and 10 planted motif pairs, m=256, excl=64",
            "n": h["n"], "m": h["m"], "excl": h["excl"], "pairs": pairs, "precision": "fp64",
            "refresh_rows": f64["refresh_rows"], "diags_per_lane": f64["diags_per_lane"],
            "items": f64["items"], "fallback_rows_per_step": f64["fallback_rows"],
            "autotune_ms": round(f64["autotune_ms"], 1),
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_sweep_band (ACAMP, FP64)",
            "achieved": round(achieved, 3),
            "peak": round(peak, 3),
            "unit": "Tlane-ops/s",
            "frac": round(achieved / peak, 4),
            "traffic": sweep_traffic(f64["refresh_rows"]),
            "ops_per_pair": OPS_PER_PAIR["acamp"],
            "kernel_ms": round(f64["sweep_ms"], 4),
        },
        "phases_ms_per_step": {
            "prep": round(f64["prep_ms"], 4),
            "sweep": round(f64["sweep_ms"], 4),
            "finalize": round(f64["finalize_ms"], 4),
        },
        "wall_s": round(f64["wall_s"], 3),
    }
    if "fp32" in h:
        f32 = h["fp32"]
        out["fp32_refresh"] = {
            "value": round(f32["value"], 3),
            "ms_per_step": round(f32["ms_per_step"], 4),
            "ms_median": round(f32["ms_median"], 4),
            "autotune_ms": round(f32["autotune_ms"], 1),
            "gain_vs_fp64": round(f32["value"] / f64["value"], 4),
            "rtol": 1e-4,
            "refresh_rows": f32["refresh_rows"],
            "diags_per_lane": f32["diags_per_lane"],
            "fallback_rows_per_step": f32["fallback_rows"],
            "phases_ms_per_step": {"prep": round(f32["prep_ms"], 4),
                                   "sweep": round(f32["sweep_ms"], 4),
                                   "finalize": round(f32["finalize_ms"], 4)},
            "sweep_gain_vs_fp64": round(f64["sweep_ms"] / f32["sweep_ms"], 4),
            "roofline": {"bound": "alu", "kernel": "k_sweep_band (ACAMP, FP32)",
                         "achieved": round(ops / (f32["sweep_ms"] * 1e-3) / 1e12, 3),
                         "peak": round(peak, 3), "unit": "Tlane-ops/s",
                         "frac": roofline_frac(ops, f32["sweep_ms"]),
                         "ops_per_pair": OPS_PER_PAIR["acamp"],
                         "kernel_ms": round(f32["sweep_ms"], 4)},
        }
    if "fp32_auto" in h:
        fa = h["fp32_auto"]
        out["fp32_auto"] = {
            "value": round(fa["value"], 3),
            "ms_per_step": round(fa["ms_per_step"], 4),
            "autotune_ms": round(fa["autotune_ms"], 1),
            "gain_vs_fp64": round(fa["value"] / f64["value"], 4),
            "rtol": 1e-4,
            "sweep": "fp32" if fa["fp32_jobs"] else "fp64",
            "refresh_rows": fa["refresh_rows"],
            "fallback_rows_per_step": fa["fallback_rows"],
        }
    if "extras" in run:
        extras(args, mp, h, torch, out)
    if "batch" in run:
        out["batch"] = batch_workload(args, mp, W, torch)
    if "configs" in run:
        out["configs"] = other_configs(args, mp, W, torch)
    if "long" in run:
        out["long_windows"] = long_windows(args, mp, W, torch)
    if args.copy_calib > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the ones read for the sweep
        src = torch.ones(args.copy_calib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = int(src.numel() * 8)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(h["T"], h["m"], h["excl"], "acamp", f64["P"], f64["I"],
                                           args.cpu_rows)
    print(json.dumps(out), flush=True)


def extras(args, mp, h, torch, out):
    """Motifs and discords, incremental appends, the anytime curve and the F
    comparator, all on the headline series."""
    f64 = h["fp64"]
    # motif / discord extraction on the headline profile (k = 10 each)
    Pd = torch.as_tensor(f64["P"], device="cuda")
    Id = torch.as_tensor(f64["I"], device="cuda")
    tk = {}
    for mode in ("motifs", "discords"):
        mp.topk(Pd, Id, 10, h["m"], mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            mp.topk(Pd, Id, 10, h["m"], mode)
        torch.cuda.synchronize()
        tk[mode + "_ms"] = round((time.perf_counter() - t0) / 5 * 1e3, 3)
    out["topk"] = {"k": 10, "excl": h["m"], **tk,
                   "note": "host wall time per call including the count read-back"}
    out["incremental"] = incremental(mp, h, torch)
    out["anytime"] = anytime_curve(mp, h, torch)
    out["acamp_fcmp"] = fcmp_variant(args, mp, h, torch)


if __name__ == "__main__":
    main()
