"""Python binding of libmp (include/mp.h): matrix profiles on an MI355X.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libmp.so. PyTorch supplies device memory and the stream. There is
no CPU fallback: importing works without a GPU, but every call needs the
built library and a gfx950 device and raises otherwise.

    import torch, paper_1901_05708_amd as mp
    T = torch.as_tensor(series, dtype=torch.float64, device="cuda")
    P, I = mp.aamp(T, m=64)                     # pure Euclidean (AAMP)
    P, I = mp.pnorm(T, m=128, p=3.0)            # p-norm
    P, I = mp.acamp(T, m=256, precision="fp32") # z-normalized (ACAMP)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
# MP_LIBRARY selects another build of the same library (e.g. a debug build).
LIB_PATH = os.environ.get("MP_LIBRARY") or os.path.join(_HERE, "libmp.so")

MP_OK, MP_EINVAL, MP_ENOMEM, MP_EHIP, MP_EUNSUPPORTED = 0, -1, -2, -3, -4
MP_FP64, MP_FP32_REFRESH, MP_FP32_AUTO = 0, 1, 2
KIND_AAMP, KIND_PNORM, KIND_ACAMP = 0, 1, 2
FP32_RTOL = 1e-4

EXPORTED = ("mp_aamp", "mp_pnorm", "mp_acamp", "mp_acamp_fcmp", "mp_profile_noalloc", "mp_batch",
            "mp_topk", "mp_anytime",
            "mp_anytime_groups", "mp_anytime_order", "mp_inc_create", "mp_inc_append",
            "mp_inc_state", "mp_inc_read", "mp_inc_destroy", "mp_strerror", "mp_release",
            "mp_set_profiling", "mp_profile_read")
ANYTIME_GROUP = 512
MP_MOTIFS, MP_DISCORDS = 0, 1
NOALLOC_MAX_N = 1 << 18


class MpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libmp error {code}: {msg}")
        self.code = code


class MpJob(ctypes.Structure):
    _fields_ = [("t_off", ctypes.c_int64), ("n", ctypes.c_int64), ("out_off", ctypes.c_int64),
                ("m", ctypes.c_int32), ("kind", ctypes.c_int32), ("excl", ctypes.c_int32),
                ("R", ctypes.c_int32), ("p", ctypes.c_double)]


class MpStats(ctypes.Structure):
    _fields_ = [("ms_prep", ctypes.c_double), ("ms_sweep", ctypes.c_double),
                ("ms_finalize", ctypes.c_double), ("ms_autotune", ctypes.c_double),
                ("pairs", ctypes.c_int64), ("fallback_rows", ctypes.c_int64),
                ("pairs_visited", ctypes.c_int64),
                ("calls", ctypes.c_int32), ("sweep_launches", ctypes.c_int32),
                ("refresh_rows", ctypes.c_int32), ("diags_per_lane", ctypes.c_int32),
                ("items", ctypes.c_int32), ("graph_replays", ctypes.c_int32),
                ("band_jobs", ctypes.c_int32), ("fp32_jobs", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load libmp.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1901_05708_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.mp_aamp.argtypes = [vp, i64, i32, i32, i32, i32, vp, vp, vp]
    lib.mp_pnorm.argtypes = [vp, i64, i32, dbl, i32, i32, i32, vp, vp, vp]
    lib.mp_acamp.argtypes = [vp, i64, i32, i32, i32, i32, vp, vp, vp]
    lib.mp_acamp_fcmp.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp]
    lib.mp_acamp_fcmp.restype = ctypes.c_int
    lib.mp_profile_noalloc.argtypes = [i32, vp, i64, i32, dbl, i32, i32, i32, vp, vp, vp]
    lib.mp_profile_noalloc.restype = ctypes.c_int
    lib.mp_batch.argtypes = [vp, ctypes.POINTER(MpJob), i32, i32, vp, vp, vp]
    for f in (lib.mp_aamp, lib.mp_pnorm, lib.mp_acamp, lib.mp_batch):
        f.restype = ctypes.c_int
    lib.mp_topk.argtypes = [vp, vp, i64, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.mp_anytime.argtypes = [i32, vp, i64, i32, dbl, i32, vp, i64, i32, vp, vp, vp]
    lib.mp_anytime.restype = ctypes.c_int
    lib.mp_anytime_groups.argtypes = [i64, i32, i32, ctypes.POINTER(i64)]
    lib.mp_anytime_groups.restype = ctypes.c_int
    lib.mp_anytime_order.argtypes = [i64, i32, i32, ctypes.c_uint64, vp, vp]
    lib.mp_anytime_order.restype = ctypes.c_int
    lib.mp_topk.restype = ctypes.c_int
    lib.mp_inc_create.argtypes = [i32, i32, dbl, i32, i64, i32, ctypes.POINTER(vp)]
    lib.mp_inc_create.restype = ctypes.c_int
    lib.mp_inc_append.argtypes = [vp, vp, i64, vp]
    lib.mp_inc_append.restype = ctypes.c_int
    lib.mp_inc_state.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp]
    lib.mp_inc_state.restype = ctypes.c_int
    lib.mp_inc_read.argtypes = [vp, vp, vp, vp]
    lib.mp_inc_read.restype = ctypes.c_int
    lib.mp_inc_destroy.argtypes = [vp]
    lib.mp_inc_destroy.restype = None
    lib.mp_strerror.argtypes = [ctypes.c_int]
    lib.mp_strerror.restype = ctypes.c_char_p
    lib.mp_release.argtypes = []
    lib.mp_release.restype = None
    lib.mp_set_profiling.argtypes = [ctypes.c_int]
    lib.mp_set_profiling.restype = None
    lib.mp_profile_read.argtypes = [ctypes.POINTER(MpStats)]
    lib.mp_profile_read.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != MP_OK:
        raise MpError(rc, load().mp_strerror(rc).decode())


def _prec(precision) -> int:
    if precision in ("fp64", MP_FP64):
        return MP_FP64
    if precision in ("fp32", "fp32_refresh", MP_FP32_REFRESH):
        return MP_FP32_REFRESH
    if precision in ("fp32_auto", MP_FP32_AUTO):
        return MP_FP32_AUTO
    raise ValueError(f"unknown precision {precision!r}")


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check_values(T):
    """The ABI's precondition on the samples: finite, |t| < 1e30 (this reads
    the tensor back, so it synchronises with the device)."""
    import torch
    if T.numel() and not bool(torch.all(torch.isfinite(T) & (T.abs() < 1e30))):
        raise ValueError("T must be finite with |t| < 1e30")


def _series(T, m: int, validate: bool = True):
    import torch
    if not isinstance(T, torch.Tensor) or T.device.type != "cuda":
        raise TypeError("T must be a torch tensor on a HIP (cuda) device")
    if T.dtype != torch.float64 or T.dim() != 1:
        raise TypeError("T must be a 1-D float64 tensor")
    T = T.contiguous()
    if validate:
        _check_values(T)
    n = T.shape[0]
    if not (1 <= m <= n):
        raise ValueError("need 1 <= m <= len(T)")
    N = n - m + 1
    P = torch.empty(N, dtype=torch.float64, device=T.device)
    I = torch.empty(N, dtype=torch.int64, device=T.device)
    return T, n, N, P, I


def aamp(T, m: int, excl: Optional[int] = None, precision="fp64", R: int = 0, stream=None,
         validate: bool = True):
    """Pure Euclidean matrix profile (mp_aamp). Returns (P, I) tensors.
    validate=True first checks the ABI's precondition on T (finite, |t| <
    1e30), which synchronises with the device; pass False in timed loops."""
    T, n, N, P, I = _series(T, m, validate)
    _check(load().mp_aamp(T.data_ptr(), n, m, excl or 0, _prec(precision), R,
                          P.data_ptr(), I.data_ptr(), _stream(stream)))
    return P, I


def pnorm(T, m: int, p: float, excl: Optional[int] = None, precision="fp64", R: int = 0,
          stream=None, validate: bool = True):
    """p-norm matrix profile (mp_pnorm), real p >= 1. Returns (P, I)."""
    T, n, N, P, I = _series(T, m, validate)
    _check(load().mp_pnorm(T.data_ptr(), n, m, float(p), excl or 0, _prec(precision), R,
                           P.data_ptr(), I.data_ptr(), _stream(stream)))
    return P, I


def acamp(T, m: int, excl: Optional[int] = None, precision="fp64", R: int = 0, stream=None,
         validate: bool = True):
    """z-normalized matrix profile (mp_acamp). Returns (P, I)."""
    T, n, N, P, I = _series(T, m, validate)
    _check(load().mp_acamp(T.data_ptr(), n, m, excl or 0, _prec(precision), R,
                           P.data_ptr(), I.data_ptr(), _stream(stream)))
    return P, I


def profile_noalloc(T, m: int, kind: str = "aamp", p: float = 2.0, excl: Optional[int] = None,
                    precision="fp64", R: int = 0, P=None, I=None, stream=None,
                    validate: bool = True):
    """mp_aamp / mp_pnorm / mp_acamp without device allocation inside the
    library (mp_profile_noalloc): at most NOALLOC_MAX_N windows, R = 0 takes
    the default interval (no autotuning). P, I may be preallocated outputs
    (contiguous float64 / int64 tensors of N entries). Returns (P, I)."""
    import torch
    T, n, N, P0, I0 = _series(T, m, validate) if P is None else _series_noout(T, m, validate)
    if P is None:
        P, I = P0, I0
    elif (I is None or P.dtype != torch.float64 or I.dtype != torch.int64 or P.numel() != N
          or I.numel() != N or not P.is_contiguous() or not I.is_contiguous()):
        raise TypeError("P, I must be contiguous float64 / int64 tensors of N entries")
    _check(load().mp_profile_noalloc(_KIND_OF[kind], T.data_ptr(), n, int(m), float(p),
                                     int(excl or 0), _prec(precision), R, P.data_ptr(),
                                     I.data_ptr(), _stream(stream)))
    return P, I


def _series_noout(T, m: int, validate: bool):
    import torch
    if not isinstance(T, torch.Tensor) or T.device.type != "cuda":
        raise TypeError("T must be a torch tensor on a HIP (cuda) device")
    if T.dtype != torch.float64 or T.dim() != 1:
        raise TypeError("T must be a 1-D float64 tensor")
    T = T.contiguous()
    if validate:
        _check_values(T)
    n = T.shape[0]
    if not (1 <= m <= n):
        raise ValueError("need 1 <= m <= len(T)")
    return T, n, n - m + 1, None, None


def acamp_fcmp(T, m: int, excl: Optional[int] = None, R: int = 0, stream=None,
               validate: bool = True):
    """z-normalized matrix profile with the sweep comparing pairs on the F
    of Sec. 4.4 instead of rho (mp_acamp_fcmp; FP64). Returns (P, I)."""
    T, n, N, P, I = _series(T, m, validate)
    _check(load().mp_acamp_fcmp(T.data_ptr(), n, m, excl or 0, R, P.data_ptr(), I.data_ptr(),
                                _stream(stream)))
    return P, I


@dataclass
class Job:
    n: int
    m: int
    kind: int = KIND_AAMP
    excl: int = 0
    R: int = 0
    p: float = 2.0


def batch_layout(jobs: Sequence[Job]):
    """Offsets (t_off, out_off) and totals for concatenated series/outputs."""
    table = (MpJob * len(jobs))()
    t_off = out_off = 0
    for b, jb in enumerate(jobs):
        table[b] = MpJob(t_off, jb.n, out_off, jb.m, jb.kind, jb.excl, jb.R, jb.p)
        t_off += jb.n
        out_off += jb.n - jb.m + 1
    return table, t_off, out_off


def batch(T_cat, jobs: Sequence[Job], precision="fp64", stream=None, out=None, table=None,
          validate: bool = True):
    """Matrix profiles of many series in one call (mp_batch). T_cat is the
    concatenation of the series; returns (P_cat, I_cat) with each job's
    outputs at its out_off (see batch_layout). Passing the same `out` tensors
    (and T_cat) again replays the library's captured graph of the batch;
    `table` may hold a prebuilt batch_layout() table to skip rebuilding it."""
    import torch
    if table is None:
        table, total_n, total_out = batch_layout(jobs)
    else:
        total_n = sum(jb.n for jb in jobs)
        total_out = sum(jb.n - jb.m + 1 for jb in jobs)
    if T_cat.dtype != torch.float64 or T_cat.device.type != "cuda" or T_cat.shape[0] < total_n:
        raise TypeError("T_cat must be a float64 cuda tensor holding every series")
    T_cat = T_cat.contiguous()
    if validate:
        _check_values(T_cat[:total_n])
    if out is None:
        P = torch.empty(max(total_out, 1), dtype=torch.float64, device=T_cat.device)
        I = torch.empty(max(total_out, 1), dtype=torch.int64, device=T_cat.device)
    else:
        P, I = out
    _check(load().mp_batch(T_cat.data_ptr(), table, len(jobs), _prec(precision),
                           P.data_ptr(), I.data_ptr(), _stream(stream)))
    return P, I


def topk(P, I, k: int, excl: int, mode: str = "motifs", stream=None):
    """Motifs (mode="motifs": smallest profile values, each pair once) or
    discords (mode="discords": largest values) of a profile (P, I) computed
    by aamp / pnorm / acamp, with exclusion zone excl (mp_topk). Returns
    (i, j, d) tensors: window, its nearest neighbour, distance. Reads the
    result count back, so it synchronises with the stream."""
    import torch
    if mode not in ("motifs", "discords"):
        raise ValueError("mode must be 'motifs' or 'discords'")
    if P.device.type != "cuda" or P.dtype != torch.float64 or I.dtype != torch.int64:
        raise TypeError("P must be float64 and I int64 tensors on a HIP device")
    P, I = P.contiguous(), I.contiguous()
    k = int(k)
    oi = torch.empty(max(k, 1), dtype=torch.int64, device=P.device)
    oj = torch.empty(max(k, 1), dtype=torch.int64, device=P.device)
    od = torch.empty(max(k, 1), dtype=torch.float64, device=P.device)
    cnt = torch.zeros(1, dtype=torch.int32, device=P.device)
    _check(load().mp_topk(P.data_ptr(), I.data_ptr(), P.shape[0], k, int(excl),
                          MP_MOTIFS if mode == "motifs" else MP_DISCORDS, oi.data_ptr(),
                          oj.data_ptr(), od.data_ptr(), cnt.data_ptr(), _stream(stream)))
    c = int(cnt.item())
    return oi[:c], oj[:c], od[:c]


_KIND_OF = {"aamp": KIND_AAMP, "pnorm": KIND_PNORM, "acamp": KIND_ACAMP}


def anytime_groups(n: int, m: int, excl: Optional[int] = None) -> int:
    """Number of diagonal groups (ANYTIME_GROUP diagonals each) of a series
    (mp_anytime_groups; host only)."""
    G = ctypes.c_int64()
    _check(load().mp_anytime_groups(int(n), int(m), int(excl or 0), ctypes.byref(G)))
    return G.value


def anytime_order(n: int, m: int, excl: Optional[int] = None, seed: int = 0):
    """Seeded random order of the diagonal groups and the admissible pairs
    covered after each prefix of it (mp_anytime_order; host only). Returns
    (order int32, cum_pairs int64) numpy arrays."""
    import numpy as np
    G = anytime_groups(n, m, excl)
    order = np.empty(G, dtype=np.int32)
    cum = np.empty(G, dtype=np.int64)
    _check(load().mp_anytime_order(int(n), int(m), int(excl or 0),
                                   ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                   order.ctypes.data_as(ctypes.c_void_p),
                                   cum.ctypes.data_as(ctypes.c_void_p)))
    return order, cum


def anytime(T, m: int, groups, kind: str = "aamp", p: float = 2.0, excl: Optional[int] = None,
            P=None, I=None, stream=None, validate: bool = True):
    """Profile over the diagonals of the listed groups (mp_anytime). With P
    and I given (an earlier result for the same series and arguments) the
    call resumes: rows keep the better of their entry and the new candidates,
    and P, I are updated in place. Returns (P, I)."""
    import numpy as np
    import torch
    T, n, N, P0, I0 = _series(T, m, validate)
    resume = P is not None or I is not None
    if resume:
        if P is None or I is None:
            raise ValueError("resume needs both P and I")
        if (P.dtype != torch.float64 or I.dtype != torch.int64 or P.numel() != N
                or I.numel() != N or not P.is_contiguous() or not I.is_contiguous()):
            raise TypeError("P, I must be contiguous float64 / int64 tensors of N entries")
    else:
        P, I = P0, I0
    g = np.ascontiguousarray(np.asarray(groups, dtype=np.int64))
    if g.size and (g.min() < 0 or g.max() > 2**31 - 1):
        raise ValueError("group index out of range")
    g = g.astype(np.int32)
    _check(load().mp_anytime(_KIND_OF[kind], T.data_ptr(), n, int(m), float(p), int(excl or 0),
                             g.ctypes.data_as(ctypes.c_void_p) if g.size else None, int(g.size),
                             1 if resume else 0, P.data_ptr(), I.data_ptr(), _stream(stream)))
    return P, I


class Anytime:
    """Anytime profile of one series: the diagonal groups in a seeded random
    order, swept a share of the pairs at a time. After advance(f) the profile
    covers at least the fraction f of all admissible pairs; every P[i] is the
    exact distance of (i, I[i]) and never increases with later calls.

        a = Anytime(T, m=256, kind="acamp", seed=1)
        P, I = a.advance(0.1)        # about 10 % of the pairs
        P, I = a.advance(1.0)        # the exact profile
    """

    def __init__(self, T, m: int, kind: str = "aamp", p: float = 2.0,
                 excl: Optional[int] = None, seed: int = 0):
        import torch
        self.T, self.m, self.kind, self.p, self.excl = T, m, kind, p, excl
        self.order, self.cum = anytime_order(T.numel(), m, excl, seed)
        self.done = 0                 # groups swept so far (a prefix of order)
        N = T.numel() - m + 1
        self.P = torch.full((N,), float("inf"), dtype=torch.float64, device=T.device)
        self.I = torch.full((N,), -1, dtype=torch.int64, device=T.device)

    @property
    def covered(self) -> float:
        """Fraction of the admissible pairs swept so far."""
        total = int(self.cum[-1]) if self.cum.size else 0
        return 1.0 if total == 0 else (int(self.cum[self.done - 1]) if self.done else 0) / total

    def advance(self, fraction: float, stream=None):
        import numpy as np
        total = int(self.cum[-1]) if self.cum.size else 0
        if fraction >= 1.0:
            want = self.order.size
        elif fraction <= 0.0:
            want = self.done
        else:   # the shortest prefix whose pairs reach the fraction
            want = int(np.searchsorted(self.cum, fraction * total, side="left")) + 1
        want = min(max(want, self.done), self.order.size)
        if want > self.done:
            anytime(self.T, self.m, self.order[self.done:want], self.kind, self.p, self.excl,
                    P=self.P, I=self.I, stream=stream, validate=self.done == 0)
            self.done = want
        return self.P, self.I


class Incremental:
    """Profile of a growing series (mp_inc_*): append samples, read the
    profile of everything appended so far.

        inc = Incremental(m=64, kind="acamp", capacity=1 << 20)
        inc.append(chunk)            # float64 HIP tensor
        P, I = inc.profile()
    """

    _KINDS = {"aamp": KIND_AAMP, "pnorm": KIND_PNORM, "acamp": KIND_ACAMP}

    def __init__(self, m: int, kind: str = "aamp", p: float = 2.0, excl: Optional[int] = None,
                 capacity: int = 1 << 20, refresh: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.mp_inc_create(int(m), self._KINDS[kind], float(p), int(excl or 0),
                                 int(capacity), int(refresh), ctypes.byref(h)))
        self._h = h
        self.m = m

    def append(self, T, stream=None):
        import torch
        if not isinstance(T, torch.Tensor) or T.device.type != "cuda" or T.dtype != torch.float64:
            raise TypeError("T must be a float64 tensor on a HIP device")
        T = T.contiguous().view(-1)
        _check(load().mp_inc_append(self._h, T.data_ptr(), T.numel(), _stream(stream)))

    def size(self):
        n, N = ctypes.c_int64(), ctypes.c_int64()
        _check(load().mp_inc_state(self._h, ctypes.byref(n), ctypes.byref(N), None, None))
        return n.value, N.value

    def profile(self, stream=None):
        """(P, I) of the series appended so far, as new tensors."""
        import torch
        n, N = self.size()
        P = torch.empty(max(N, 0), dtype=torch.float64, device="cuda")
        I = torch.empty(max(N, 0), dtype=torch.int64, device="cuda")
        if N > 0:
            _check(load().mp_inc_read(self._h, P.data_ptr(), I.data_ptr(), _stream(stream)))
        return P, I

    def close(self):
        if self._h:
            load().mp_inc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def release():
    load().mp_release()


def set_profiling(on: bool):
    load().mp_set_profiling(1 if on else 0)


def profile_read() -> dict:
    st = MpStats()
    _check(load().mp_profile_read(ctypes.byref(st)))
    return st.as_dict()


def pair_count(n: int, m: int, excl: int) -> int:
    """Admissible unordered pairs (i < j, j - i >= excl) of a series."""
    N = n - m + 1
    if N <= excl:
        return 0
    k = N - excl
    return k * (k + 1) // 2


def default_excl(m: int) -> int:
    return (m + 3) // 4
