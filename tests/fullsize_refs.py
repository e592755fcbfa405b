"""Stored oracle rows of the full-size workloads (test helper).

The files under tests/golden/fullsize/ are written by
tests/golden/make_fullsize_refs.py, which calls only the oracle and the
seeded generators. load() regenerates nothing: the caller passes the series
it generated, and load() checks it against the SHA-256 stored with the rows
(a changed generator must not be checked against stale answers)."""
import hashlib
import os

import numpy as np

DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize")


def series_hash(T) -> str:
    return hashlib.sha256(np.ascontiguousarray(T, dtype=np.float64).tobytes()).hexdigest()


def batch_hash(series) -> str:
    return hashlib.sha256(b"".join(np.ascontiguousarray(T, dtype=np.float64).tobytes()
                                   for T in series)).hexdigest()


def path(name: str) -> str:
    return os.path.join(DIR, name + ".npz")


def load(name: str, T=None, series=None):
    """(rows, P, I, Q) of a stored file (plus ``job`` for the batch file),
    after checking the stored hash against T (or the batch's series)."""
    z = np.load(path(name))
    if T is not None:
        assert str(z["series_sha256"]) == series_hash(T), f"{name}: the series changed"
    if series is not None:
        assert str(z["series_sha256"]) == batch_hash(series), f"{name}: the batch changed"
    n_done = len(z["P"])
    out = {k: z[k] for k in z.files}
    out["rows"] = out["rows"][:n_done]
    return out
