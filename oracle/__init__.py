"""FP64 CPU oracle for TRAKNN -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product path (the HIP library and its
Python binding) never imports, links or calls it, and shares no code with it.

The arithmetic lives in ``traknn_oracle.c`` (plain C, double precision, fixed
summation order, OpenMP over independent rows/pairs only). This module builds
that file with gcc on first use and marshals numpy arrays through ctypes.

What is computed (paper, Section 3.2):
  * Eq. 2: D_L(i, j) = sum_{m<L} ||X_{i+m} - X_{j+m}||^2 by direct differences;
  * exclusion zone |t - j| >= L (e = L - 1);
  * Eq. 3: s_t = mean of the k smallest D_L(t, j) over candidates, ties by the
    smaller j;
  * the gradient of sum_t w_t s_t with the neighbour sets held fixed;
  * the local intrinsic dimension of Section 5.1 (Levina-Bickel maximum
    likelihood kNN estimator) from the sorted neighbour distances.

Pins (what ties this code to something other than itself) are in
``tests/test_oracle_pins.py``; every function here is pinned there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "traknn_oracle.c")
_LIB = os.path.join(_HERE, "libtraknn_oracle.so")
_lock = threading.Lock()
_lib = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fopenmp", "-fno-fast-math",
            "-ffp-contract=off", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i64, i32 = ctypes.c_int64, ctypes.c_int
            lib.oracle_snapshot_dist.argtypes = [_f64p, i64, i64, _f64p]
            lib.oracle_traj_dist_from_snapshot.argtypes = [_f64p, i64, i32, _f64p]
            lib.oracle_traj_dist_rows.argtypes = [_f64p, i64, i64, i32, _i64p, i64, _f64p]
            lib.oracle_traj_dist_rows_multi.argtypes = [_f64p, i64, i64, i32, _i64p, i64,
                                                        _f64p]
            lib.oracle_pair_traj_dist.argtypes = [_f64p, i64, i64, i32, _i64p, _i64p, i64, _f64p]
            lib.oracle_knn_rows.argtypes = [_f64p, _i64p, i64, i64, i32, i32, _i32p,
                                            _f64p, _f64p, _f64p]
            lib.oracle_score_grad.argtypes = [_f64p, i64, i64, i32, i32, _i32p, _f64p, _f64p]
            lib.oracle_local_dim.argtypes = [_f64p, i64, i32, _f64p]
            lib.oracle_num_threads.argtypes = []
            for f in (lib.oracle_snapshot_dist, lib.oracle_traj_dist_from_snapshot,
                      lib.oracle_traj_dist_rows, lib.oracle_traj_dist_rows_multi,
                      lib.oracle_pair_traj_dist,
                      lib.oracle_knn_rows, lib.oracle_score_grad, lib.oracle_local_dim,
                      lib.oracle_num_threads):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")


def _x64(X) -> np.ndarray:
    X = np.asarray(X)
    if X.ndim == 1:
        X = X[:, None]
    if X.ndim > 2:
        X = X.reshape(X.shape[0], -1)
    return np.ascontiguousarray(X, dtype=np.float64)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def snapshot_dist(X) -> np.ndarray:
    """S[i, j] = ||X_i - X_j||^2 (T x T), direct differences."""
    X = _x64(X)
    T, D = X.shape
    S = np.empty((T, T), dtype=np.float64)
    _check(_load().oracle_snapshot_dist(X, T, D, S), "snapshot_dist")
    return S


def traj_dist_from_snapshot(S, L: int) -> np.ndarray:
    """D_L (n' x n') as direct sums over m of a snapshot matrix S (T x T)."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    T = S.shape[0]
    n = T - L + 1
    Dm = np.empty((n, n), dtype=np.float64)
    _check(_load().oracle_traj_dist_from_snapshot(S, T, int(L), Dm), "traj_dist")
    return Dm


def traj_dist(X, L: int) -> np.ndarray:
    """Full trajectory distance matrix D_L (n' x n'), Eq. 2 as a direct sum."""
    S = snapshot_dist(X)
    T = S.shape[0]
    n = T - L + 1
    Dm = np.empty((n, n), dtype=np.float64)
    _check(_load().oracle_traj_dist_from_snapshot(S, T, int(L), Dm), "traj_dist")
    return Dm


def traj_dist_rows(X, L: int, rows) -> np.ndarray:
    """Rows D_L(t, :) for t in ``rows``, straight from X (no S)."""
    X = _x64(X)
    T, D = X.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.size, T - L + 1), dtype=np.float64)
    _check(_load().oracle_traj_dist_rows(X, T, D, int(L), rows, rows.size, out),
           "traj_dist_rows")
    return out


def traj_dist_rows_multi(X, L_max: int, rows) -> np.ndarray:
    """Rows D_L(t, :) for every L = 1..L_max, straight from X: [L_max, r, T],
    entry [L-1, r, j] = D_L(rows[r], j) for j < T - L + 1, +inf beyond."""
    X = _x64(X)
    T, D = X.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((L_max, rows.size, T), dtype=np.float64)
    _check(_load().oracle_traj_dist_rows_multi(X, T, D, int(L_max), rows, rows.size, out),
           "traj_dist_rows_multi")
    return out


def knn_rows_multi(X, L_max: int, k: int, rows):
    """Sampled rows of every length L = 1..L_max from one pass over X: a list
    whose entry L - 1 is (idx, dist, score, gap, drows) as knn_rows returns
    them for length L (rows must exist for L_max)."""
    allrows = traj_dist_rows_multi(X, L_max, rows)
    T = allrows.shape[2]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = []
    for L in range(1, L_max + 1):
        drows = np.ascontiguousarray(allrows[L - 1, :, :T - L + 1])
        out.append(knn_from_rows(drows, rows, L, k) + (drows,))
    return out


def pair_traj_dist(X, L: int, ti, tj) -> np.ndarray:
    X = _x64(X)
    T, D = X.shape
    ti = np.ascontiguousarray(ti, dtype=np.int64).ravel()
    tj = np.ascontiguousarray(tj, dtype=np.int64).ravel()
    out = np.empty(ti.size, dtype=np.float64)
    _check(_load().oracle_pair_traj_dist(X, T, D, int(L), ti, tj, ti.size, out),
           "pair_traj_dist")
    return out


def knn_from_rows(drows, rows, L: int, k: int):
    """Exclusion-zone kNN + score on precomputed rows of D_L.

    Returns (idx [r,k] int32, dist [r,k], score [r], gap [r])."""
    drows = np.ascontiguousarray(drows, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    nr, n = drows.shape
    idx = np.empty((nr, k), dtype=np.int32)
    dist = np.empty((nr, k), dtype=np.float64)
    score = np.empty(nr, dtype=np.float64)
    gap = np.empty(nr, dtype=np.float64)
    _check(_load().oracle_knn_rows(drows, rows, nr, n, int(L), int(k), idx, dist,
                                   score, gap), "knn_rows")
    return idx, dist, score, gap


def knn(X, L: int, k: int):
    """All rows: (idx [n',k], dist [n',k], score [n'], gap [n'])."""
    Dm = traj_dist(X, L)
    rows = np.arange(Dm.shape[0], dtype=np.int64)
    return knn_from_rows(Dm, rows, L, k)


def knn_rows(X, L: int, k: int, rows):
    """Sampled rows straight from X, for sizes where S does not fit:
    (idx, dist, score, gap, drows)."""
    drows = traj_dist_rows(X, L, rows)
    return knn_from_rows(drows, rows, L, k) + (drows,)


def local_dim(dist) -> np.ndarray:
    """Levina-Bickel maximum-likelihood local intrinsic dimension (the
    estimator of Section 5.1) from sorted squared neighbour distances
    ``dist`` [r, k]: out[:, q] is the estimate from the q + 1 nearest
    (column 0, one neighbour, is NaN)."""
    dist = np.ascontiguousarray(dist, dtype=np.float64)
    r, k = dist.shape
    out = np.empty((r, k), dtype=np.float64)
    _check(_load().oracle_local_dim(dist, r, int(k), out), "local_dim")
    return out


def score_grad(X, L: int, k: int, idx, w) -> np.ndarray:
    """d(sum_t w_t s_t)/dX with neighbour sets ``idx`` (n' x k) held fixed."""
    X = _x64(X)
    T, D = X.shape
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    if idx.shape != (T - L + 1, k) or w.shape != (T - L + 1,):
        raise ValueError("idx must be (n', k) and w (n',)")
    g = np.empty((T, D), dtype=np.float64)
    _check(_load().oracle_score_grad(X, T, D, int(L), int(k), idx, w, g), "score_grad")
    return g
