"""CPU oracle for the Manifold k-NN query path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It shares no code with the HIP path and imports nothing from it.

Contents:
  * ``knn_bruteforce`` -- FP64 brute-force k-NN over the prefix P_{1:m} (C, OpenMP), the
    plain definition the method reaches exactly (Sec. 3 Eq. 2, Theorem 1, Sec. 4.2
    prefix-subset queries, Sec. 4.3 deletion equivalence).
  * ``successors.successor_lists`` -- exact brute-force successor lists (Sec. 3: p_j joins
    L_i iff inserting p_j prunes the Voronoi cell of p_i), for tiny clouds.
  * ``dpknn.dp_knn`` -- the steps of Alg. 1 and Alg. 2 on given lists, to check that a
    successor table answers k-NN exactly and to count the work per query.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knn_bruteforce.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_knn.argtypes = [P, ctypes.c_int64, P, P, ctypes.c_int64, P, ctypes.c_int32,
                                   P, ctypes.c_int64, P, P, P, P, ctypes.c_int]
        lib.oracle_knn.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def knn_bruteforce(points_by_rank: np.ndarray, queries: np.ndarray, k: int = 0,
                   m: Optional[int] = None, live: Optional[np.ndarray] = None,
                   k_per_query: Optional[np.ndarray] = None,
                   m_per_query: Optional[np.ndarray] = None, threads: int = 0):
    """Exact k-NN by exhaustive FP64 scan.

    Returns (idx int32, dist float32, D float64).  With a scalar k the arrays are [nq, k];
    with ``k_per_query`` they are flat, row i occupying [row_off[i], row_off[i+1]) where
    row_off = concatenate([0], cumsum(k_per_query)), and row_off is returned as a 4th item.
    """
    lib = _load()
    P = np.ascontiguousarray(points_by_rank, dtype=np.float32)
    Q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, 3)
    n = P.shape[0]
    nq = Q.shape[0]
    lv = None if live is None else np.ascontiguousarray(live, dtype=np.uint8)
    mm = n if m is None else int(m)
    marr = None if m_per_query is None else np.ascontiguousarray(m_per_query, dtype=np.int32)
    if k_per_query is not None:
        karr = np.ascontiguousarray(k_per_query, dtype=np.int32)
        row_off = np.zeros(nq + 1, dtype=np.int64)
        np.cumsum(karr, out=row_off[1:])
        tot = int(row_off[-1])
        idx = np.empty(tot, dtype=np.int32)
        dist = np.empty(tot, dtype=np.float32)
        D = np.empty(tot, dtype=np.float64)
        rc = lib.oracle_knn(_ptr(P), n, _ptr(lv), _ptr(Q), nq, _ptr(karr), 0, _ptr(marr), mm,
                            _ptr(row_off), _ptr(idx), _ptr(dist), _ptr(D), threads)
        if rc != 0:
            raise ValueError("oracle_knn rejected its arguments")
        return idx, dist, D, row_off
    k = int(k)
    idx = np.empty((nq, k), dtype=np.int32)
    dist = np.empty((nq, k), dtype=np.float32)
    D = np.empty((nq, k), dtype=np.float64)
    rc = lib.oracle_knn(_ptr(P), n, _ptr(lv), _ptr(Q), nq, None, k, _ptr(marr), mm, None,
                        _ptr(idx), _ptr(dist), _ptr(D), threads)
    if rc != 0:
        raise ValueError("oracle_knn rejected its arguments")
    return idx, dist, D
