"""CPU FP64 oracle for tree field integration.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg are the only users. The library never imports
this package, and this package imports nothing from the library; it shares
no code with the device path.

The oracle is the plain definition of the problem (Section 1, equation
"integration"; Section 2, equation "stad-target"):
``out[v] = sum_w f(dist_T(v, w)) F[w]`` with exact integer tree distances
from one traversal per source row and compensated FP64 sums. See
``tfi_oracle.c`` for the C implementation this module wraps.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tfi_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None


class OracleError(RuntimeError):
    pass


_CODES = {-1: "bad argument", -2: "malformed tree", -3: "bad weight / overflow",
          -4: "kernel table shorter than a distance that occurs"}


def build(force=False):
    """Compile the oracle with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        p = C.c_void_p
        i64 = C.c_int64
        lib.oracle_integrate.argtypes = [i64, p, p, p, i64, p, i64, p, i64, p, C.c_int]
        lib.oracle_pair_hist.argtypes = [i64, p, p, p, p, i64, p, i64, p, i64, C.c_int]
        lib.oracle_distances.argtypes = [i64, p, p, p, i64, p]
        lib.oracle_diameter.argtypes = [i64, p, p, p]
        lib.oracle_expdp.argtypes = [i64, p, p, p, p, i64, p, i64, p]
        lib.oracle_num_threads.argtypes = [C.c_int]
        for fn in (lib.oracle_integrate, lib.oracle_pair_hist,
                   lib.oracle_distances, lib.oracle_diameter,
                   lib.oracle_expdp, lib.oracle_num_threads):
            fn.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _tree(parent, weight):
    parent = np.ascontiguousarray(parent, dtype=np.int64)
    weight = np.ascontiguousarray(weight, dtype=np.int32)
    if parent.shape != weight.shape or parent.ndim != 1:
        raise OracleError("parent and weight must be 1-D of equal length")
    return parent, weight


def _check(rc):
    if rc:
        raise OracleError(_CODES.get(rc, f"error {rc}"))


def num_threads(n=0):
    return _load().oracle_num_threads(int(n))


def integrate(parent, weight, f, F, rows=None, threads=0):
    """``out[i] = sum_w f[dist(rows[i], w)] * F[w]`` in FP64 (all vertices
    when ``rows`` is None). ``F`` may be 1-D (one channel) or [N x d]."""
    lib = _load()
    parent, weight = _tree(parent, weight)
    F = np.asarray(F, dtype=np.float64)
    vec = F.ndim == 1
    F2 = np.ascontiguousarray(F.reshape(len(parent), 1) if vec else F)
    if F2.ndim != 2 or F2.shape[0] != len(parent):
        raise OracleError("F must be [N] or [N x d]")
    d = F2.shape[1]
    f = np.ascontiguousarray(f, dtype=np.float64)
    if rows is None:
        r = None
        nr = len(parent)
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        nr = len(r)
    out = np.zeros((nr, d), dtype=np.float64)
    _check(lib.oracle_integrate(len(parent), _ptr(parent), _ptr(weight),
                                _ptr(f), len(f), _ptr(F2), d, _ptr(r), nr,
                                _ptr(out), int(threads)))
    return out[:, 0] if vec else out


def pair_hist(parent, weight, G, F, length, rows=None, threads=0):
    """``h[k] = sum_{v in rows, w : dist(v,w) = k} <G[v], F[w]>``."""
    lib = _load()
    parent, weight = _tree(parent, weight)
    n = len(parent)
    G2 = np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(n, -1))
    F2 = np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(n, -1))
    if G2.shape != F2.shape:
        raise OracleError("G and F must have the same shape")
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = n if r is None else len(r)
    h = np.zeros(int(length), dtype=np.float64)
    _check(lib.oracle_pair_hist(n, _ptr(parent), _ptr(weight), _ptr(G2),
                                _ptr(F2), G2.shape[1], _ptr(r), nr, _ptr(h),
                                len(h), int(threads)))
    return h


def distances(parent, weight, rows=None):
    """Exact integer distance rows (``-1`` between trees of a forest)."""
    lib = _load()
    parent, weight = _tree(parent, weight)
    n = len(parent)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = n if r is None else len(r)
    D = np.empty((nr, n), dtype=np.int64)
    _check(lib.oracle_distances(n, _ptr(parent), _ptr(weight), _ptr(r), nr,
                                _ptr(D)))
    return D


def diameter(parent, weight):
    lib = _load()
    parent, weight = _tree(parent, weight)
    out = np.zeros(1, dtype=np.int64)
    _check(lib.oracle_diameter(len(parent), _ptr(parent), _ptr(weight),
                               _ptr(out)))
    return int(out[0])


def expdp(parent, weight, c, lam, F):
    """Two-pass tree recursion for ``f(d) = sum_j c_j lam_j^d``."""
    lib = _load()
    parent, weight = _tree(parent, weight)
    n = len(parent)
    F = np.asarray(F, dtype=np.float64)
    vec = F.ndim == 1
    F2 = np.ascontiguousarray(F.reshape(n, -1))
    c = np.ascontiguousarray(np.atleast_1d(c), dtype=np.float64)
    lam = np.ascontiguousarray(np.atleast_1d(lam), dtype=np.float64)
    out = np.zeros_like(F2)
    _check(lib.oracle_expdp(n, _ptr(parent), _ptr(weight), _ptr(c), _ptr(lam),
                            len(c), _ptr(F2), F2.shape[1], _ptr(out)))
    return out[:, 0] if vec else out
