"""Bulk oracle operations in plain C (TEST INFRASTRUCTURE ONLY).

`oracle/c/fieldops.c` evaluates multilinear extensions of large vectors (the
input layer of a full-size proof) where pure Python would take minutes. It
shares nothing with the HIP library; `tests/test_oracle_fast.py` pins it to the
Python oracle on random and edge values.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "fieldops.c")
LIB = os.path.join(HERE, "c", "liboraclefield.so")
_lib = None


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", LIB + ".tmp", SRC]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle C helper failed to build:\n" + res.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        vp = ctypes.c_void_p
        L.oracle_mulmod_many.argtypes = [vp, vp, vp, ctypes.c_uint64]
        L.oracle_addsub_many.argtypes = [vp, vp, vp, vp, ctypes.c_uint64]
        L.oracle_mle.argtypes = [vp, ctypes.c_uint32, vp, vp, vp]
        L.oracle_poly_eval.argtypes = [vp, ctypes.c_uint64, vp, vp]
        _lib = L
    return _lib


def _words(limbs: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(limbs, dtype=np.uint32)
    return a.view(np.uint64).reshape(-1, 4)


def _ints_to_words(vals) -> np.ndarray:
    out = np.zeros((len(vals), 4), dtype=np.uint64)
    for i, v in enumerate(vals):
        for k in range(4):
            out[i, k] = (v >> (64 * k)) & (2**64 - 1)
    return out


def _words_to_ints(w: np.ndarray):
    return [int(r[0]) | (int(r[1]) << 64) | (int(r[2]) << 128) | (int(r[3]) << 192) for r in w]


def mulmod_many(a, b):
    A, B = _ints_to_words(a), _ints_to_words(b)
    out = np.zeros_like(A)
    lib().oracle_mulmod_many(A.ctypes.data, B.ctypes.data, out.ctypes.data, len(a))
    return _words_to_ints(out)


def addsub_many(a, b):
    A, B = _ints_to_words(a), _ints_to_words(b)
    s, d = np.zeros_like(A), np.zeros_like(A)
    lib().oracle_addsub_many(A.ctypes.data, B.ctypes.data, s.ctypes.data, d.ctypes.data, len(a))
    return _words_to_ints(s), _words_to_ints(d)


def mle_limbs(limbs: np.ndarray, r) -> int:
    """V~(r) for V given as canonical (2^k, 8) uint32 limbs and r as Python ints."""
    V = _words(limbs)
    k = len(r)
    if V.shape[0] != 1 << k:
        raise ValueError("table size does not match the point")
    R = _ints_to_words(list(r))
    scratch = np.zeros((max(1, V.shape[0] // 2), 4), dtype=np.uint64)
    out = np.zeros((1, 4), dtype=np.uint64)
    lib().oracle_mle(V.ctypes.data, k, R.ctypes.data, scratch.ctypes.data, out.ctypes.data)
    return _words_to_ints(out)[0]


def poly_eval_limbs(limbs: np.ndarray, x: int) -> int:
    """f(x) = sum_b V[b] x^b for V given as canonical (count, 8) uint32 limbs."""
    V = _words(limbs)
    X = _ints_to_words([x])
    out = np.zeros((1, 4), dtype=np.uint64)
    lib().oracle_poly_eval(V.ctypes.data, V.shape[0], X.ctypes.data, out.ctypes.data)
    return _words_to_ints(out)[0]
