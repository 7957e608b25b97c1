"""Counter-based random draws for the synthetic relations.

Two implementations of the same definitions live here:

* ``NativeRNG`` calls the C generator in ``rng.c`` (OpenMP; used for every
  relation the tests and benchmarks build, at any size);
* the ``ref_*`` functions are plain numpy restatements of the same formulas,
  used only by tests to pin the C code on small draws.

Definitions (SplitMix64 in counter mode, Steele et al., OOPSLA 2014):
draw ``i`` of stream ``K`` is ``mix64(K + (i+1)*GAMMA)``; a unit double keeps
its top 53 bits; a normal draw is Box-Muller on unit draws ``2i`` and ``2i+1``;
a bounded integer is ``lo + floor(u*(hi-lo))``; a table draw returns the
smallest ``k`` with ``u < cdf[k]``.

Nothing here evaluates aggregates: this module only produces inputs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rng.c")
_LIB = os.path.join(_HERE, "_rng.so")

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def build(force: bool = False) -> str:
    """Compile the native generator with gcc (host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class NativeRNG:
    """ctypes view of ``rng.c``."""

    def __init__(self):
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64, u64, i32, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        lib.dg_stream_key.restype = u64
        lib.dg_stream_key.argtypes = [u64, ctypes.c_char_p]
        lib.dg_fill_u64.argtypes = [u64, i64, P]
        lib.dg_fill_unit_f64.argtypes = [u64, i64, P]
        lib.dg_fill_uniform_f32.argtypes = [u64, i64, f64, f64, P]
        lib.dg_fill_normal_f32.argtypes = [u64, i64, f64, f64, P]
        lib.dg_fill_normal_f64.argtypes = [u64, i64, f64, f64, P]
        lib.dg_fill_uniform_i32.argtypes = [u64, i64, i32, i32, P]
        lib.dg_fill_from_cdf_i32.argtypes = [u64, i64, P, i32, P]
        lib.dg_sort_u64.restype = ctypes.c_int
        lib.dg_sort_u64.argtypes = [P, i64]
        lib.dg_compose.argtypes = [i64, ctypes.c_int, P, P, P]
        lib.dg_decompose.argtypes = [i64, ctypes.c_int, P, P, P]
        self.lib = lib

    @staticmethod
    def _p(a: np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data_as(ctypes.c_void_p)

    def key(self, seed: int, name: str) -> int:
        return int(self.lib.dg_stream_key(seed, name.encode()))

    def u64(self, key: int, n: int) -> np.ndarray:
        out = np.empty(n, np.uint64)
        self.lib.dg_fill_u64(key, n, self._p(out))
        return out

    def unit(self, key: int, n: int) -> np.ndarray:
        out = np.empty(n, np.float64)
        self.lib.dg_fill_unit_f64(key, n, self._p(out))
        return out

    def uniform_f32(self, key: int, n: int, lo: float, hi: float) -> np.ndarray:
        out = np.empty(n, np.float32)
        self.lib.dg_fill_uniform_f32(key, n, lo, hi, self._p(out))
        return out

    def normal_f32(self, key: int, n: int, mean: float, sd: float) -> np.ndarray:
        out = np.empty(n, np.float32)
        self.lib.dg_fill_normal_f32(key, n, mean, sd, self._p(out))
        return out

    def normal_f64(self, key: int, n: int, mean: float, sd: float) -> np.ndarray:
        out = np.empty(n, np.float64)
        self.lib.dg_fill_normal_f64(key, n, mean, sd, self._p(out))
        return out

    def uniform_i32(self, key: int, n: int, lo: int, hi: int) -> np.ndarray:
        out = np.empty(n, np.int32)
        self.lib.dg_fill_uniform_i32(key, n, lo, hi, self._p(out))
        return out

    def from_cdf_i32(self, key: int, n: int, cdf: np.ndarray) -> np.ndarray:
        cdf = np.ascontiguousarray(cdf, np.float64)
        out = np.empty(n, np.int32)
        self.lib.dg_fill_from_cdf_i32(key, n, self._p(cdf), len(cdf), self._p(out))
        return out

    def sort_u64(self, a: np.ndarray) -> np.ndarray:
        a = np.ascontiguousarray(a, np.uint64)
        if self.lib.dg_sort_u64(self._p(a), len(a)) != 0:
            raise MemoryError("radix sort scratch allocation failed")
        return a

    def compose(self, cols, radix) -> np.ndarray:
        n = len(cols[0])
        cols = [np.ascontiguousarray(c, np.int32) for c in cols]
        ptrs = (ctypes.c_void_p * len(cols))(*[c.ctypes.data for c in cols])
        rad = np.asarray(radix, np.int64)
        out = np.empty(n, np.uint64)
        self.lib.dg_compose(n, len(cols), ptrs, self._p(rad), self._p(out))
        return out

    def decompose(self, comp: np.ndarray, radix):
        n = len(comp)
        cols = [np.empty(n, np.int32) for _ in radix]
        ptrs = (ctypes.c_void_p * len(cols))(*[c.ctypes.data for c in cols])
        rad = np.asarray(radix, np.int64)
        self.lib.dg_decompose(n, len(cols), self._p(np.ascontiguousarray(comp)), self._p(rad), ptrs)
        return cols


_native = None


def native() -> NativeRNG:
    global _native
    if _native is None:
        _native = NativeRNG()
    return _native


# ---------------------------------------------------------------------------
# numpy restatements (small n only), used to pin the C generator
# ---------------------------------------------------------------------------

def ref_mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def ref_key(seed: int, name: str) -> int:
    h = 0xCBF29CE484222325
    for b in name.encode():
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    s = (seed * 0x9E3779B97F4A7C15 + 1) & 0xFFFFFFFFFFFFFFFF
    a = int(ref_mix64(np.array([s], np.uint64))[0])
    return int(ref_mix64(np.array([a ^ h], np.uint64))[0])


def ref_u64(key: int, n: int, start: int = 0) -> np.ndarray:
    i = np.arange(start, start + n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return ref_mix64(np.uint64(key) + (i + np.uint64(1)) * GAMMA)


def ref_unit(key: int, n: int, start: int = 0) -> np.ndarray:
    return (ref_u64(key, n, start) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def ref_normal_f32(key: int, n: int, mean: float, sd: float) -> np.ndarray:
    u = ref_unit(key, 2 * n)
    z = np.sqrt(-2.0 * np.log(1.0 - u[0::2])) * np.cos(2.0 * np.pi * u[1::2])
    return (mean + sd * z).astype(np.float32)


def ref_uniform_i32(key: int, n: int, lo: int, hi: int) -> np.ndarray:
    v = np.floor(ref_unit(key, n) * (float(hi) - float(lo))).astype(np.int64)
    return (lo + np.minimum(v, hi - lo - 1)).astype(np.int32)


def ref_from_cdf_i32(key: int, n: int, cdf: np.ndarray) -> np.ndarray:
    u = ref_unit(key, n)
    k = np.searchsorted(np.asarray(cdf, np.float64), u, side="right")
    return np.minimum(k, len(cdf) - 1).astype(np.int32)
