"""CPU oracle for the causal-set interval-abundance path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1805_04463_amd``) and never imports it.

The arithmetic lives in ``causal_oracle.c`` (plain C, OpenMP, fp64 predicates
without contraction, quad-precision action); ``brute.py`` is an independent
pure-Python enumeration for tiny sets.  Both follow Cunningham (2018):
App. A for the sprinklings, Ch. 4 for the causal relation, the naive and
optimised interval-abundance algorithms, and the BD actions of Sec. 4.2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "causal_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
# ORACLE_SANITIZE=1 selects a build instrumented with AddressSanitizer and
# UndefinedBehaviorSanitizer (any finding aborts).  The interpreter is not instrumented,
# so such a process must start with the ASan runtime preloaded (LD_PRELOAD).
_SANITIZE = os.environ.get("ORACLE_SANITIZE", "") == "1"
_LIB_PATH = os.path.join(_BUILD, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-g"]

MINK2_DIAMOND, MINK4_DIAMOND, DS4_SLAB, DS2_SLAB, MINK3_DIAMOND = 0, 1, 2, 3, 4
PLANES = {MINK2_DIAMOND: 2, MINK4_DIAMOND: 4, DS4_SLAB: 7, DS2_SLAB: 3, MINK3_DIAMOND: 3}
DIM = {MINK2_DIAMOND: 2, MINK4_DIAMOND: 4, DS4_SLAB: 4, DS2_SLAB: 2, MINK3_DIAMOND: 3}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (no HIP involved)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", *(_SAN_FLAGS if _SANITIZE else []),
               "-o", tmp, _SRC, "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u64, i64, dbl, c_int = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        p = ctypes.c_void_p
        L.or_splitmix64_next.argtypes = [ctypes.POINTER(u64)]
        L.or_splitmix64_next.restype = u64
        L.or_draw.argtypes = [u64, u64, u64]
        L.or_draw.restype = u64
        L.or_sprinkle.argtypes = [c_int, dbl, u64, i64, p]
        L.or_sprinkle.restype = c_int
        L.or_ld_words.argtypes = [i64]
        L.or_ld_words.restype = i64
        L.or_causal_matrix.argtypes = [c_int, p, i64, p, i64]
        L.or_causal_matrix.restype = c_int
        L.or_causal_rows.argtypes = [c_int, p, i64, p, i64, p, i64]
        L.or_causal_rows.restype = c_int
        L.or_histogram_naive.argtypes = [p, i64, i64, p]
        L.or_histogram_naive.restype = c_int
        L.or_histogram_naive_elems.argtypes = [p, i64, i64, p, p, i64]
        L.or_histogram_naive_elems.restype = c_int
        L.or_histogram_fast.argtypes = [p, i64, i64, p, i64, i64]
        L.or_histogram_fast.restype = i64
        L.or_histogram_fast_rows.argtypes = [p, i64, i64, p, p, i64]
        L.or_histogram_fast_rows.restype = i64
        L.or_pair_interval.argtypes = [p, i64, i64, i64]
        L.or_c3_double.restype = dbl
        L.or_c3_double.argtypes = []
        L.or_dalembertian.restype = c_int
        L.or_dalembertian.argtypes = [p, i64, i64, c_int, dbl, p, p, p, p]
        L.or_dalembertian_cols.restype = c_int
        L.or_dalembertian_cols.argtypes = [p, i64, i64, c_int, dbl, p, p, i64, p, p, p]
        L.or_pair_interval.restype = i64
        L.or_degrees.argtypes = [p, i64, i64, p, p, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.or_degrees.restype = c_int
        L.or_longest_chain.argtypes = [p, i64, i64, p, p, i64, p, p]
        L.or_longest_chain.restype = c_int
        L.or_action.argtypes = [p, i64, c_int, dbl, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
        L.or_action.restype = c_int
        L.or_smear_weight.argtypes = [c_int, i64, dbl]
        L.or_smear_weight.restype = dbl
        L.or_max_threads.restype = c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def splitmix64_sequence(state: int, count: int) -> list[int]:
    """The published sequential SplitMix64 outputs from ``state``."""
    s = ctypes.c_uint64(state)
    return [lib().or_splitmix64_next(ctypes.byref(s)) for _ in range(count)]


def draw(seed: int, stream: int, c: int) -> int:
    return lib().or_draw(seed, stream, c)


def sprinkle(region: int, n: int, seed: int, eta0: float = 1.2) -> np.ndarray:
    """Time-ordered sprinkling; returns SoA planes of shape (planes, n), float64."""
    out = np.zeros((PLANES[region], n), dtype=np.float64)
    rc = lib().or_sprinkle(region, eta0, seed, n, _ptr(out))
    if rc != 0:
        raise ValueError("or_sprinkle failed")
    return out


def ld_words(n: int) -> int:
    return lib().or_ld_words(n)


def causal_matrix(region: int, coords: np.ndarray, ld: int | None = None) -> np.ndarray:
    """Symmetric packed causal matrix, uint64 array (n, ld)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n = coords.shape[1]
    ld = ld_words(n) if ld is None else ld
    bits = np.zeros((n, ld), dtype=np.uint64)
    if lib().or_causal_matrix(region, _ptr(coords), n, _ptr(bits), ld) != 0:
        raise ValueError("or_causal_matrix failed")
    return bits


def causal_rows(region: int, coords: np.ndarray, rows, ld: int | None = None) -> np.ndarray:
    """Rows `rows` of the symmetric packed causal matrix, uint64 array (len(rows), ld)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    n = coords.shape[1]
    ld = ld_words(n) if ld is None else ld
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((len(rows), ld), dtype=np.uint64)
    if lib().or_causal_rows(region, _ptr(coords), n, _ptr(rows), len(rows), _ptr(out), ld) != 0:
        raise ValueError("or_causal_rows failed")
    return out


def histogram_naive(bits: np.ndarray, n: int) -> np.ndarray:
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    hist = np.zeros(max(n - 1, 1), dtype=np.uint64)
    if lib().or_histogram_naive(_ptr(bits), n, bits.shape[1], _ptr(hist)) != 0:
        raise ValueError("or_histogram_naive failed")
    return hist


def histogram_naive_elems(bits: np.ndarray, n: int, elems) -> np.ndarray:
    """The definitional tier over the listed elements j only (all pairs i ≺ j)."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    hist = np.zeros(max(n - 1, 1), dtype=np.uint64)
    if lib().or_histogram_naive_elems(_ptr(bits), n, bits.shape[1], _ptr(hist), _ptr(elems),
                                      len(elems)) != 0:
        raise ValueError("or_histogram_naive_elems failed")
    return hist


def histogram_fast(bits: np.ndarray, n: int, row_begin: int = 0, row_end: int | None = None):
    """Returns (hist, pairs_counted) over rows [row_begin, row_end)."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    row_end = n if row_end is None else row_end
    hist = np.zeros(max(n - 1, 1), dtype=np.uint64)
    pairs = lib().or_histogram_fast(_ptr(bits), n, bits.shape[1], _ptr(hist), row_begin, row_end)
    if pairs < 0:
        raise ValueError("or_histogram_fast failed")
    return hist, pairs


def histogram_fast_rows(bits: np.ndarray, n: int, rows):
    """Fast tier over the listed rows only; returns (hist, pairs_counted)."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    hist = np.zeros(max(n - 1, 1), dtype=np.uint64)
    pairs = lib().or_histogram_fast_rows(_ptr(bits), n, bits.shape[1], _ptr(hist), _ptr(rows),
                                         len(rows))
    if pairs < 0:
        raise ValueError("or_histogram_fast_rows failed")
    return hist, pairs


def pair_interval(bits: np.ndarray, i: int, j: int) -> int:
    return lib().or_pair_interval(_ptr(bits), bits.shape[1], i, j)


def degrees(bits: np.ndarray, n: int):
    """(indeg, outdeg, number of 3-chains, number of relations)."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    ind = np.zeros(n, dtype=np.int64)
    outd = np.zeros(n, dtype=np.int64)
    c3, rel = ctypes.c_uint64(0), ctypes.c_uint64(0)
    lib().or_degrees(_ptr(bits), n, bits.shape[1], _ptr(ind), _ptr(outd),
                     ctypes.byref(c3), ctypes.byref(rel))
    return ind, outd, c3.value, rel.value


def longest_chain(bits: np.ndarray, n: int, lo, hi, heights: bool = False):
    """Alg. "Maximal Chain Length" for pairs (lo[s], hi[s]), -1 <= lo < hi <= n, where -1
    and n are virtual elements below and above every element.  Returns (length, height):
    length[s] = links on the longest chain from lo[s] to hi[s] (0 when unrelated);
    height[s, k] = links on the longest chain from lo[s] to k for k in the Alexandroff
    set or k = hi[s], else 0 (None unless heights)."""
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    lo = np.ascontiguousarray(np.atleast_1d(lo), dtype=np.int64)
    hi = np.ascontiguousarray(np.atleast_1d(hi), dtype=np.int64)
    assert lo.shape == hi.shape
    length = np.zeros(len(lo), dtype=np.int64)
    h = np.zeros((len(lo), n), dtype=np.int64) if heights else None
    rc = lib().or_longest_chain(_ptr(bits), n, bits.shape[1], _ptr(lo), _ptr(hi), len(lo),
                                _ptr(length), _ptr(h) if heights else None)
    if rc != 0:
        raise ValueError("bad longest-chain arguments")
    return length, h


def action(hist: np.ndarray, n: int, dim: int, eps: float = 0.0):
    """(S, kappa) from the abundances; eps == 0 gives the local action."""
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    out, kap = ctypes.c_double(0.0), ctypes.c_double(0.0)
    if lib().or_action(_ptr(hist), n, dim, eps, ctypes.byref(out), ctypes.byref(kap)) != 0:
        raise ValueError("or_action failed")
    return out.value, kap.value


def dalembertian(bits: np.ndarray, n: int, dim: int, ell: float, phi: np.ndarray):
    """B^(d+1) phi for every element (Sec. 4.1), with the summand count and the sum of
    absolute summands of each element: (out, terms, abs_sum)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    assert phi.shape == (n,)
    out = np.empty(n, dtype=np.float64)
    terms = np.empty(n, dtype=np.int64)
    mag = np.empty(n, dtype=np.float64)
    if lib().or_dalembertian(_ptr(bits), n, bits.shape[1], dim, ell, _ptr(phi), _ptr(out),
                             _ptr(terms), _ptr(mag)) != 0:
        raise ValueError("or_dalembertian failed")
    return out, terms, mag


def dalembertian_cols(bits: np.ndarray, n: int, dim: int, ell: float, phi: np.ndarray, js):
    """dalembertian() for the elements js only: (out, terms, abs_sum) in the order of js."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    js = np.ascontiguousarray(js, dtype=np.int64)
    assert phi.shape == (n,)
    out = np.empty(len(js), dtype=np.float64)
    terms = np.empty(len(js), dtype=np.int64)
    mag = np.empty(len(js), dtype=np.float64)
    if lib().or_dalembertian_cols(_ptr(bits), n, bits.shape[1], dim, ell, _ptr(phi), _ptr(js),
                                  len(js), _ptr(out), _ptr(terms), _ptr(mag)) != 0:
        raise ValueError("or_dalembertian_cols failed")
    return out, terms, mag


def smear_weight(dim: int, m: int, eps: float) -> float:
    return lib().or_smear_weight(dim, m, eps)


def max_threads() -> int:
    return lib().or_max_threads()


def pipeline(region: int, n: int, seed: int, eps_list=(), eta0: float = 1.2, fast: bool = False):
    """Sprinkle -> matrix -> histogram -> actions, all on the CPU."""
    coords = sprinkle(region, n, seed, eta0)
    bits = causal_matrix(region, coords)
    hist = histogram_fast(bits, n)[0] if fast else histogram_naive(bits, n)
    dim = DIM[region]
    acts = {0.0: action(hist, n, dim, 0.0)[0]}
    for e in eps_list:
        acts[e] = action(hist, n, dim, e)[0]
    return coords, bits, hist, acts
