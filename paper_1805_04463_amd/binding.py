"""Thin ctypes binding of libcausal.so (declared in include/causal.h).

Argument marshalling only: every step runs in the library's HIP kernels.  Functions
carry the C entry points' names.  Device buffers are torch tensors on the current
ROCm device; work is enqueued on ``torch.cuda.current_stream()`` unless a stream is
given.  The library must have been built (``paper_1805_04463_amd.build.build()``);
there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libcausal.so")

CS_MINK2_DIAMOND, CS_MINK4_DIAMOND, CS_DS4_SLAB, CS_DS2_SLAB, CS_MINK3_DIAMOND = 0, 1, 2, 3, 4
CS_COUNT_BITSET, CS_COUNT_MFMA, CS_COUNT_MFMA_FP4, CS_COUNT_BITSET_DENSE = 0, 1, 2, 3
REGION_DIM = {CS_MINK2_DIAMOND: 2, CS_MINK4_DIAMOND: 4, CS_DS4_SLAB: 4, CS_DS2_SLAB: 2,
              CS_MINK3_DIAMOND: 3}

SYMBOLS = [
    "cs_coord_planes", "cs_ld_words", "cs_status_string", "cs_sprinkle_workspace_bytes",
    "cs_sprinkle", "cs_causal_matrix", "cs_histogram_workspace_bytes", "cs_interval_histogram",
    "cs_action", "cs_batch_plan", "cs_batch_workspace_bytes", "cs_batch_hist_len",
    "cs_batch_hist_offset", "cs_batch_coords_offset", "cs_batch_bits_offset", "cs_batch_run",
    "cs_batch_free", "cs_batch_graph_create", "cs_batch_graph_launch", "cs_batch_graph_destroy", "cs_autotune", "cs_measure_mfma_peak",
    "cs_dalembertian_workspace_bytes", "cs_dalembertian", "cs_longest_chain_workspace_bytes",
    "cs_longest_chain", "cs_degrees", "cs_interval_histogram_noalloc",
]


class CausalError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CausalError(f"{LIB_PATH} is missing: run paper_1805_04463_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        i64, u64, dbl, c_int, p, sz = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t)
        sig = {
            "cs_coord_planes": (c_int, [c_int]),
            "cs_ld_words": (i64, [i64]),
            "cs_status_string": (ctypes.c_char_p, [c_int]),
            "cs_sprinkle_workspace_bytes": (sz, [c_int, i64]),
            "cs_sprinkle": (c_int, [c_int, dbl, u64, i64, p, p, sz, p]),
            "cs_causal_matrix": (c_int, [c_int, p, i64, p, i64, p]),
            "cs_histogram_workspace_bytes": (sz, [i64, c_int]),
            "cs_interval_histogram": (c_int, [p, i64, i64, c_int, p, p, sz, p]),
            "cs_interval_histogram_noalloc": (c_int, [p, i64, i64, c_int, p, p]),
            "cs_action": (c_int, [p, i64, c_int, dbl, p, p]),
            "cs_dalembertian_workspace_bytes": (sz, [i64, c_int]),
            "cs_dalembertian": (c_int, [p, i64, i64, c_int, dbl, c_int, p, p, p, sz, p]),
            "cs_longest_chain_workspace_bytes": (sz, [i64, i64]),
            "cs_longest_chain": (c_int, [p, i64, i64, p, p, i64, p, p, p, sz, p]),
            "cs_degrees": (c_int, [p, i64, i64, p, p, p]),
            "cs_batch_plan": (c_int, [i64, p, c_int, c_int, p, ctypes.c_char_p, ctypes.POINTER(p)]),
            "cs_batch_workspace_bytes": (sz, [p]),
            "cs_batch_hist_len": (i64, [p]),
            "cs_batch_hist_offset": (i64, [p, i64]),
            "cs_batch_coords_offset": (i64, [p, i64]),
            "cs_batch_bits_offset": (i64, [p, i64]),
            "cs_batch_run": (c_int, [p, p, p, p, p, sz, p]),
            "cs_batch_free": (c_int, [p]),
            "cs_batch_graph_create": (c_int, [p, p, p, p, p, sz, ctypes.POINTER(p)]),
            "cs_batch_graph_launch": (c_int, [p, p]),
            "cs_batch_graph_destroy": (c_int, [p]),
            "cs_autotune": (c_int, [ctypes.c_char_p, i64, c_int, p]),
            "cs_measure_mfma_peak": (c_int, [c_int, ctypes.POINTER(dbl), p]),
        }
        for name, (res, args) in sig.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().cs_status_string(rc).decode()
        raise CausalError(f"{what}: {msg} (status {rc})")


def _dev():
    if not torch.cuda.is_available():
        raise CausalError("no ROCm GPU visible to torch")
    return torch.device("cuda", torch.cuda.current_device())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise CausalError("expected a device tensor")
    if not t.is_contiguous():
        raise CausalError("expected a contiguous tensor")
    if t.device.index != torch.cuda.current_device():
        raise CausalError(f"tensor on {t.device}, but the current device is "
                          f"cuda:{torch.cuda.current_device()}")
    return ctypes.c_void_p(t.data_ptr())


def _need(t, name: str, dtypes, numel: int | None = None, min_numel: int | None = None,
          shape: tuple | None = None):
    """Validate a caller's tensor before its pointer crosses the ABI: the library trusts
    the sizes it is given, so a short buffer here would become an out-of-bounds access on
    the device."""
    if not isinstance(t, torch.Tensor):
        raise CausalError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype not in dtypes:
        raise CausalError(f"{name}: dtype {t.dtype}, expected one of {list(dtypes)}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise CausalError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if numel is not None and t.numel() != numel:
        raise CausalError(f"{name}: {t.numel()} elements, expected {numel}")
    if min_numel is not None and t.numel() < min_numel:
        raise CausalError(f"{name}: {t.numel()} elements, expected at least {min_numel}")
    if not t.is_contiguous():
        raise CausalError(f"{name}: expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _on_device(*tensors):
    """Every tensor lives on the current ROCm device (checked after the shapes)."""
    for t in tensors:
        _ptr(t)


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def _int(x, name: str) -> int:
    if isinstance(x, bool) or not isinstance(x, (int,)) and not hasattr(x, "__index__"):
        raise CausalError(f"{name}: expected an integer, got {type(x).__name__}")
    return int(x)


def _bits(bits, n: int):
    """The packed matrix: int64 (n', ld) with n' >= n rows and ld >= cs_ld_words(n)."""
    if not isinstance(bits, torch.Tensor) or bits.dim() != 2:
        raise CausalError("bits: expected a 2-D (rows, ld_words) tensor")
    if n < 2:
        raise CausalError(f"n = {n}: need at least 2 elements")
    if bits.shape[0] < n:
        raise CausalError(f"bits: {bits.shape[0]} rows for n = {n}")
    ld = bits.shape[1]
    if ld < lib().cs_ld_words(n):
        raise CausalError(f"bits: {ld} words per row, n = {n} needs {lib().cs_ld_words(n)}")
    return _need(bits, "bits", _WORDS), ld


_WORDS = (torch.int64, torch.uint64) if hasattr(torch, "uint64") else (torch.int64,)
_F64 = (torch.float64,)
_BYTES = (torch.uint8, torch.int8) + _WORDS


def _u8_workspace(nbytes: int) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=_dev())


def cs_coord_planes(region: int) -> int:
    return lib().cs_coord_planes(region)


def cs_ld_words(n: int) -> int:
    return lib().cs_ld_words(n)


def cs_sprinkle(region: int, n: int, seed: int, eta0: float = 1.2, stream=None) -> torch.Tensor:
    """Time-ordered coordinates, float64 device tensor (planes, n)."""
    n = _int(n, "n")
    planes = lib().cs_coord_planes(region)
    if planes < 0:
        raise CausalError(f"unknown region {region}")
    if n < 2:
        raise CausalError(f"n = {n}: need at least 2 points")
    coords = torch.empty((planes, n), dtype=torch.float64, device=_dev())
    ws_bytes = lib().cs_sprinkle_workspace_bytes(region, n)
    ws = _u8_workspace(ws_bytes)
    _check(lib().cs_sprinkle(region, eta0, seed & (2**64 - 1), n, _ptr(coords), _ptr(ws), ws_bytes,
                             _stream(stream)), "cs_sprinkle")
    coords._cs_keepalive = ws  # workspace must outlive the enqueued kernels
    return coords


def cs_causal_matrix(region: int, coords: torch.Tensor, n: int | None = None,
                     ld_words: int | None = None, out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    """Symmetric packed matrix as an int64 device tensor (n, ld) holding uint64 words."""
    planes = lib().cs_coord_planes(region)
    if planes < 0:
        raise CausalError(f"unknown region {region}")
    if not isinstance(coords, torch.Tensor) or coords.dim() != 2:
        raise CausalError("coords: expected a 2-D (planes, n) tensor")
    n = coords.shape[1] if n is None else _int(n, "n")
    pc = _need(coords, "coords", _F64, shape=(planes, n))
    if n < 2:
        raise CausalError(f"n = {n}: need at least 2 points")
    ld = lib().cs_ld_words(n) if ld_words is None else _int(ld_words, "ld_words")
    if ld < lib().cs_ld_words(n):
        raise CausalError(f"ld_words = {ld}: n = {n} needs {lib().cs_ld_words(n)}")
    bits = out if out is not None else torch.empty((n, ld), dtype=torch.int64, device=_dev())
    pb = _need(bits, "out", _WORDS, shape=(n, ld))
    _on_device(coords, bits)
    _check(lib().cs_causal_matrix(region, pc, n, pb, ld, _stream(stream)), "cs_causal_matrix")
    return bits


def cs_interval_histogram(bits: torch.Tensor, n: int, counter: int = CS_COUNT_MFMA,
                          out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                          stream=None) -> torch.Tensor:
    """N_m for m = 0..n-2 as an int64 device tensor (uint64 counts)."""
    n = _int(n, "n")
    pbits, ld = _bits(bits, n)
    hist = out if out is not None else torch.empty(n - 1, dtype=torch.int64, device=_dev())
    ph = _need(hist, "out", _WORDS, numel=n - 1)
    ws_bytes = lib().cs_histogram_workspace_bytes(n, counter)
    ws = workspace if workspace is not None else _u8_workspace(ws_bytes)
    pw = _need(ws, "workspace", _BYTES)
    _on_device(bits, hist, ws)
    _check(lib().cs_interval_histogram(pbits, n, ld, counter, ph, pw, _nbytes(ws),
                                       _stream(stream)), "cs_interval_histogram")
    hist._cs_keepalive = ws
    return hist


def cs_interval_histogram_noalloc(bits: torch.Tensor, n: int, out: torch.Tensor,
                                  counter: int = CS_COUNT_MFMA, stream=None) -> torch.Tensor:
    """cs_interval_histogram into the caller's `out` (n-1 int64), with the library's static
    scratch instead of a workspace: no device memory is allocated."""
    n = _int(n, "n")
    pbits, ld = _bits(bits, n)
    ph = _need(out, "out", _WORDS, numel=n - 1)
    _on_device(bits, out)
    _check(lib().cs_interval_histogram_noalloc(pbits, n, ld, counter, ph, _stream(stream)),
           "cs_interval_histogram_noalloc")
    return out


def cs_dalembertian(bits: torch.Tensor, n: int, dim: int, ell: float, phi: torch.Tensor,
                    counter: int = CS_COUNT_MFMA_FP4, out: torch.Tensor | None = None,
                    workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """B^(d+1) phi for every element as a float64 device tensor (phi: n float64 on device)."""
    n = _int(n, "n")
    pbits, ld = _bits(bits, n)
    pphi = _need(phi, "phi", _F64, numel=n)
    o = out if out is not None else torch.empty(n, dtype=torch.float64, device=_dev())
    po = _need(o, "out", _F64, numel=n)
    ws_bytes = lib().cs_dalembertian_workspace_bytes(n, counter)
    ws = workspace if workspace is not None else _u8_workspace(max(ws_bytes, 1))
    pw = _need(ws, "workspace", _BYTES)
    _on_device(bits, phi, o, ws)
    _check(lib().cs_dalembertian(pbits, n, ld, dim, float(ell), counter, pphi, po, pw,
                                 _nbytes(ws), _stream(stream)), "cs_dalembertian")
    o._cs_keepalive = ws
    return o


def cs_longest_chain(bits: torch.Tensor, n: int, lo, hi, heights: bool = False,
                     workspace: torch.Tensor | None = None, stream=None):
    """Longest chains (links) from lo[s] to hi[s] for every pair, -1 and n being the
    virtual elements below and above everything.  Returns (length, height): int32 device
    tensors of count and (count, n) elements (height None unless requested).  Blocks until
    done."""
    import numpy as np
    n = _int(n, "n")
    pbits, ld = _bits(bits, n)
    lo_h = np.ascontiguousarray(np.atleast_1d(lo), dtype=np.int64)
    hi_h = np.ascontiguousarray(np.atleast_1d(hi), dtype=np.int64)
    if lo_h.shape != hi_h.shape or lo_h.ndim != 1:
        raise CausalError("lo and hi must be 1-D and of the same length")
    count = len(lo_h)
    length = torch.empty(count, dtype=torch.int32, device=_dev())
    height = torch.empty((count, n), dtype=torch.int32, device=_dev()) if heights else None
    ws_bytes = lib().cs_longest_chain_workspace_bytes(n, count)
    ws = workspace if workspace is not None else _u8_workspace(max(ws_bytes, 1))
    pw = _need(ws, "workspace", _BYTES)
    _on_device(bits, ws)
    _check(lib().cs_longest_chain(pbits, n, ld, lo_h.ctypes.data_as(ctypes.c_void_p),
                                  hi_h.ctypes.data_as(ctypes.c_void_p), count, _ptr(length),
                                  _ptr(height) if heights else None, pw, _nbytes(ws),
                                  _stream(stream)), "cs_longest_chain")
    return length, height


def cs_degrees(bits: torch.Tensor, n: int, stream=None):
    """(indeg, outdeg) of every element as int64 device tensors."""
    n = _int(n, "n")
    pbits, ld = _bits(bits, n)
    ind = torch.empty(n, dtype=torch.int64, device=_dev())
    outd = torch.empty(n, dtype=torch.int64, device=_dev())
    _on_device(bits)
    _check(lib().cs_degrees(pbits, n, ld, _ptr(ind), _ptr(outd), _stream(stream)), "cs_degrees")
    return ind, outd


def cs_action(hist: torch.Tensor, n: int, dim: int, eps: float = 0.0,
              out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The action as a one-element float64 device tensor."""
    n = _int(n, "n")
    if n < 2:
        raise CausalError(f"n = {n}: need at least 2 elements")
    ph = _need(hist, "hist", _WORDS, min_numel=n - 1)
    o = out if out is not None else torch.empty(1, dtype=torch.float64, device=_dev())
    po = _need(o, "out", _F64, min_numel=1)
    _on_device(hist, o)
    _check(lib().cs_action(ph, n, dim, float(eps), po, _stream(stream)), "cs_action")
    return o


class BatchPlan:
    """Host-side plan of an ensemble of 1+1 diamonds (wraps cs_batch_plan)."""

    def __init__(self, sizes, counter: int = CS_COUNT_MFMA, eps=(0.0,), tune_cache=None):
        import numpy as np
        self.sizes = np.ascontiguousarray(sizes, dtype=np.int64)
        self.eps = np.ascontiguousarray(eps, dtype=np.float64)
        self.count = len(self.sizes)
        h = ctypes.c_void_p()
        tc = tune_cache.encode() if tune_cache else None
        _check(lib().cs_batch_plan(self.count, self.sizes.ctypes.data_as(ctypes.c_void_p), counter,
                                   len(self.eps), self.eps.ctypes.data_as(ctypes.c_void_p), tc,
                                   ctypes.byref(h)), "cs_batch_plan")
        self.handle = h
        self.ws_bytes = lib().cs_batch_workspace_bytes(h)
        self.hist_len = lib().cs_batch_hist_len(h)
        self.offsets = [lib().cs_batch_hist_offset(h, k) for k in range(self.count)]
        # byte offsets of each instance's coordinates and matrix in the workspace
        self.coords_offsets = [lib().cs_batch_coords_offset(h, k) for k in range(self.count)]
        self.bits_offsets = [lib().cs_batch_bits_offset(h, k) for k in range(self.count)]

    def _buffers(self, seeds, hist, actions, workspace):
        ptrs = (_need(seeds, "seeds", _WORDS, numel=self.count),
                _need(hist, "hist", _WORDS, min_numel=self.hist_len),
                _need(actions, "actions", _F64, min_numel=self.count * len(self.eps)),
                _need(workspace, "workspace", _BYTES))
        _on_device(seeds, hist, actions, workspace)
        return ptrs

    def run(self, seeds: torch.Tensor, hist: torch.Tensor, actions: torch.Tensor,
            workspace: torch.Tensor, stream=None):
        ps, ph, pa, pw = self._buffers(seeds, hist, actions, workspace)
        _check(lib().cs_batch_run(self.handle, ps, ph, pa, pw, _nbytes(workspace),
                                  _stream(stream)), "cs_batch_run")

    def graph(self, seeds: torch.Tensor, hist: torch.Tensor, actions: torch.Tensor,
              workspace: torch.Tensor) -> "BatchGraph":
        ps, ph, pa, pw = self._buffers(seeds, hist, actions, workspace)
        g = ctypes.c_void_p()
        _check(lib().cs_batch_graph_create(self.handle, ps, ph, pa, pw, _nbytes(workspace),
                                           ctypes.byref(g)), "cs_batch_graph_create")
        return BatchGraph(g, (seeds, hist, actions, workspace, self))

    def __del__(self):
        try:
            if getattr(self, "handle", None) is not None and self.handle.value:
                lib().cs_batch_free(self.handle)
        except Exception:
            pass


class BatchGraph:
    """An instantiated HIP graph of one ensemble run (wraps cs_batch_graph_*)."""

    def __init__(self, handle, keepalive):
        self.handle = handle
        self._keep = keepalive

    def launch(self, stream=None):
        _check(lib().cs_batch_graph_launch(self.handle, _stream(stream)), "cs_batch_graph_launch")

    def __del__(self):
        try:
            if self.handle is not None and self.handle.value:
                lib().cs_batch_graph_destroy(self.handle)
        except Exception:
            pass


def cs_autotune(cache_path: str, n_bucket: int = 0, counter: int = -1, stream=None):
    """Tune the ensemble counters' tiles per size bucket (n_bucket 0: all buckets; counter
    -1: all three counters) and write the choices to the JSON file cache_path."""
    _check(lib().cs_autotune(cache_path.encode(), _int(n_bucket, "n_bucket"), int(counter),
                             _stream(stream)), "cs_autotune")


def cs_measure_mfma_peak(counter: int, stream=None) -> float:
    """Sustained MFMA throughput (TOP/s) of the operand type of `counter` on this device."""
    out = ctypes.c_double(0.0)
    _check(lib().cs_measure_mfma_peak(counter, ctypes.byref(out), _stream(stream)),
           "cs_measure_mfma_peak")
    return out.value
