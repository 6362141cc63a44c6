"""CPU oracle for exact delta-temporal motif counts -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does, and shares no code with it.

Two independent C implementations, compiled with gcc into ``liboracle.so``:

* ``alg``   -- the paper's FAST-Star (Algorithm 1) and FAST-Tri (Algorithm 2)
               run per center as written, OpenMP over centers (Section IV-C);
               returns the paper's raw counters Star|Pair|Tri (56 x u64).
* ``brute`` -- every chronological edge triple inside delta classified by the
               definition (Definitions 2-3, Problem 1); returns raw counters
               built from each counter's definition and the class counts.

``brute4`` and ``local4`` (tm_motif4.c) count the 32 classes of four-node
three-edge motifs, the higher-order extension the paper leaves to future work,
by two enumerations of the same definition.

``merge`` turns raw counters into the 36 motif counts (Sections IV-A/IV-B:
isomorphic Pair cells, Tri orbit sum / 3) in the 6x6 layout.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
# The mutation tests point this at a deliberately broken copy of the oracle
# to show that the pins in tests/test_oracle.py reject it.
_LIB_PATH = os.environ.get("TM_ORACLE_LIB") or _DEFAULT_LIB
_SOURCES = [os.path.join(_HERE, "tm_oracle.c"), os.path.join(_HERE, "tm_brute.c"),
            os.path.join(_HERE, "tm_motif4.c")]
_lib = None

# status codes of the C functions
OK, EINVAL, ENOMEM, EINTERNAL = 0, -1, -2, -6


def compile_lib(sources, out_path: str) -> str:
    """gcc -O3 -fopenmp shared library from the given C sources."""
    tmp = out_path + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp] + list(sources)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out_path)
    return out_path


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (portable -O3, OpenMP)."""
    if force or not os.path.exists(_DEFAULT_LIB):
        compile_lib(_SOURCES, _DEFAULT_LIB)
    return _DEFAULT_LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) and _LIB_PATH == _DEFAULT_LIB:
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p32 = ctypes.POINTER(ctypes.c_int32)
        p64 = ctypes.POINTER(ctypes.c_int64)
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        pu32 = ctypes.POINTER(ctypes.c_uint32)
        lib.oracle_alg.argtypes = [p32, p32, p64, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_int64, ctypes.c_int, pu64]
        lib.oracle_alg.restype = ctypes.c_int
        lib.oracle_alg_centers.argtypes = [p32, p32, p64, ctypes.c_uint64, ctypes.c_uint32,
                                           ctypes.c_int64, pu32, ctypes.c_uint64, ctypes.c_int,
                                           pu64]
        lib.oracle_alg_centers.restype = ctypes.c_int
        lib.oracle_brute.argtypes = [p32, p32, p64, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_int64, pu64, pu64]
        lib.oracle_brute.restype = ctypes.c_int
        lib.oracle4_brute.argtypes = [p32, p32, p64, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_int64, pu64]
        lib.oracle4_brute.restype = ctypes.c_int
        lib.oracle4_local.argtypes = [p32, p32, p64, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_int64, ctypes.c_int, pu64]
        lib.oracle4_local.restype = ctypes.c_int
        lib.oracle_merge.argtypes = [pu64, pu64]
        lib.oracle_merge.restype = ctypes.c_int
        lib.oracle_validate.argtypes = [p32, p32, p64, ctypes.c_uint64, ctypes.c_uint32]
        lib.oracle_validate.restype = ctypes.c_int
        for name in ("oracle_layout_star", "oracle_layout_tri"):
            getattr(lib, name).restype = ctypes.c_int
        lib.oracle_layout_star.argtypes = [ctypes.c_int] * 4
        lib.oracle_layout_tri.argtypes = [ctypes.c_int] * 3
        lib.oracle_layout_pair.argtypes = [ctypes.c_int] * 2
        lib.oracle_layout_pair.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle status {code}")
        self.code = code


def _arrays(src, dst, t):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int64)
    if not (src.shape == dst.shape == t.shape) or src.ndim != 1:
        raise ValueError("src, dst, t must be 1-D arrays of one length")
    return src, dst, t


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _n_of(src, dst, n):
    if n is not None:
        return int(n)
    return int(max(src.max(), dst.max())) + 1 if src.size else 0


def alg(src, dst, t, delta: int, n: int | None = None, threads: int = 0) -> np.ndarray:
    """Raw counters (56 x u64) by the paper's Algorithms 1 and 2."""
    lib = _load()
    src, dst, t = _arrays(src, dst, t)
    raw = np.zeros(56, dtype=np.uint64)
    rc = lib.oracle_alg(_ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                        _ptr(t, ctypes.c_int64), src.size, _n_of(src, dst, n), int(delta),
                        int(threads), _ptr(raw, ctypes.c_uint64))
    if rc:
        raise OracleError(rc)
    return raw


def alg_centers(src, dst, t, delta: int, centers, n: int | None = None,
                threads: int = 0) -> np.ndarray:
    """Raw counters contributed by the listed center nodes only."""
    lib = _load()
    src, dst, t = _arrays(src, dst, t)
    c = np.ascontiguousarray(centers, dtype=np.uint32)
    raw = np.zeros(56, dtype=np.uint64)
    rc = lib.oracle_alg_centers(_ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                                _ptr(t, ctypes.c_int64), src.size, _n_of(src, dst, n),
                                int(delta), _ptr(c, ctypes.c_uint32), c.size, int(threads),
                                _ptr(raw, ctypes.c_uint64))
    if rc:
        raise OracleError(rc)
    return raw


def brute(src, dst, t, delta: int, n: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """(raw[56], canon[36]) by enumerating the definition."""
    lib = _load()
    src, dst, t = _arrays(src, dst, t)
    raw = np.zeros(56, dtype=np.uint64)
    canon = np.zeros(36, dtype=np.uint64)
    rc = lib.oracle_brute(_ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                          _ptr(t, ctypes.c_int64), src.size, _n_of(src, dst, n), int(delta),
                          _ptr(raw, ctypes.c_uint64), _ptr(canon, ctypes.c_uint64))
    if rc:
        raise OracleError(rc)
    return raw, canon


def brute4(src, dst, t, delta: int, n: int | None = None) -> np.ndarray:
    """Four-node three-edge motif counts (32 x u64, layout in tm_motif4.c) by
    classifying every chronological edge triple inside delta."""
    lib = _load()
    src, dst, t = _arrays(src, dst, t)
    out = np.zeros(32, dtype=np.uint64)
    rc = lib.oracle4_brute(_ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                           _ptr(t, ctypes.c_int64), src.size, _n_of(src, dst, n), int(delta),
                           _ptr(out, ctypes.c_uint64))
    if rc:
        raise OracleError(rc)
    return out


def local4(src, dst, t, delta: int, n: int | None = None, threads: int = 0) -> np.ndarray:
    """The same 32 counts, enumerated per center node (stars) and per middle
    edge (paths)."""
    lib = _load()
    src, dst, t = _arrays(src, dst, t)
    out = np.zeros(32, dtype=np.uint64)
    rc = lib.oracle4_local(_ptr(src, ctypes.c_int32), _ptr(dst, ctypes.c_int32),
                           _ptr(t, ctypes.c_int64), src.size, _n_of(src, dst, n), int(delta),
                           int(threads), _ptr(out, ctypes.c_uint64))
    if rc:
        raise OracleError(rc)
    return out


def merge(raw) -> np.ndarray:
    """36 motif counts as a 6x6 uint64 matrix (row i, column j = M_ij)."""
    lib = _load()
    raw = np.ascontiguousarray(raw, dtype=np.uint64)
    out = np.zeros(36, dtype=np.uint64)
    rc = lib.oracle_merge(_ptr(raw, ctypes.c_uint64), _ptr(out, ctypes.c_uint64))
    if rc:
        raise OracleError(rc)
    return out.reshape(6, 6)


def count(src, dst, t, delta: int, n: int | None = None, threads: int = 0) -> np.ndarray:
    """The 6x6 motif count matrix (paper's algorithms + merge)."""
    return merge(alg(src, dst, t, delta, n=n, threads=threads))


def layout_star(ty: int, d1: int, d2: int, d3: int) -> int:
    return _load().oracle_layout_star(ty, d1, d2, d3)


def layout_tri(a: int, b: int, c: int) -> int:
    return _load().oracle_layout_tri(a, b, c)


def layout_pair(d2: int, d3: int) -> int:
    return _load().oracle_layout_pair(d2, d3)


def canon_to_grid(canon) -> np.ndarray:
    """Place class counts in canonical order (brute's output) on the 6x6 grid
    using the oracle's layout."""
    canon = np.asarray(canon, dtype=np.uint64)
    out = np.zeros(36, dtype=np.uint64)
    for ty in range(3):
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    out[layout_star(ty, a, b, c)] += canon[ty * 8 + a * 4 + b * 2 + c]
    for b in range(2):
        for c in range(2):
            out[layout_pair(b, c)] += canon[24 + b * 2 + c]
    for a in range(2):
        for b in range(2):
            for c in range(2):
                out[layout_tri(a, b, c)] += canon[28 + a * 4 + b * 2 + c]
    return out.reshape(6, 6)
