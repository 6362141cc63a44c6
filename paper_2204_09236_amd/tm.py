"""Python binding of libtm.so (ctypes).  Argument marshalling only: every step
of the counting path runs in the library's HIP kernels.

Inputs are either host numpy arrays (copied in by the library) or torch
tensors on the GPU (read in place on the current torch stream).  Results are
numpy uint64 arrays: ``count`` gives the 6x6 motif matrix M_ij, ``count_raw``
the paper's 56 raw counters (Star | Pair | Tri).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtm.so")

TM_OK, TM_EINVAL, TM_ENOMEM, TM_EHIP, TM_EAGAIN, TM_ENOTFOUND, TM_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
# motif families (tm_count_masked)
STARS, PAIRS, TRIANGLES, ALL_MOTIFS = 1, 2, 4, 7
HUB_OFF = 0xFFFFFFFF   # hub_min value that keeps the hub triangle pass off
TM_HOST_PTRS, TM_DEVICE_PTRS = 0, 1


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.tm_build_graph.argtypes = [vp, vp, vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, vp,
                                   ctypes.POINTER(vp)]
    lib.tm_build_graph.restype = ctypes.c_int
    lib.tm_graph_free.argtypes = [vp]
    lib.tm_graph_free.restype = None
    lib.tm_count.argtypes = [vp, ctypes.c_int64, u64p]
    lib.tm_count_masked.argtypes = [vp, ctypes.c_int64, ctypes.c_uint32, u64p]
    lib.tm_count.restype = ctypes.c_int
    lib.tm_count_raw.argtypes = [vp, ctypes.c_int64, u64p]
    lib.tm_count_raw.restype = ctypes.c_int
    lib.tm_count_raw_tuned.argtypes = [vp, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_uint32, u64p]
    lib.tm_count_raw_tuned.restype = ctypes.c_int
    lib.tm_merge.argtypes = [u64p, u64p]
    lib.tm_merge.restype = ctypes.c_int
    lib.tm_graph_info.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), u64p, u64p, u64p, u64p]
    lib.tm_graph_info.restype = ctypes.c_int
    lib.tm_graph_sequences.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.tm_graph_sequences.restype = ctypes.c_int
    lib.tm_prof_enable.argtypes = [ctypes.c_int]
    lib.tm_prof_enable.restype = None
    lib.tm_prof_only.argtypes = [ctypes.c_char_p]
    lib.tm_prof_only.restype = None
    lib.tm_prof_reset.argtypes = []
    lib.tm_prof_reset.restype = None
    lib.tm_prof_read.argtypes = [ctypes.c_int, ctypes.c_char_p, ctypes.c_int, u64p,
                                 ctypes.POINTER(ctypes.c_double)]
    lib.tm_prof_read.restype = ctypes.c_int
    lib.tm_build_batch.argtypes = [vp, vp, vp, u64p, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32,
                                   ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.tm_build_batch.restype = ctypes.c_int
    lib.tm_graph_count.argtypes = [vp]
    lib.tm_graph_count.restype = ctypes.c_uint32
    lib.tm_count_batch.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), u64p]
    lib.tm_count_batch.restype = ctypes.c_int
    lib.tm_count_batch_raw.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), u64p]
    lib.tm_count_batch_raw.restype = ctypes.c_int
    lib.tm_count_batch_raw_ex.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, u64p]
    lib.tm_count_batch_raw_ex.restype = ctypes.c_int
    lib.tm_autotune.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint32),
                                ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                ctypes.POINTER(ctypes.c_float)]
    lib.tm_autotune.restype = ctypes.c_int
    lib.tm_autotune_multi.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_uint32,
                                      ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                      ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_float)]
    lib.tm_autotune_multi.restype = ctypes.c_int
    lib.tm_count4.argtypes = [vp, ctypes.c_int64, u64p, u64p]
    lib.tm_count4.restype = ctypes.c_int
    lib.tm_count_multi.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_uint32, u64p]
    lib.tm_count_multi.restype = ctypes.c_int
    lib.tm_count_multi_raw.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_uint32, u64p]
    lib.tm_count_multi_raw.restype = ctypes.c_int
    lib.tm_stream_create.argtypes = [ctypes.c_int64, ctypes.c_uint32, vp, ctypes.POINTER(vp)]
    lib.tm_stream_create.restype = ctypes.c_int
    lib.tm_stream_append.argtypes = [vp, vp, vp, vp, ctypes.c_uint64, ctypes.c_int, u64p]
    lib.tm_stream_append.restype = ctypes.c_int
    lib.tm_stream_totals.argtypes = [vp, u64p, u64p, u64p]
    lib.tm_stream_totals.restype = ctypes.c_int
    lib.tm_stream_free.argtypes = [vp]
    lib.tm_stream_free.restype = None
    lib.tm_server_create.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.POINTER(vp)]
    lib.tm_server_create.restype = ctypes.c_int
    lib.tm_submit.argtypes = [vp, ctypes.c_uint64, vp, vp, vp, ctypes.c_uint64, ctypes.c_uint32,
                              ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]
    lib.tm_submit.restype = ctypes.c_int
    lib.tm_poll.argtypes = [vp, ctypes.c_uint64, u64p, u64p]
    lib.tm_poll.restype = ctypes.c_int
    lib.tm_wait.argtypes = [vp, ctypes.c_uint64, u64p, u64p, ctypes.c_uint32]
    lib.tm_wait.restype = ctypes.c_int
    lib.tm_server_stats.argtypes = [vp, u64p]
    lib.tm_server_stats.restype = ctypes.c_int
    lib.tm_server_destroy.argtypes = [vp]
    lib.tm_server_destroy.restype = None
    lib.tm_strerror.argtypes = [ctypes.c_int]
    lib.tm_strerror.restype = ctypes.c_char_p
    lib.tm_last_error.argtypes = []
    lib.tm_last_error.restype = ctypes.c_char_p
    lib.tm_count_noalloc.argtypes = [vp, ctypes.c_int64, u64p]
    lib.tm_count_noalloc.restype = ctypes.c_int
    lib.tm_debug_alloc_calls.argtypes = []
    lib.tm_debug_alloc_calls.restype = ctypes.c_uint64
    lib.tm_debug_force_edge_sort.argtypes = [ctypes.c_int]
    lib.tm_debug_force_edge_sort.restype = None
    lib.tm_debug_lookback_giveup.argtypes = [ctypes.c_int]
    lib.tm_debug_lookback_giveup.restype = None
    return lib


_lib = _load()


class TMError(RuntimeError):
    def __init__(self, code: int):
        detail = _lib.tm_last_error().decode(errors="replace")
        super().__init__(f"{_lib.tm_strerror(code).decode()} ({code}): {detail}")
        self.code = code


def _check(rc: int) -> None:
    if rc != TM_OK:
        raise TMError(rc)


def _u64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _is_torch_device(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


class Graph:
    """A device-resident graph: S_u sequences and node-pair edge sets."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    @property
    def handle(self):
        if not self._h:
            raise ValueError("graph was freed")
        return self._h

    def count(self, delta: int, families: int = 7) -> np.ndarray:
        """36 motif counts (6 x 6).  families: OR of STARS, PAIRS, TRIANGLES
        (tm_count_masked); cells of the other families are 0."""
        out = np.zeros(36, dtype=np.uint64)
        if families == ALL_MOTIFS:
            _check(_lib.tm_count(self.handle, int(delta), _u64(out)))
        else:
            _check(_lib.tm_count_masked(self.handle, int(delta), int(families), _u64(out)))
        return out.reshape(6, 6)

    def count_noalloc(self, delta: int) -> np.ndarray:
        """36 motif counts (6 x 6) by tm_count_noalloc: no device allocation,
        workspace in the library's fixed device array."""
        out = np.zeros(36, dtype=np.uint64)
        _check(_lib.tm_count_noalloc(self.handle, int(delta), _u64(out)))
        return out.reshape(6, 6)

    def count_raw(self, delta: int, run_chunk: int = 0, tri_lane_max: int = 0,
                  hub_min: int = 0) -> np.ndarray:
        """Raw counters; the partition parameters (0 = tuned or default,
        hub_min=HUB_OFF: no hub pass) change the schedule, never the result."""
        raw = np.zeros(56, dtype=np.uint64)
        _check(_lib.tm_count_raw_tuned(self.handle, int(delta), int(run_chunk), int(tri_lane_max),
                                       int(hub_min), _u64(raw)))
        return raw

    def count_multi(self, deltas) -> np.ndarray:
        """Counts for several windows in one call: (k, 6, 6)."""
        d = np.ascontiguousarray(deltas, dtype=np.int64).reshape(-1)
        out = np.zeros((d.size, 36), dtype=np.uint64)
        _check(_lib.tm_count_multi(self.handle, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   d.size, _u64(out)))
        return out.reshape(d.size, 6, 6)

    def count4(self, delta: int, with_raw: bool = False):
        """Four-node three-edge motif counts (32, layout of tm_count4); with
        with_raw also the 56 raw three-edge counters of the same delta."""
        out = np.zeros(32, dtype=np.uint64)
        raw = np.zeros(56, dtype=np.uint64)
        _check(_lib.tm_count4(self.handle, int(delta), _u64(raw), _u64(out)))
        return (out, raw) if with_raw else out

    def count_multi_raw(self, deltas) -> np.ndarray:
        """Raw counters for several windows in one call: (k, 56)."""
        d = np.ascontiguousarray(deltas, dtype=np.int64).reshape(-1)
        out = np.zeros((d.size, 56), dtype=np.uint64)
        _check(_lib.tm_count_multi_raw(self.handle, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       d.size, _u64(out)))
        return out

    @property
    def num_graphs(self) -> int:
        return int(_lib.tm_graph_count(self.handle))

    def _deltas(self, deltas) -> np.ndarray:
        d = np.ascontiguousarray(np.broadcast_to(np.asarray(deltas, dtype=np.int64),
                                                 (self.num_graphs,)))
        return d

    def count_batch(self, deltas) -> np.ndarray:
        """(G, 6, 6) motif counts, graph i with window deltas[i]."""
        d = self._deltas(deltas)
        out = np.zeros((d.size, 36), dtype=np.uint64)
        _check(_lib.tm_count_batch(self.handle, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   _u64(out)))
        return out.reshape(-1, 6, 6)

    def count_batch_raw(self, deltas) -> np.ndarray:
        """(G, 56) raw counters, graph i with window deltas[i]."""
        d = self._deltas(deltas)
        out = np.zeros((d.size, 56), dtype=np.uint64)
        _check(_lib.tm_count_batch_raw(self.handle,
                                       d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _u64(out)))
        return out

    def count_batch_raw_ex(self, deltas, run_chunk: int = 0, tri_lane_max: int = 0,
                           use_graph: bool = True, hub_min: int = 0) -> np.ndarray:
        d = self._deltas(deltas)
        out = np.zeros((d.size, 56), dtype=np.uint64)
        _check(_lib.tm_count_batch_raw_ex(self.handle,
                                          d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          int(run_chunk), int(tri_lane_max), int(hub_min),
                                          1 if use_graph else 0, _u64(out)))
        return out

    def autotune(self, deltas) -> dict:
        d = self._deltas(deltas)
        c, l, h, ms = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_float()
        _check(_lib.tm_autotune(self.handle, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                ctypes.byref(c), ctypes.byref(l), ctypes.byref(h), ctypes.byref(ms)))
        return {"run_chunk": c.value, "tri_lane_max": l.value, "hub_min": h.value, "ms": ms.value}

    def autotune_multi(self, deltas) -> dict:
        """The autotuner for count_multi of one graph over these windows."""
        d = np.ascontiguousarray(deltas, dtype=np.int64).reshape(-1)
        c, l, h, ms = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_float()
        _check(_lib.tm_autotune_multi(self.handle, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      d.size, ctypes.byref(c), ctypes.byref(l), ctypes.byref(h),
                                      ctypes.byref(ms)))
        return {"run_chunk": c.value, "tri_lane_max": l.value, "hub_min": h.value, "ms": ms.value}

    def info(self) -> dict:
        n = ctypes.c_uint32()
        m, mp, me, md = (ctypes.c_uint64() for _ in range(4))
        _check(_lib.tm_graph_info(self.handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(mp),
                                  ctypes.byref(me), ctypes.byref(md)))
        return {"n": n.value, "m": m.value, "multi_pairs": mp.value, "multi_pair_edges": me.value,
                "max_degree": md.value}

    def sequences(self) -> dict:
        inf = self.info()
        n, m = inf["n"], inf["m"]
        off = np.zeros(n + 1, np.uint32)
        t = np.zeros(2 * m, np.int64)
        nbr = np.zeros(2 * m, np.uint32)
        dr = np.zeros(2 * m, np.uint8)
        ids = np.zeros(2 * m, np.uint32)
        _check(_lib.tm_graph_sequences(self.handle, off.ctypes.data, t.ctypes.data, nbr.ctypes.data,
                                       dr.ctypes.data, ids.ctypes.data))
        return {"off": off, "t": t, "nbr": nbr, "dir": dr, "id": ids}

    def free(self) -> None:
        if self._h:
            _lib.tm_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


def build_graph(src, dst, t, n: int | None = None, stream=None) -> Graph:
    """Build the device graph.  ``src``/``dst``/``t`` are int32/int32/int64,
    either host numpy arrays or torch tensors on the GPU (then read on
    ``stream``, default: torch's current stream)."""
    h = ctypes.c_void_p()
    if _is_torch_device(src):
        import torch
        if not (src.dtype == torch.int32 and dst.dtype == torch.int32 and t.dtype == torch.int64):
            raise TypeError("device inputs must be int32, int32, int64 tensors")
        src, dst, t = src.contiguous(), dst.contiguous(), t.contiguous()
        m = src.numel()
        if stream is None:
            stream = torch.cuda.current_stream()
        sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        _check(_lib.tm_build_graph(src.data_ptr(), dst.data_ptr(), t.data_ptr(), m,
                                   int(n or 0), TM_DEVICE_PTRS, sp, ctypes.byref(h)))
    else:
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        tt = np.ascontiguousarray(t, dtype=np.int64)
        if not (s.shape == d.shape == tt.shape and s.ndim == 1):
            raise ValueError("src, dst, t must be 1-D arrays of one length")
        sp = ctypes.c_void_p(int(stream) if stream is not None else 0)
        _check(_lib.tm_build_graph(s.ctypes.data, d.ctypes.data, tt.ctypes.data, s.size,
                                   int(n or 0), TM_HOST_PTRS, sp, ctypes.byref(h)))
    return Graph(h)


def build_batch(graphs, stream=None) -> Graph:
    """Build G independent graphs as one device object.  ``graphs`` is a list
    of (src, dst, t) or (src, dst, t, n) host arrays with node ids local to
    each graph (n = 0 or missing: max id + 1)."""
    srcs, dsts, ts, ns = [], [], [], []
    for gr in graphs:
        srcs.append(np.ascontiguousarray(gr[0], dtype=np.int32))
        dsts.append(np.ascontiguousarray(gr[1], dtype=np.int32))
        ts.append(np.ascontiguousarray(gr[2], dtype=np.int64))
        ns.append(int(gr[3]) if len(gr) > 3 and gr[3] is not None else 0)
    off = np.zeros(len(graphs) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([a.size for a in srcs])
    src = np.concatenate(srcs) if srcs else np.zeros(0, np.int32)
    dst = np.concatenate(dsts) if dsts else np.zeros(0, np.int32)
    t = np.concatenate(ts) if ts else np.zeros(0, np.int64)
    return build_batch_arrays(src, dst, t, off, np.asarray(ns, dtype=np.uint32), stream=stream)


def build_batch_arrays(src, dst, t, edge_off, node_count, stream=None) -> Graph:
    """Batched build from concatenated arrays (host numpy or GPU torch
    tensors) with host ``edge_off`` (G + 1) and ``node_count`` (G)."""
    off = np.ascontiguousarray(edge_off, dtype=np.uint64)
    nc = np.ascontiguousarray(node_count, dtype=np.uint32)
    G = nc.size
    if off.size != G + 1:
        raise ValueError("edge_off needs G + 1 entries")
    h = ctypes.c_void_p()
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    ncp = nc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    if _is_torch_device(src):
        import torch
        if not (src.dtype == torch.int32 and dst.dtype == torch.int32 and t.dtype == torch.int64):
            raise TypeError("device inputs must be int32, int32, int64 tensors")
        src, dst, t = src.contiguous(), dst.contiguous(), t.contiguous()
        if stream is None:
            stream = torch.cuda.current_stream()
        sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        _check(_lib.tm_build_batch(src.data_ptr(), dst.data_ptr(), t.data_ptr(), offp, ncp, G,
                                   TM_DEVICE_PTRS, sp, ctypes.byref(h)))
    else:
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        tt = np.ascontiguousarray(t, dtype=np.int64)
        sp = ctypes.c_void_p(int(stream) if stream is not None else 0)
        _check(_lib.tm_build_batch(s.ctypes.data, d.ctypes.data, tt.ctypes.data, offp, ncp, G,
                                   TM_HOST_PTRS, sp, ctypes.byref(h)))
    return Graph(h)


def count(src, dst, t, delta: int, n: int | None = None) -> np.ndarray:
    with build_graph(src, dst, t, n=n) as g:
        return g.count(delta)


def merge(raw) -> np.ndarray:
    raw = np.ascontiguousarray(raw, dtype=np.uint64)
    out = np.zeros(36, dtype=np.uint64)
    _check(_lib.tm_merge(_u64(raw), _u64(out)))
    return out.reshape(6, 6)


class Stream:
    """Incremental counts of an append-only edge stream (tm.h: tm_stream_*).
    ``append`` returns the 6 x 6 counts of the instances whose last edge is
    in the batch; batches must not go back in time."""

    def __init__(self, delta: int, n: int = 0, stream=None):
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(0)
        if stream is not None:
            sp = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self._sp = sp
        _check(_lib.tm_stream_create(int(delta), int(n), sp, ctypes.byref(h)))
        self._h = h

    def append(self, src, dst, t) -> np.ndarray:
        out = np.zeros(36, dtype=np.uint64)
        if _is_torch_device(src):
            import torch
            if not (src.dtype == torch.int32 and dst.dtype == torch.int32 and t.dtype == torch.int64):
                raise TypeError("device inputs must be int32, int32, int64 tensors")
            src, dst, t = src.contiguous(), dst.contiguous(), t.contiguous()
            _check(_lib.tm_stream_append(self._h, src.data_ptr(), dst.data_ptr(), t.data_ptr(),
                                         src.numel(), TM_DEVICE_PTRS, _u64(out)))
        else:
            s = np.ascontiguousarray(src, dtype=np.int32)
            d = np.ascontiguousarray(dst, dtype=np.int32)
            tt = np.ascontiguousarray(t, dtype=np.int64)
            if not (s.shape == d.shape == tt.shape and s.ndim == 1):
                raise ValueError("src, dst, t must be 1-D arrays of one length")
            _check(_lib.tm_stream_append(self._h, s.ctypes.data, d.ctypes.data, tt.ctypes.data,
                                         s.size, TM_HOST_PTRS, _u64(out)))
        return out.reshape(6, 6)

    def totals(self) -> tuple[np.ndarray, int, int]:
        """(6 x 6 counts of every edge so far, edges so far, edges kept in the tail)."""
        out = np.zeros(36, dtype=np.uint64)
        e, k = ctypes.c_uint64(), ctypes.c_uint64()
        _check(_lib.tm_stream_totals(self._h, _u64(out), ctypes.byref(e), ctypes.byref(k)))
        return out.reshape(6, 6), e.value, k.value

    def free(self):
        if self._h:
            _lib.tm_stream_free(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


class Server:
    """Request loop with continuous batching (see tm.h: tm_server_*)."""

    def __init__(self, budget_bytes: int, max_inflight: int = 16, max_queue: int = 1 << 20):
        h = ctypes.c_void_p()
        _check(_lib.tm_server_create(int(budget_bytes), int(max_inflight), int(max_queue),
                                     ctypes.byref(h)))
        self._h = h

    def submit(self, delta: int, src=None, dst=None, t=None, n: int = 0, key: int = 0) -> int:
        """Queue a request; returns its ticket.  Raises TMError (code
        TM_EAGAIN when the queue is full)."""
        tk = ctypes.c_uint64()
        if src is None:
            _check(_lib.tm_submit(self._h, int(key), None, None, None, 0, int(n), int(delta),
                                  ctypes.byref(tk)))
        else:
            s = np.ascontiguousarray(src, dtype=np.int32)
            d = np.ascontiguousarray(dst, dtype=np.int32)
            tt = np.ascontiguousarray(t, dtype=np.int64)
            _check(_lib.tm_submit(self._h, int(key), s.ctypes.data, d.ctypes.data, tt.ctypes.data,
                                  s.size, int(n), int(delta), ctypes.byref(tk)))
        return tk.value

    def poll(self, ticket: int):
        """(status, 6x6 counts or None, (submit, start, done) ns); status
        TM_EAGAIN while pending.  A final status releases the ticket."""
        out = np.zeros(36, dtype=np.uint64)
        times = np.zeros(3, dtype=np.uint64)
        rc = _lib.tm_poll(self._h, int(ticket), _u64(out), _u64(times))
        return rc, (out.reshape(6, 6) if rc == TM_OK else None), tuple(int(x) for x in times)

    def wait(self, ticket: int, timeout_ms: int = 600000):
        out = np.zeros(36, dtype=np.uint64)
        times = np.zeros(3, dtype=np.uint64)
        rc = _lib.tm_wait(self._h, int(ticket), _u64(out), _u64(times), int(timeout_ms))
        return rc, (out.reshape(6, 6) if rc == TM_OK else None), tuple(int(x) for x in times)

    def stats(self) -> dict:
        st = np.zeros(8, dtype=np.uint64)
        _check(_lib.tm_server_stats(self._h, _u64(st)))
        keys = ["queued", "in_flight", "resident_graphs", "resident_bytes", "in_flight_bytes",
                "completed", "failed", "budget"]
        return {k: int(v) for k, v in zip(keys, st)}

    def close(self) -> None:
        if self._h:
            _lib.tm_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- kernel timing
def prof_enable(on: bool = True) -> None:
    _lib.tm_prof_enable(1 if on else 0)


def prof_only(name: str | None) -> None:
    """Trace only launches of ``name`` (None: all)."""
    _lib.tm_prof_only(name.encode() if name else None)


def prof_reset() -> None:
    _lib.tm_prof_reset()


def prof_read() -> dict:
    """{kernel name: (launches, total ms)} for launches since the last reset."""
    out = {}
    i = 0
    buf = ctypes.create_string_buffer(128)
    while True:
        n, ms = ctypes.c_uint64(), ctypes.c_double()
        rc = _lib.tm_prof_read(i, buf, 128, ctypes.byref(n), ctypes.byref(ms))
        if rc != TM_OK:
            break
        out[buf.value.decode()] = (n.value, ms.value)
        i += 1
    return out


def last_error() -> str:
    """This thread's last error message from the library (for a failed
    request: the message of the call that failed it)."""
    return (_lib.tm_last_error() or b"").decode()


def debug_alloc_calls() -> int:
    """Device allocations the library has served so far (cache hits included)."""
    return int(_lib.tm_debug_alloc_calls())


def debug_force_edge_sort(on: bool) -> None:
    """Testing: every later build makes its edge-position index by the
    partition and bucket fill, whatever its size."""
    _lib.tm_debug_force_edge_sort(1 if on else 0)


def debug_lookback_giveup(on: bool) -> None:
    """Failure-path testing: every look-back wait of later builds gives up
    at once (the build then returns TM_EINTERNAL)."""
    _lib.tm_debug_lookback_giveup(1 if on else 0)


def library():
    """The loaded ctypes library (for ABI checks)."""
    return _lib
