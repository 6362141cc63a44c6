"""C-ABI checks that need no GPU: the library loads, exports every function
include/tm.h declares, and its host-side merge agrees with the oracle's own
copy of the 36-cell layout."""
import os
import re

import numpy as np
import pytest

import oracle
from motif_defs import GRID, grid_from_canon

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(tm_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    import paper_2204_09236_amd as pkg
    lib = pkg.tm.library()
    names = declared_functions()
    assert "tm_build_graph" in names and "tm_count" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_library_is_in_tree():
    import paper_2204_09236_amd as pkg
    assert os.path.dirname(pkg.tm.LIB_PATH) == os.path.join(ROOT, "paper_2204_09236_amd")


def _symmetric_raw(rng):
    """A raw counter vector that satisfies the merge's self-checks: Pair
    views mirrored, and the three Tri views of each class equal."""
    raw = np.zeros(56, np.uint64)
    raw[:24] = rng.integers(0, 1000, 24)
    pair = rng.integers(0, 1000, 4)
    for a in range(2):
        for b in range(2):
            raw[24 + 0 + a * 2 + b] = pair[a * 2 + b]
            raw[24 + 4 + (1 - a) * 2 + (1 - b)] = pair[a * 2 + b]
    cls = rng.integers(0, 1000, 8)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                v = cls[a * 4 + b * 2 + c]
                raw[32 + a * 4 + b * 2 + c] = v
                raw[40 + (1 - c) * 4 + (1 - b) * 2 + (1 - a)] = v
                raw[48 + c * 4 + (1 - a) * 2 + (1 - b)] = v
    return raw


def test_merge_layout_agrees_with_oracle_and_spec():
    from paper_2204_09236_amd import merge
    rng = np.random.default_rng(5)
    for _ in range(20):
        raw = _symmetric_raw(rng)
        lib_grid = merge(raw)
        np.testing.assert_array_equal(lib_grid, oracle.merge(raw))
        canon = np.concatenate([raw[:24], raw[24:28], raw[32:40]])
        np.testing.assert_array_equal(lib_grid, grid_from_canon(canon))
    assert len(set(GRID.values())) == 36


def test_merge_rejects_broken_symmetry():
    from paper_2204_09236_amd import TMError, merge
    raw = np.zeros(56, np.uint64)
    raw[24] = 1
    with pytest.raises(TMError):
        merge(raw)
    raw = np.zeros(56, np.uint64)
    raw[32] = 3
    with pytest.raises(TMError):
        merge(raw)


def test_null_arguments_rejected_without_a_device():
    """Entry points check their pointers before any HIP call: a NULL graph
    or output gives TM_EINVAL (-1) and an error message, on a host with no
    GPU as well."""
    import ctypes
    import paper_2204_09236_amd as pkg
    lib = pkg.tm.library()
    d = (ctypes.c_int64 * 3)(600, 3600, 86400)
    out36 = (ctypes.c_uint64 * (36 * 3))()
    raw56 = (ctypes.c_uint64 * (56 * 3))()
    out32 = (ctypes.c_uint64 * 32)()
    calls = [
        ("tm_autotune", (None, d, None, None, None, None)),
        ("tm_autotune_multi", (None, d, 3, None, None, None, None)),
        ("tm_count", (None, 600, None)),
        ("tm_count_raw", (None, 600, raw56)),
        ("tm_count_masked", (None, 600, 7, None)),
        ("tm_count_multi", (None, d, 3, None)),
        ("tm_count_multi_raw", (None, d, 3, raw56)),
        ("tm_count4", (None, 600, raw56, out32)),
        ("tm_graph_info", (None, None, None, None, None, None)),
        ("tm_merge", (None, out36)),
    ]
    for name, args in calls:
        rc = getattr(lib, name)(*args)
        assert rc == -1, (name, rc)
    msg = lib.tm_last_error()
    assert msg, "no error message after a rejected call"
