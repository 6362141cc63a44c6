"""Exact delta-temporal motif counting on AMD Instinct MI355X (gfx950).

The counting path runs in the HIP library ``libtm.so`` (C ABI in
``include/tm.h``); this package is its thin Python binding.  Importing it
fails loudly if the library has not been built.
"""
from .tm import (ALL_MOTIFS, HUB_OFF, PAIRS, STARS, TRIANGLES, Graph, Server, Stream, TMError,  # noqa: F401
                 build_batch, build_batch_arrays, build_graph, count, debug_alloc_calls,
                 debug_force_edge_sort, debug_lookback_giveup, last_error, merge,
                 prof_enable, prof_only, prof_read, prof_reset)
