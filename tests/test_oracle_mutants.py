"""The oracle's pins reject plausible mistakes.

Each case applies one small edit to a copy of the oracle's C source:
- a dropped term
- a wrong direction, index or operand order
- an exclusive delta bound
- a lost tie-break
- swapped triangle types
- a wrong slice in the merge

It compiles the copy on the CPU and runs the pins of the part it edits
against it: tests/test_oracle.py for the three-edge oracle, tests/test_oracle4.py
for the four-node one (the wrapper loads the library named by TM_ORACLE_LIB).  Every mutant must make
that suite fail; the unmodified source, built the same way, must pass it.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DIR = os.path.join(ROOT, "oracle")

# (name, file, original text, replacement)
MUTANTS = [
    ("alg1-dropped-term", "tm_oracle.c",
     "raw[I_STAR(1, e1.dir, d, e3.dir)] += n_e[d] - mv;",
     "raw[I_STAR(1, e1.dir, d, e3.dir)] += n_e[d];"),
    ("alg1-map-direction", "tm_oracle.c",
     "mp->m_cnt[e3.dir][e3.v] += 1;", "mp->m_cnt[1 - e3.dir][e3.v] += 1;"),
    ("alg1-exclusive-delta", "tm_oracle.c",
     "if (e3.t - e1.t > delta) break;", "if (e3.t - e1.t >= delta) break;"),
    ("alg1-star3-transposed", "tm_oracle.c",
     "raw[I_STAR(2, e1.dir, d, e3.dir)] += mp->m_cnt[d][e1.v];",
     "raw[I_STAR(2, e1.dir, e3.dir, d)] += mp->m_cnt[d][e1.v];"),
    ("alg1-star1-wrong-neighbour", "tm_oracle.c",
     "raw[I_STAR(0, e1.dir, d, e3.dir)] += mp->m_cnt[d][e3.v];",
     "raw[I_STAR(0, e1.dir, d, e3.dir)] += mp->m_cnt[d][e1.v];"),
    ("tie-rule-drops-id", "tm_oracle.c",
     "return ta < tb || (ta == tb && ia < ib);", "return ta < tb;"),
    ("alg2-far-edge-direction", "tm_oracle.c",
     "int dk = ((uint32_t)r->src[ek] == v) ? DIR_O : DIR_IN;",
     "int dk = ((uint32_t)r->src[ek] == w) ? DIR_O : DIR_IN;"),
    ("alg2-types-swapped", "tm_oracle.c", "type = 0;", "type = 2;"),
    ("alg2-exclusive-delta", "tm_oracle.c",
     "if (ej.t > ei.t + delta) break;", "if (ej.t >= ei.t + delta) break;"),
    ("merge-pair-slice", "tm_oracle.c",
     "res[oracle_layout_pair(b, c)] += raw[I_PAIR(DIR_O, b, c)];",
     "res[oracle_layout_pair(b, c)] += raw[I_PAIR(DIR_IN, b, c)];"),
    ("merge-orbit-map", "tm_oracle.c",
     "uint64_t y = raw[I_TRI(1, 1 - c, 1 - b, 1 - a)];",
     "uint64_t y = raw[I_TRI(1, c, b, a)];"),
    ("layout-star-columns", "tm_oracle.c",
     "int col = 1 + 2 * (d2 == DIR_O) + (d1 == DIR_IN);",
     "int col = 1 + 2 * (d1 == DIR_IN) + (d2 == DIR_O);"),
    ("brute-star-type", "tm_brute.c",
     "int type = p12 ? 0 : (p02 ? 1 : 2);", "int type = p12 ? 2 : (p02 ? 1 : 0);"),
    ("brute-triangle-c", "tm_brute.c",
     "int c = S[e[0]] == v ? 0 : 1;", "int c = S[e[0]] == v ? 1 : 0;"),
    ("brute-pair-d3", "tm_brute.c",
     "d3 = S[e[2]] == p ? 0 : 1;", "d3 = S[e[1]] == p ? 0 : 1;"),
    ("brute-tie-order", "tm_brute.c",
     "return x < y ? -1 : (x > y);", "return x > y ? -1 : (x < y);"),
    ("brute-exclusive-delta", "tm_brute.c",
     "if (t[ord[c]] - t[ord[a]] > delta) break;",
     "if (t[ord[c]] - t[ord[a]] >= delta) break;"),
]


MUTANTS4 = [
    ("m4-local-reading-end", "tm_motif4.c", "if (rx < ry) { /* a - s - d - w */",
     "if (rx > ry) { /* a - s - d - w */"),
    ("m4-local-star-leaves", "tm_motif4.c", "if (nk == ni || nk == nj) continue;",
     "if (nk == ni) continue;"),
    ("m4-local-exclusive-delta", "tm_motif4.c", "if (hi - lo > delta) continue;",
     "if (hi - lo >= delta) continue;"),
    ("m4-local-triangle-not-excluded", "tm_motif4.c", "if (w == s || w == a) continue;",
     "if (w == s) continue;"),
    ("m4-brute-middle-bit", "tm_motif4.c", "f[mid] = (S[E[mid]] == v1);",
     "f[mid] = (S[E[mid]] == v2);"),
    ("m4-brute-star-direction", "tm_motif4.c", "idx = idx * 2 + (S[E[k]] == center ? 0 : 1);",
     "idx = idx * 2 + (S[E[k]] == center ? 1 : 0);"),
    ("m4-tie-order", "tm_motif4.c", "return x < y ? -1 : (x > y);",
     "return x > y ? -1 : (x < y);"),
]


def _build(workdir, edit):
    srcs = []
    for f in ("tm_oracle.c", "tm_brute.c", "tm_motif4.c"):
        with open(os.path.join(ORACLE_DIR, f)) as fh:
            text = fh.read()
        if edit is not None and edit[0] == f:
            assert text.count(edit[1]) == 1, f"mutation site not unique in {f}: {edit[1]}"
            text = text.replace(edit[1], edit[2])
        path = os.path.join(workdir, f)
        with open(path, "w") as fh:
            fh.write(text)
        srcs.append(path)
    return oracle.compile_lib(srcs, os.path.join(workdir, "liboracle_variant.so"))


def _run_pins(lib, pins="test_oracle.py"):
    env = dict(os.environ, TM_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", pins),
                        "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def _case(edit, pins="test_oracle.py"):
    with tempfile.TemporaryDirectory() as d:
        return _run_pins(_build(d, edit), pins)


def test_unmodified_copy_passes():
    rc, out = _case(None)
    assert rc == 0, out
    rc, out = _case(None, "test_oracle4.py")
    assert rc == 0, out


def test_every_mutant_is_caught():
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda m: _case((m[1], m[2], m[3])), MUTANTS))
    survivors = [m[0] for m, (rc, out) in zip(MUTANTS, results) if rc == 0]
    assert not survivors, f"mutants not caught by the pins: {survivors}"
    # each failure is a failed assertion, not a broken build or collection error
    for m, (rc, out) in zip(MUTANTS, results):
        assert rc == 1, f"{m[0]}: pytest exit {rc}\n{out}"


def test_every_four_node_mutant_is_caught():
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda m: _case((m[1], m[2], m[3]), "test_oracle4.py"), MUTANTS4))
    survivors = [m[0] for m, (rc, out) in zip(MUTANTS4, results) if rc == 0]
    assert not survivors, f"mutants not caught by the pins: {survivors}"
    for m, (rc, out) in zip(MUTANTS4, results):
        assert rc == 1, f"{m[0]}: pytest exit {rc}\n{out}"
