"""Mutation tests of the oracle's pins: plausible mistakes are planted in a copy of the oracle's
C source (an off-by-one sample or splitter index, a dropped tie-break, a row-major scan, wrong
pad keys, a short bisection range, a flipped float order, a misplaced piece), each copy is built
on its own, and the oracle pin tests (tests/test_oracle.py) are run against it in a separate
process.  Every mutant must make at least one pin fail.  CPU only; the real oracle is untouched."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dss_oracle.c")

# (name, text in the oracle source, replacement)
MUTANTS = [
    ("sample_position", ": k * w - 1;", ": (k - 1) * w;"),
    ("splitter_index", "g[j - 1] = S[j * m - 1];", "g[j - 1] = S[(j - 1) * m];"),
    ("rank_ties", "return key < gkey || (key == gkey && pos <= gpos);",
     "return key < gkey || (key == gkey && pos < gpos);"),
    ("rank_ignores_position", "return key < gkey || (key == gkey && pos <= gpos);",
     "return key <= gkey;"),
    # Tie-breaks reversed.  (Dropping them instead is an equivalent mutant with glibc, whose
    # qsort is a stable merge sort and sees items and samples already in tie-break order.)
    ("item_tie_break", "if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;",
     "if (a->idx != b->idx) return a->idx < b->idx ? 1 : -1;"),
    ("sample_tie_break", "if (a->pos != b->pos) return a->pos < b->pos ? -1 : 1;",
     "if (a->pos != b->pos) return a->pos < b->pos ? 1 : -1;"),
    ("pad_key", "A[t].key = key_max(kind);", "A[t].key = 0;"),
    ("bisection_range", "uint64_t lo = 0, hi = L; /* invariant", "uint64_t lo = 0, hi = L - 1; /* invariant"),
    ("scan_row_major",
     "for (uint64_t j = 0; j < s; ++j) {\n        bsz[j] = 0;\n        for (uint64_t i = 0; i < m; ++i) {",
     "for (uint64_t j = 0; j < s; ++j) bsz[j] = 0;\n    for (uint64_t i = 0; i < m; ++i) {\n        for (uint64_t j = 0; j < s; ++j) {"),
    ("piece_start", "out[l[i * s + j] + x] = A[i * L + r[i * (s + 1) + j] + x];",
     "out[l[i * s + j] + x] = A[i * L + r[i * (s + 1) + j] + x - (x > 0)];"),
    ("bucket_sort_skipped", "qsort(out + start, bsz[j], sizeof(item_t), cmp_item);", ""),
    ("f32_negatives_unflipped", "return (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);",
     "return (bits & 0x80000000u) ? (bits & 0x7FFFFFFFu) : (bits | 0x80000000u);"),
    ("values_left_behind", "if (vals_out) vals_out[t] = out[t].val;",
     "if (vals_out) vals_out[t] = vals_in ? vals_in[t] : 0;"),
    # the randomized-splitter variant (R8)
    ("random_draw_index", "oracle_splitmix64(seed, i * s + k);",
     "oracle_splitmix64(seed, i * s + k + 1);"),
    ("random_position_bits", "return ((d >> 32) * L) >> 32;",
     "return ((d & 0xFFFFFFFFull) * L) >> 32;"),
    ("random_last_bucket_open", "if (sampling && j == s) lo = L;", ""),
    ("splitmix_finaliser_shift", "z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;",
     "z = (z ^ (z >> 29)) * 0x94D049BB133111EBull;"),
]


def _build(tmp_path, text, name):
    c = tmp_path / f"{name}.c"
    c.write_text(text)
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w", str(c), "-o",
                           str(so)])
    return str(so)


def _run_pins(lib, args=()):
    env = dict(os.environ, DSS_ORACLE_LIB=lib)
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle.py"), "-x",
           "-q", "-p", "no:cacheprovider", *args]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.fixture(scope="module")
def source():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    return open(SRC).read()


def test_harness_passes_unchanged_copy(source, tmp_path):
    lib = _build(tmp_path, source, "unchanged")
    r = _run_pins(lib, ["-k", "worked_example or insertion_sort or f32_total_order"])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, tmp_path, name, old, new):
    assert source.count(old) == 1, f"mutation site of {name} not found exactly once"
    lib = _build(tmp_path, source.replace(old, new), name)
    r = _run_pins(lib)
    assert r.returncode != 0, f"no pin caught the {name} mutant:\n" + r.stdout[-1500:]
