"""The oracle's pins catch plausible mistakes: each test plants one slip in a
copy of oracle.cpp (on the CPU), builds it, and runs the pin suites of
test_oracle_sfc.py and test_oracle_index.py against it; they must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")

# (what, text to replace, replacement, anchor): the first occurrence of the
# text after the anchor (the start of the file when the anchor is empty) is
# replaced, so a slip lands inside the function it names.
MUTANTS = [
    ("Morton axes swapped inside a bit group", "<< (dim * b + d);", "<< (dim * b + (dim - 1 - d));"),
    ("Hilbert without the Gray-code step", "for (int i = 1; i < dim; ++i) X[i] ^= X[i - 1];",
     "for (int i = 1; i < dim; ++i) X[i] ^= 0u;"),
    ("pairs with equal keys in descending id order", "(a.key == b.key && a.id < b.id)",
     "(a.key == b.key && a.id > b.id)"),
    ("kNN ties not broken by id", "else if (k > 0 && c < best.top()) { best.pop(); best.push(c); }\n        }\n        std::vector",
     "else if (k > 0 && c.first < best.top().first) { best.pop(); best.push(c); }\n        }\n        std::vector"),
    ("range boxes open at the low end", "if (p[d] < box[d] || p[d] > box[D + d]) return false;",
     "if (p[d] <= box[d] || p[d] > box[D + d]) return false;"),
    ("greedy leaves of phi instead of balanced chunks", "return j * n / L;",
     "return j * ((n + L - 1) / L) < n ? j * ((n + L - 1) / L) : n;"),
    # (comparing the new candidate by distance alone is no slip here: the scan
    # runs in id order, so a later candidate never wins a tie anyway)
    ("raw-point kNN heap ordered by distance alone",
     "std::priority_queue<std::pair<uint64_t, uint32_t>> best;",
     "auto by_d = [](const std::pair<uint64_t, uint32_t>& a, const std::pair<uint64_t, uint32_t>& b) "
     "{ return a.first < b.first; };\n"
     "        std::priority_queue<std::pair<uint64_t, uint32_t>, std::vector<std::pair<uint64_t, uint32_t>>, "
     "decltype(by_d)> best(by_d);", "void ora_knn_points("),
    ("raw-point kNN ids off by one", "(uint32_t)i};", "(uint32_t)(i + 1)};", "void ora_knn_points("),
    ("raw-point range count never counts point 0", "for (uint64_t i = 0; i < n; ++i) c += in_box",
     "for (uint64_t i = 1; i < n; ++i) c += in_box", "void ora_range_count_points("),
    ("raw-point range count with the box rows swapped", "c += in_box(dim, pts + i * dim, boxes + b * 2 * dim);",
     "c += in_box(dim, pts + i * dim, boxes + b * 2 * dim + (b & 1) * dim);", "void ora_range_count_points("),
]


def _plant(src, old, new, anchor):
    at = src.index(anchor) if anchor else 0
    i = src.index(old, at)
    return src[:i] + new + src[i + len(old):]


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_a_planted_mistake(tmp_path, mutant):
    what, old, new = mutant[:3]
    anchor = mutant[3] if len(mutant) > 3 else ""
    src = open(SRC).read()
    assert src.count(old) >= 1, what
    mut = tmp_path / "oracle_mutant.cpp"
    planted = _plant(src, old, new, anchor)
    assert planted != src, what
    mut.write_text(planted)
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", str(so), str(mut)])
    env = dict(os.environ, PSI_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_sfc.py"),
                        os.path.join(ROOT, "tests", "test_oracle_index.py"),
                        os.path.join(ROOT, "tests", "test_oracle_points.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught: {what}"
