"""The oracle's pins catch plausible mistakes: each test plants one slip in a
copy of oracle.cpp (on the CPU), builds it, and runs the pin suites of
test_oracle_sfc.py and test_oracle_index.py against it; they must fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")

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
]


@pytest.mark.parametrize("what,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_a_planted_mistake(tmp_path, what, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, what
    mut = tmp_path / "oracle_mutant.cpp"
    mut.write_text(src.replace(old, new, 1))
    so = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", str(so), str(mut)])
    env = dict(os.environ, PSI_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_sfc.py"),
                        os.path.join(ROOT, "tests", "test_oracle_index.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught: {what}"
