"""The oracle's pins must reject plausible mistakes.

Each mutant is the oracle built with one deliberate error planted at compile
time (a dropped term, a reversed tie rule, a one-sided fill, ...).  The pins of
``test_oracle.py``, ``test_oracle_methods.py`` and ``test_oracle_graph.py``
are run against it in a subprocess and must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    1: "geodesic-tree parent is the largest-index tight neighbour",
    2: "d_+ drops f(q): w = 2 f(p)",
    3: "extrema ties ordered by decreasing index",
    4: "redundancy fill writes only one orientation of D",
    5: "least-filled ties ignore the extrema rank",
    6: "centroid ties go to the largest index",
    7: "border propagation omits the bottom row",
    8: "multiband weight drops the constant 1",
    9: "extrema method takes the most filled of the farthest points",
    10: "spiral turns drop their left column",
    11: "spiral repulsion removes the pixels on one side of s only",
    12: "graph boundary rule counts degrees equal to the average",
}


@pytest.mark.parametrize("k", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, k):
    sys.path.insert(0, ROOT)
    import oracle
    lib = oracle.build(out=str(tmp_path / f"libmutant{k}.so"), mutant=k)
    env = dict(os.environ, GAPD_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py"),
                        os.path.join(ROOT, "tests", "test_oracle_methods.py"),
                        os.path.join(ROOT, "tests", "test_oracle_graph.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {k} ({MUTANTS[k]}) passed every pin"
