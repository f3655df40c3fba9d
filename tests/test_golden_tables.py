"""Consistency of the transcribed n10 tables (tests/golden/paper_tables_n10.json):
one record per printed value of Tables 5-8 in columns p = 1..7, each cited,
classified by the space of its coarsest level, and agreeing with the values
the oracle is pinned to (tests/golden/paper_n10.json)."""
import collections
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TAB = json.load(open(os.path.join(HERE, "golden", "paper_tables_n10.json")))["cases"]
OLD = json.load(open(os.path.join(HERE, "golden", "paper_n10.json")))["cases"]


def test_every_printed_value_once():
    cites = [c["cite"] for c in TAB]
    assert len(cites) == len(set(cites)) == 427
    per = collections.Counter(c["cite"].split(",")[0] for c in TAB)
    # Tables 5 and 6: 4 subtables x 5 strategies; Table 7: 3 x 3 mesh sizes;
    # Table 8: 3 x 4 penalty factors; 7 columns each
    for t in "56":
        for s in "abcd":
            assert per["Table %s(%s)" % (t, s)] == 35
    for s in "abc":
        assert per["Table 7(%s)" % s] == 21 and per["Table 8(%s)" % s] == 28


def test_classification_follows_the_coarsest_space():
    for c in TAB:
        assert c["compare"] in ("band", "upper", "skip") and c["n10"] > 0
        if c["compare"] == "skip":
            assert c["reason"]
        elif "c" in c["strategy"]:
            assert c["compare"] == "band"
        else:
            assert c["compare"] == "upper"
        if c["strategy"] == "p" and c["k"] == 1:
            assert c["compare"] == "skip"
        else:  # only the single-level cases are not compared
            assert c["compare"] != "skip", c["cite"]


def test_agrees_with_the_oracle_pins():
    tab = {c["cite"]: c for c in TAB}
    for o in OLD:
        t = tab[o["cite"].split(" (")[0]]
        for key in ("n10", "strategy", "pseq", "ip", "N", "k", "curved"):
            assert t[key] == o[key], (o["cite"], key)


def test_coarse_grid_of_the_cube():
    """Sec. 5.3: the cube's coarse grid has 2^d (or 3^d, 5^d) elements, not
    one, so h-coarsening of the 4^3, 8^3 and 16^3 table meshes stops at 2^3
    elements.  On that coarse grid the oracle's curvilinear SIPG matrix (the
    0.15 deformation, cubic mapping, the paper's penalty) is positive
    definite at every degree the tables use, while on the cube as a single
    element it is not (k = 1): a coarse solve of one element could not be
    the paper's."""
    import numpy as np
    from oracle import mesh as om
    from oracle import sipg
    one = om.BoxMesh((1, 1, 1), lo=(-1.0,) * 3, hi=(1.0,) * 3, deform=0.15, waves=2)
    A = sipg.assemble(one, 1)
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    assert np.linalg.eigvalsh(0.5 * (A + A.T))[0] < 0
    two = om.BoxMesh((2, 2, 2), lo=(-1.0,) * 3, hi=(1.0,) * 3, deform=0.15, waves=2)
    for k in range(1, 6):
        A = sipg.assemble(two, k)
        A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
        assert np.linalg.eigvalsh(0.5 * (A + A.T))[0] > 0, k
