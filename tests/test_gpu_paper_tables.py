"""The paper's printed iteration counts n10 reproduced by the GPU solver.

Tables 5-8 (columns p = 1..7; tests/golden/paper_tables_n10.json): PCG with
the hybrid V-cycle on the cube case of Sec. 5.3 (domain [-1,1]^3,
u = prod sin(3 pi x_j), homogeneous Dirichlet data, Chebyshev(5) smoothing,
the curvilinear cases with the 0.15 amplitude deformation), for every
coarsening strategy, p-sequence, mesh size and penalty factor the tables
list.  The cube's coarse grid has 2^3 elements (Sec. 5.3: 2^d, 3^d or 5^d
coarse-grid elements), so h-coarsening stops at two elements per direction.
The paper's coarse solve is CG + AMG to 1e-3 and ours exact: where the
coarsest level is continuous FE the two agree within 5%; where it is DG, on
which the paper finds AMG weak, the exact solve can only lower n10, so ours
must not exceed the printed value by more than 5%.  Single-level cases are
listed in the file with the reason they are not compared.

The strategies Tables 5 and 6 do not print (hc, hcp, pc, pch): Sec. 5.4.1
states that c-coarsening at the coarsest level or between h- and
p-coarsening leaves the convergence rate of the base method unchanged, so
their n10 must lie within 5% of the range the paper prints for that base
family in the same column (h, hp, hpc for hc and hcp; p, ph, phc for pc and
pch; pc and pch from p = 2, since at p = 1 they start with the c-transfer on
the finest level).

Table 10 (Sec. 5.4.6; tests/golden/paper_table10_n10.json): the cph
solver on the Cartesian 80^3 mesh at p = 3 with n_s = 2..10 smoothing
steps, FP32 V-cycle inside FP64 CG, within 5% of the printed values.
"""
import json
import os

import numpy as np
import pytest

from paper_1910_01900_amd import hmg

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ALL = json.load(open(os.path.join(HERE, "golden", "paper_tables_n10.json")))["cases"]
CASES = [c for c in ALL if c["compare"] != "skip"]
TABLE10 = json.load(open(os.path.join(HERE, "golden", "paper_table10_n10.json")))["cases"]
H_MIN = 2  # the cube's 2^3 coarse grid


def c_variants():
    """hc, hcp (h-like) and pc, pch (p-like) for every subtable and column of
    Tables 5 and 6, each with the printed values of its base family."""
    fam = {"hc": ("h", "hp", "hpc"), "hcp": ("h", "hp", "hpc"), "pc": ("p", "ph", "phc"),
           "pch": ("p", "ph", "phc")}
    rows = {}
    for c in ALL:
        sub = c["cite"].split(",")[0]
        if sub.split("(")[0].strip() in ("Table 5", "Table 6"):
            rows[(sub, c["strategy"], c["k"])] = c
    out = []
    for (sub, strat, k), c in sorted(rows.items()):
        for new, base in fam.items():
            if strat != base[0]:
                continue
            if strat == "p" and k == 1:
                continue  # no p-level: the c-transfer would be on the finest level
            printed = [rows[(sub, b, k)] for b in base if (sub, b, k) in rows]
            printed = [p for p in printed if p["compare"] != "skip"]
            out.append(dict(c, strategy=new, cite="%s, Sec. 5.4.1: %s has the rate of rows %s, column p=%d"
                            % (sub, new, "/".join(base), k),
                            lo=min(p["n10"] for p in printed), hi=max(p["n10"] for p in printed)))
    return out


VARIANTS = c_variants()


def cube_mesh(case):
    N, k = case["N"], case["k"]
    return hmg.Mesh((N, N, N), k, (-1.0,) * 3, (1.0,) * 3, case["curved"], 0.15 if case["curved"] else 0.0, 2,
                    (0,) * 6, case["ip"], None)


def n10_of(case, mg_prec=hmg.F64, n_s=5):
    mesh = cube_mesh(case)
    H = hmg.Hierarchy(mesh, case["strategy"], pseq=case["pseq"], h_min=H_MIN, smoother_degree=n_s, mg_prec=mg_prec)
    b = hmg.Level(mesh).rhs_sine(3 * np.pi)
    _, st = H.solve(b, rtol=1e-10, maxit=600)
    return st["n10"]


@pytest.mark.parametrize("case", CASES, ids=[c["cite"] for c in CASES])
def test_gpu_solver_reproduces_paper_n10(case):
    n10 = n10_of(case)
    print("%s: paper %.1f, ours %.2f" % (case["cite"], case["n10"], n10), flush=True)
    if case["compare"] == "band":
        assert abs(n10 - case["n10"]) <= 0.05 * case["n10"], (n10, case["n10"])
    else:
        assert n10 <= 1.05 * case["n10"], (n10, case["n10"])


def test_c_variants_cover_tables_5_and_6():
    # 2 h-like strategies x 7 columns in 5(a) and 6(a), 2 p-like strategies x
    # columns p = 2..7 in (b)-(d): at p = 1, pc and pch begin with the
    # c-transfer on the finest level, the case the paper treats separately
    assert len(VARIANTS) == 2 * (2 * 7 + 3 * (2 * 6))
    assert {v["strategy"] for v in VARIANTS} == {"hc", "hcp", "pc", "pch"}


@pytest.mark.parametrize("case", VARIANTS, ids=[c["cite"] for c in VARIANTS])
def test_gpu_c_variants_keep_the_base_rate(case):
    n10 = n10_of(case)
    print("%s: paper %.1f..%.1f, ours %.2f" % (case["cite"], case["lo"], case["hi"], n10), flush=True)
    assert 0.95 * case["lo"] <= n10 <= 1.05 * case["hi"], (n10, case["lo"], case["hi"])


@pytest.mark.parametrize("case", TABLE10, ids=[c["cite"] for c in TABLE10])
def test_gpu_table10_smoothing_steps(case):
    n10 = n10_of(case, mg_prec=hmg.F32, n_s=case["n_s"])
    print("%s: paper %.1f, ours %.2f" % (case["cite"], case["n10"], n10), flush=True)
    assert abs(n10 - case["n10"]) <= 0.05 * case["n10"], (n10, case["n10"])
