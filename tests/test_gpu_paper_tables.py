"""The paper's printed iteration counts n10 (Tables 5-8, columns p = 1..7;
tests/golden/paper_tables_n10.json) reproduced by the GPU solver: PCG with
the hybrid V-cycle on the cube case of Sec. 5.3 (domain [-1,1]^3,
u = prod sin(3 pi x_j), homogeneous Dirichlet data, Chebyshev(5) smoothing,
the curvilinear cases with the 0.15 amplitude deformation), for every
coarsening strategy, p-sequence, mesh size and penalty factor the tables
list.  The paper's coarse solve is CG + AMG to 1e-3 and ours exact (Jacobi-
PCG to 1e-3 above 8192 unknowns): where the coarsest level is continuous
FE the two agree within 5%; where it is DG, on which the paper finds AMG
weak, the exact solve can only lower n10, so ours must not exceed the
printed value by more than 5%.  Cases that cannot be compared are listed in
the file with the reason."""
import json
import os

import numpy as np
import pytest

from paper_1910_01900_amd import hmg

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = [c for c in json.load(open(os.path.join(HERE, "golden", "paper_tables_n10.json")))["cases"]
         if c["compare"] != "skip"]


@pytest.mark.parametrize("case", CASES, ids=[c["cite"] for c in CASES])
def test_gpu_solver_reproduces_paper_n10(case):
    N, k = case["N"], case["k"]
    mesh = hmg.Mesh((N, N, N), k, (-1.0,) * 3, (1.0,) * 3, case["curved"], 0.15 if case["curved"] else 0.0, 2,
                    (0,) * 6, case["ip"], None)
    H = hmg.Hierarchy(mesh, case["strategy"], pseq=case["pseq"], h_min=1, smoother_degree=5, mg_prec=hmg.F64)
    b = hmg.Level(mesh).rhs_sine(3 * np.pi)
    _, st = H.solve(b, rtol=1e-10, maxit=600)
    print("%s: paper %.1f, ours %.2f" % (case["cite"], case["n10"], st["n10"]), flush=True)
    if case["compare"] == "band":
        assert abs(st["n10"] - case["n10"]) <= 0.05 * case["n10"], (st["n10"], case["n10"])
    else:
        assert st["n10"] <= 1.05 * case["n10"], (st["n10"], case["n10"])
