"""Graph-recorded solves (hmg_hierarchy_set_graph): PCG iterations and
V-cycles replayed from HIP graphs give bitwise the eager results, over
several replays with eager work and synchronisations between them, after a
change of the solution vector (new recording) and for both precisions of
the V-cycle."""
import numpy as np
import pytest
import torch

from paper_1910_01900_amd import hmg
from paper_1910_01900_amd.inputs import uniform

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mg_prec", [hmg.F64, hmg.F32])
@pytest.mark.parametrize("k,deformed", [(3, False), (4, True)])
def test_graph_solve_bitwise_equals_eager(mg_prec, k, deformed):
    print("graph solve k=%d deformed=%s prec=%d" % (k, deformed, mg_prec), flush=True)
    mesh = hmg.Mesh((8, 8, 8), k, deformed=deformed, amp=0.05)
    He = hmg.Hierarchy(mesh, "cph", h_min=2, mg_prec=mg_prec)
    Hg = hmg.Hierarchy(mesh, "cph", h_min=2, mg_prec=mg_prec, graph=True)
    b = torch.as_tensor(uniform(3, He.n_dofs), device="cuda")
    xe, ste = He.solve(b, rtol=1e-10)
    x1 = torch.zeros_like(b)
    x2 = torch.zeros_like(b)
    for rep in range(3):  # replays of one recording, eager work in between
        x1.zero_()
        _, st = Hg.solve(b, x1, rtol=1e-10)
        torch.cuda.synchronize()
        assert st["iters"] == ste["iters"] and st["rn"] == ste["rn"], (rep, st, ste)
        assert torch.equal(x1, xe), rep
        _ = (b * 2.0).sum().item()
    _, st = Hg.solve(b, x2, rtol=1e-10)  # another x: recorded again
    assert torch.equal(x2, xe)


def test_graph_vcycle_bitwise_equals_eager():
    """One recording replayed on new data in the same buffers."""
    mesh = hmg.Mesh((8, 8, 8), 3, deformed=True, amp=0.05)
    He = hmg.Hierarchy(mesh, "cph", h_min=2, mg_prec=hmg.F32)
    Hg = hmg.Hierarchy(mesh, "cph", h_min=2, mg_prec=hmg.F32, graph=True)
    rbuf = torch.zeros(He.n_dofs, dtype=torch.float64, device="cuda")
    zbuf = torch.zeros_like(rbuf)
    for seed in (4, 5, 4, 6):
        rbuf.copy_(torch.as_tensor(uniform(seed, He.n_dofs), device="cuda"))
        ze = He.vcycle(rbuf.clone())
        Hg.vcycle(rbuf, zbuf)
        torch.cuda.synchronize()
        assert torch.equal(zbuf, ze), seed
