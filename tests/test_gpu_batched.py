"""GPU parity of the batched operator (several vectors per launch): every
vector's result equals the single-vector launch bit for bit and the oracle's
definition (Sec. 4 operator, Sec. 2 fluxes) within the single-vector bounds.
Covers Cartesian and curvilinear levels, FP64 and FP32, batch sizes that do
and do not fill a workgroup's slots, and ragged meshes."""
import numpy as np
import pytest
import torch

from gpu_helpers import meshes, rel_inf, to_np
from oracle import sipg
from paper_1910_01900_amd import hmg
from paper_1910_01900_amd.inputs import uniform

pytestmark = pytest.mark.gpu


def _batch(L, nrhs, seed0):
    U = L.vectors(nrhs)
    for r in range(nrhs):
        U[r, :L.n_dofs] = torch.as_tensor(uniform(seed0 + r, L.n_dofs), dtype=L.dtype)
    return U


@pytest.mark.parametrize("k,deformed,nrhs", [(1, False, 3), (2, True, 5), (2, True, 64), (3, False, 8),
                                             (4, True, 3), (4, True, 8), (5, False, 2), (5, True, 13),
                                             (6, True, 4), (7, True, 3)])
@pytest.mark.parametrize("prec", [hmg.F64, hmg.F32])
def test_batched_apply_equals_single(k, deformed, nrhs, prec):
    print("batched k=%d deformed=%s nrhs=%d prec=%d" % (k, deformed, nrhs, prec), flush=True)
    hm, om = meshes((5, 3, 2), k, deformed, bc=(0, 1, 0, 0, 1, 0), waves=2, amp=0.08)
    L = hmg.Level(hm, prec=prec)
    U = _batch(L, nrhs, 40)
    V = L.apply_batched(U)
    torch.cuda.synchronize()
    for r in range(nrhs):
        single = L.apply(U[r, :L.n_dofs].contiguous())
        assert torch.equal(V[r, :L.n_dofs], single), r
    # one vector against the oracle at the single-vector bar
    r = nrhs - 1
    ref = sipg.apply(om, k, to_np(U[r, :L.n_dofs])).ravel()
    assert rel_inf(to_np(V[r, :L.n_dofs]), ref) < (1e-12 if prec == hmg.F64 else 1e-5)


@pytest.mark.parametrize("prec", [hmg.F64, hmg.F32])
def test_batched_residual_equals_single(prec):
    hm, _ = meshes((4, 4, 3), 3, True)
    L = hmg.Level(hm, prec=prec)
    U, B = _batch(L, 6, 60), _batch(L, 6, 70)
    Rb = L.residual_batched(B, U)
    torch.cuda.synchronize()
    for r in range(6):
        single = L.residual(B[r, :L.n_dofs].contiguous(), U[r, :L.n_dofs].contiguous())
        assert torch.equal(Rb[r, :L.n_dofs], single), r


def test_batched_apply_full_size_sampled():
    """k=4 on the curvilinear 64^3 mesh, 8 vectors: sampled rows against
    single-vector applies."""
    hm = hmg.Mesh((64, 64, 64), 4, deformed=True, amp=0.05)
    L = hmg.Level(hm, prec=hmg.F32)
    U = _batch(L, 8, 80)
    V = L.apply_batched(U)
    torch.cuda.synchronize()
    for r in (0, 5, 7):
        single = L.apply(U[r, :L.n_dofs].contiguous())
        assert torch.equal(V[r, :L.n_dofs], single), r
