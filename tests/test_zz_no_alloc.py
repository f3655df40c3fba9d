"""The operator apply that allocates nothing (hmg_operator_apply_noalloc):
called through the C ABI twice in a row on continuous FE levels, the
second with a smaller input, each result equal bit for bit to
hmg_operator_apply on the same level (both run the same kernels; only the
element-local buffer differs) and within 1e-12 of the oracle's assembled
FE matrix; DG levels; and the size limit, refused before any launch."""
import numpy as np
import pytest
import torch

from gpu_helpers import meshes, rel_inf, to_np
from oracle import fe as ofe
from paper_1910_01900_amd import hmg
from paper_1910_01900_amd.inputs import uniform

pytestmark = pytest.mark.gpu


def _pair(L, seed):
    u = L.vector(uniform(seed, L.n_dofs))
    ref = L.apply(u)
    got = L.apply_noalloc(u, torch.full_like(u, float("nan")))
    torch.cuda.synchronize()
    return u, ref, got


def test_noalloc_fe_twice_second_smaller():
    big_h, big_o = meshes((6, 5, 4), 3, True, bc=(0, 1, 0, 0, 1, 0))
    small_h, small_o = meshes((3, 2, 2), 2, True)
    for (hm, om, k, prec, seed) in ((big_h, big_o, 3, hmg.F64, 90), (small_h, small_o, 2, hmg.F64, 91),
                                    (small_h, small_o, 2, hmg.F32, 92)):
        L = hmg.Level(hm, space=hmg.FE, prec=prec)
        print("noalloc FE k=%d prec=%d nel=%s" % (k, prec, hm.nel), flush=True)
        u, ref, got = _pair(L, seed)
        assert bool((got == ref).all())
        if prec == hmg.F64:
            A = ofe.assemble(om, k)
            assert rel_inf(to_np(got), A @ to_np(u)) < 1e-12


def test_noalloc_dg_equals_apply():
    hm, _ = meshes((3, 3, 2), 4, True)
    L = hmg.Level(hm)
    _, ref, got = _pair(L, 93)
    assert bool((got == ref).all())


def test_noalloc_refuses_levels_beyond_the_static_buffer():
    # FE degree 7 on 26^3 Cartesian elements: 17,576 x 512 x 8 B = 72 MB > 64 MiB
    hm = hmg.Mesh((26, 26, 26), 7)
    L = hmg.Level(hm, space=hmg.FE)
    u = L.vector()
    v = torch.full_like(u, 3.0)
    with pytest.raises(hmg.HmgError) as ei:
        L.apply_noalloc(u, v)
    assert ei.value.code == -2
    assert bool((v == 3.0).all())
    # the same level through the workspace path still works
    L.apply(L.vector(np.ones(L.n_dofs)), v)
    assert bool(torch.isfinite(v).all())
