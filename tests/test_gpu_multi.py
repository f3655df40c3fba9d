"""GPU parity of the multi-mesh batch (many DG meshes of uneven size and
degree, several vectors each, under one launch schedule): every mesh's and
vector's result equals the single-mesh launch bit for bit, under every
schedule (one launch per degree group or one launch for all Cartesian meshes,
one workgroup per tile or persistent workgroups with 1, 2 or 4 chunks per
tile), and the oracle's operator (Sec. 4, Sec. 2 fluxes) within the
single-mesh bounds.  Residual and Chebyshev (Alg. 3) launches likewise; the
autotuner's choice changes no result."""
import numpy as np
import pytest
import torch

from gpu_helpers import meshes, rel_inf, to_np
from oracle import sipg
from paper_1910_01900_amd import hmg
from paper_1910_01900_amd.inputs import multi_meshes, uniform

pytestmark = pytest.mark.gpu

# (nel, k, deformed): ragged sizes, every degree, both geometry kinds
MIXED = [((3, 2, 2), 1, False), ((4, 3, 5), 2, False), ((2, 2, 2), 3, True), ((3, 3, 2), 4, False),
         ((2, 3, 2), 5, True), ((2, 2, 2), 7, False), ((5, 4, 3), 2, False), ((1, 1, 1), 6, False),
         ((3, 1, 2), 6, True), ((2, 2, 3), 3, False), ((2, 3, 3), 4, True), ((2, 1, 3), 7, True)]
CARTESIAN = [m for m in MIXED if not m[2]]
SENTINEL = 7.0


def _levels(spec, prec):
    out = []
    for nel, k, deformed in spec:
        hm, om = meshes(nel, k, deformed, bc=(0, 1, 0, 0, 1, 0), amp=0.08, waves=2)
        out.append((hmg.Level(hm, prec=prec), om, k))
    return out


def _fill(B, seed0):
    """Packed vector: U[-1,1) in every vector, SENTINEL in the padding."""
    v = torch.full((B.total,), SENTINEL, dtype=B.dtype, device="cuda")
    for i, L in enumerate(B.levels):
        for r in range(B.nrhs):
            B.view(v, i, r).copy_(torch.as_tensor(uniform(seed0 + 17 * i + r, L.n_dofs), dtype=B.dtype))
    return v


def _padding_untouched(B, v):
    for i, L in enumerate(B.levels):
        for r in range(B.nrhs):
            o = B.offset[i] + r * B.ld[i]
            pad = v[o + L.n_dofs:o + B.ld[i]]
            if pad.numel():
                assert bool((pad == SENTINEL).all()), (i, r)


def _check_equal_single(B, U, V):
    torch.cuda.synchronize()
    for i, L in enumerate(B.levels):
        for r in range(B.nrhs):
            single = L.apply(B.view(U, i, r).contiguous())
            assert torch.equal(B.view(V, i, r), single), (i, r)


SCHEDULES = [dict(single=False, persistent=False, chunks_per_tile=1, blocks_per_cu=1),
             dict(single=False, persistent=True, chunks_per_tile=1, blocks_per_cu=1),
             dict(single=False, persistent=True, chunks_per_tile=2, blocks_per_cu=2),
             dict(single=False, persistent=True, chunks_per_tile=4, blocks_per_cu=1)]


@pytest.mark.parametrize("prec", [hmg.F64, hmg.F32])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_batch_apply_equals_single_every_schedule(prec, nrhs):
    print("batch apply prec=%d nrhs=%d" % (prec, nrhs), flush=True)
    lv = _levels(MIXED, prec)
    B = hmg.Batch([L for L, _, _ in lv], nrhs)
    U = _fill(B, 300)
    for sch in SCHEDULES:
        print("  schedule", sch, flush=True)
        B.set_schedule(**sch)
        V = torch.full((B.total,), SENTINEL, dtype=B.dtype, device="cuda")
        B.apply(U, V)
        _check_equal_single(B, U, V)
        _padding_untouched(B, V)
    # two meshes against the oracle at the single-mesh bar
    for i in (2, 5):
        L, om, k = lv[i]
        ref = sipg.apply(om, k, to_np(B.view(U, i, nrhs - 1))).ravel()
        assert rel_inf(to_np(B.view(V, i, nrhs - 1)), ref) < (1e-12 if prec == hmg.F64 else 1e-5)


@pytest.mark.parametrize("prec", [hmg.F64, hmg.F32])
def test_single_launch_cartesian(prec):
    print("single launch prec=%d" % prec, flush=True)
    lv = _levels(CARTESIAN, prec)
    B = hmg.Batch([L for L, _, _ in lv], 2)
    U = _fill(B, 500)
    for persistent, q, bpc in ((False, 1, 1), (True, 1, 1), (True, 4, 2)):
        B.set_schedule(single=True, persistent=persistent, chunks_per_tile=q, blocks_per_cu=bpc)
        assert B.schedule()["single"]
        V = torch.full((B.total,), SENTINEL, dtype=B.dtype, device="cuda")
        B.apply(U, V)
        _check_equal_single(B, U, V)
        _padding_untouched(B, V)


def test_single_launch_rejects_curved():
    lv = _levels(MIXED[:3], hmg.F64)
    B = hmg.Batch([L for L, _, _ in lv], 1)
    with pytest.raises(hmg.HmgError) as e:
        B.set_schedule(single=True)
    assert e.value.code == -2
    with pytest.raises(hmg.HmgError):
        B.set_schedule(persistent=False, chunks_per_tile=2)


def test_many_tiny_meshes():
    """40 one- and two-element meshes: tiles of many meshes share every XCD range."""
    spec = [((1 + (i % 2), 1, 1), 1 + (i % 7), False) for i in range(40)]
    lv = _levels(spec, hmg.F64)
    B = hmg.Batch([L for L, _, _ in lv], 2)
    U = _fill(B, 700)
    for sch in SCHEDULES + [dict(single=True, persistent=False, chunks_per_tile=1, blocks_per_cu=1)]:
        B.set_schedule(**sch)
        V = B.apply(U)
        _check_equal_single(B, U, V)


@pytest.mark.parametrize("prec", [hmg.F64, hmg.F32])
def test_batch_residual_and_chebyshev_equal_single(prec):
    print("batch residual/chebyshev prec=%d" % prec, flush=True)
    lv = _levels(MIXED, prec)
    levels = [L for L, _, _ in lv]
    B = hmg.Batch(levels, 2)
    U, Bv = _fill(B, 900), _fill(B, 950)
    B.set_schedule(persistent=True, chunks_per_tile=2, blocks_per_cu=1)
    R = B.residual(Bv, U)
    torch.cuda.synchronize()
    for i, L in enumerate(levels):
        for r in range(2):
            single = L.residual(B.view(Bv, i, r).contiguous(), B.view(U, i, r).contiguous())
            assert torch.equal(B.view(R, i, r), single), (i, r)
    lmax = [L.lambda_max() for L in levels]
    for degree in (3, 4):
        B.set_chebyshev(lmax, degree)
        X = U.clone()
        B.chebyshev(Bv, X)
        torch.cuda.synchronize()
        for i, L in enumerate(levels):
            for r in range(2):
                x = B.view(U, i, r).contiguous()
                L.chebyshev(B.view(Bv, i, r).contiguous(), x, degree, lmax[i])
                assert torch.equal(B.view(X, i, r), x), (degree, i, r)


def test_autotune_keeps_results():
    lv = _levels(MIXED, hmg.F64)
    B = hmg.Batch([L for L, _, _ in lv], 3)
    U = _fill(B, 1100)
    V0 = B.apply(U)
    ms = B.autotune(U, B.vector(), reps=3)
    assert ms > 0
    s = B.schedule()
    assert not s["single"] and len(s["units"]) == len({(d, k) for _, k, d in MIXED})
    for u in s["units"]:
        assert u["ms"] > 0 and u["grid"] % 8 == 0 and u["chunks_per_tile"] in (1, 2, 4)
    V1 = B.apply(U)
    torch.cuda.synchronize()
    assert torch.equal(V0, V1)
    # Cartesian only: the single launch is a candidate too
    lc = _levels(CARTESIAN, hmg.F32)
    Bc = hmg.Batch([L for L, _, _ in lc], 2)
    Uc = _fill(Bc, 1200)
    W0 = Bc.apply(Uc)
    Bc.autotune(Uc, Bc.vector(), reps=3)
    W1 = Bc.apply(Uc)
    torch.cuda.synchronize()
    assert torch.equal(W0, W1)


def test_multi_workload_sampled():
    """The 64-mesh benchmark batch (unit cubes N ~ U{4..24}, k ~ U{2..7}),
    4 vectors, FP64, autotuned: sampled meshes against single applies."""
    spec = multi_meshes()
    levels = [hmg.Level(hmg.Mesh((N, N, N), k), prec=hmg.F64) for N, k in spec]
    B = hmg.Batch(levels, 4)
    U = B.vector()
    g = torch.Generator(device="cuda").manual_seed(5)
    U.uniform_(-1, 1, generator=g)
    B.autotune(U, B.vector(), reps=2)
    V = B.apply(U)
    torch.cuda.synchronize()
    for i in (0, 3, 17, 40, 63):
        for r in (0, 3):
            single = levels[i].apply(B.view(U, i, r).contiguous())
            assert torch.equal(B.view(V, i, r), single), (i, r)


def test_batch_max_vectors_tiny_meshes():
    """nrhs = 64 (the limit) on one-element and ragged meshes of several degrees."""
    spec = [((1, 1, 1), 2, False), ((2, 1, 3), 4, False), ((1, 2, 1), 3, True), ((3, 1, 1), 7, False)]
    lv = _levels(spec, hmg.F32)
    B = hmg.Batch([L for L, _, _ in lv], 64)
    U = _fill(B, 1300)
    for sch in (SCHEDULES[0], SCHEDULES[3]):
        B.set_schedule(**sch)
        V = torch.full((B.total,), SENTINEL, dtype=B.dtype, device="cuda")
        B.apply(U, V)
        _check_equal_single(B, U, V)
        _padding_untouched(B, V)
