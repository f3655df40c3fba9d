"""GPU parity of the multigrid components (Sec. 3: transfers, Chebyshev,
V-cycle of Alg. 2, PCG of Alg. 1) against the oracle, plus the documented
failure paths of the solver."""
import numpy as np
import pytest

from gpu_helpers import meshes, rel_inf, to_np
from oracle import fe as ofe
from oracle import sipg, solver, transfer
from paper_1910_01900_amd import hmg
from paper_1910_01900_amd.inputs import uniform

pytestmark = pytest.mark.gpu


def _transfer_case(kind, space, kf, kc, nel_f, nel_c, deformed, prec=hmg.F64):
    hf, of = meshes(nel_f, kf, deformed, bc=(0, 1, 0, 0, 1, 0))
    hc, oc = meshes(nel_c, kc, deformed, bc=(0, 1, 0, 0, 1, 0))
    if kind == "c":
        F, Cl = hmg.Level(hf, prec=prec), hmg.Level(hc, space=hmg.FE, prec=prec)
        P = transfer.c_prolongation(of, kf)
    else:
        F, Cl = hmg.Level(hf, space=space, prec=prec), hmg.Level(hc, space=space, prec=prec)
        if kind == "p":
            P = transfer.dg_p(of, kf, kc) if space == hmg.DG else transfer.fe_p(of, kf, kc)
        else:
            P = transfer.dg_h(of, kf) if space == hmg.DG else transfer.fe_h(of, kf)
    return F, Cl, hmg.Transfer(F, Cl, kind), P


@pytest.mark.parametrize("kind,space,kf,kc,nel_f,nel_c", [
    ("p", hmg.DG, 4, 2, (3, 2, 3), (3, 2, 3)),
    ("p", hmg.DG, 7, 3, (2, 2, 3), (2, 2, 3)),
    ("h", hmg.DG, 3, 3, (4, 2, 6), (2, 1, 3)),
    ("c", None, 3, 3, (3, 2, 3), (3, 2, 3)),
    ("p", hmg.FE, 4, 2, (3, 2, 3), (3, 2, 3)),
    ("p", hmg.FE, 2, 1, (3, 2, 3), (3, 2, 3)),
    ("h", hmg.FE, 1, 1, (4, 2, 6), (2, 1, 3)),
    ("h", hmg.FE, 2, 2, (4, 4, 2), (2, 2, 1)),
])
def test_transfers_match_oracle(kind, space, kf, kc, nel_f, nel_c):
    F, Cl, T, P = _transfer_case(kind, space, kf, kc, nel_f, nel_c, True)
    c = uniform(20, Cl.n_dofs)
    f0 = uniform(21, F.n_dofs)
    f = F.vector(f0)
    T.prolongate_add(Cl.vector(c), f)
    assert rel_inf(to_np(f), f0 + P @ c) < 1e-13
    r = uniform(22, F.n_dofs)
    assert rel_inf(to_np(T.restrict(F.vector(r))), P.T @ r) < 1e-13


# node-count pairs outside the hierarchies' p-sequences (k -> k-1, floor(k/2),
# 1): the transfer kernel with run-time node counts
@pytest.mark.parametrize("kind,space,kf,kc,nel_f", [
    ("p", hmg.DG, 7, 2, (3, 2, 3)),
    ("p", hmg.DG, 5, 3, (2, 3, 2)),
    ("p", hmg.DG, 7, 4, (2, 2, 3)),
    ("p", hmg.FE, 6, 4, (2, 3, 2)),
])
def test_transfers_other_degree_pairs_match_oracle(kind, space, kf, kc, nel_f):
    F, Cl, T, P = _transfer_case(kind, space, kf, kc, nel_f, nel_f, True)
    c = uniform(23, Cl.n_dofs)
    f0 = uniform(24, F.n_dofs)
    f = F.vector(f0)
    T.prolongate_add(Cl.vector(c), f)
    assert rel_inf(to_np(f), f0 + P @ c) < 1e-13
    r = uniform(25, F.n_dofs)
    assert rel_inf(to_np(T.restrict(F.vector(r))), P.T @ r) < 1e-13


@pytest.mark.parametrize("kind,space,kf,kc,nel_f,nel_c", [
    ("p", hmg.DG, 7, 3, (2, 2, 3), (2, 2, 3)),
    ("h", hmg.DG, 5, 5, (4, 2, 2), (2, 1, 1)),
    ("p", hmg.DG, 6, 3, (2, 2, 3), (2, 2, 3)),
    ("p", hmg.FE, 4, 2, (3, 2, 3), (3, 2, 3)),
    ("p", hmg.DG, 7, 2, (3, 2, 3), (3, 2, 3)),
])
def test_transfers_fp32_match_oracle(kind, space, kf, kc, nel_f, nel_c):
    # FP32 data and FP32-rounded 1-D matrices; sums of at most n^3 products
    F, Cl, T, P = _transfer_case(kind, space, kf, kc, nel_f, nel_c, True, prec=hmg.F32)
    c = uniform(26, Cl.n_dofs)
    f0 = uniform(27, F.n_dofs)
    f = F.vector(f0)
    T.prolongate_add(Cl.vector(c), f)
    ref = f0.astype(np.float32).astype(np.float64) + P @ c.astype(np.float32).astype(np.float64)
    assert rel_inf(to_np(f), ref) < 2e-6
    r = uniform(28, F.n_dofs).astype(np.float32).astype(np.float64)
    assert rel_inf(to_np(T.restrict(F.vector(r))), P.T @ r) < 2e-6


def _oracle_hierarchy(om, k, strategy, pseq, h_min, H):
    lv = H.levels()
    oh = solver.Hierarchy(om, k, strategy, pseq=pseq, h_min=h_min, lmax=[l["lmax"] for l in lv[:-1]])
    spec = [(l["space"], l["k"], l["mesh"].nel) for l in oh.levels]
    assert spec == [(l["space"], l["degree"], l["nel"]) for l in lv]
    return oh


@pytest.mark.parametrize("strategy,k,nel,deformed", [
    ("cph", 3, (4, 4, 4), True),
    ("p", 4, (3, 2, 3), False),
    ("ph", 2, (4, 4, 2), True),
    ("hpc", 3, (4, 4, 4), False),
])
def test_vcycle_matches_oracle(strategy, k, nel, deformed):
    hm, om = meshes(nel, k, deformed, bc=(0, 0, 0, 1, 0, 0))
    H = hmg.Hierarchy(hm, strategy, pseq=1, h_min=1)
    oh = _oracle_hierarchy(om, k, strategy, 1, 1, H)
    # the GPU lambda_max estimates agree with the oracle's (same start vectors)
    for l, lev in enumerate(H.levels()[:-1]):
        from oracle import rng
        A = oh.levels[l]["A"]
        ref = solver.lanczos_lmax(A, oh.levels[l]["dinv"], rng.uniform_pm1(1 + l, A.shape[0]))
        assert abs(lev["lmax"] - ref) <= 1e-8 * ref
    b = uniform(30, H.n_dofs)
    import torch
    x = to_np(H.vcycle(torch.as_tensor(b, device="cuda")))
    err = rel_inf(x, oh.vcycle(b))
    # one V-cycle is a fixed sequence of operator applies, transfers and the
    # coarse solve, each within 1e-12 of the oracle's (measured 2e-15 to 8e-15)
    print("vcycle %s k=%d: rel err %.3e" % (strategy, k, err))
    assert err < 1e-12


def test_vcycle_fp32_close_to_fp64():
    import torch
    k = 3
    hm, om = meshes((4, 4, 4), k, True)
    H64 = hmg.Hierarchy(hm, "cph", h_min=1)
    H32 = hmg.Hierarchy(hm, "cph", h_min=1, mg_prec=hmg.F32)
    b = torch.as_tensor(uniform(31, H64.n_dofs), device="cuda")
    x64, x32 = to_np(H64.vcycle(b)), to_np(H32.vcycle(b))
    assert rel_inf(x32, x64) < 1e-4


def test_pcg_cube_k3_8_reaches_tolerance():
    """The Cartesian 8^3, k = 3 workload: p-multigrid (3 -> 1), Chebyshev(5),
    exact coarse solve; the final residual is recomputed with the oracle's
    assembled matrix."""
    import torch
    k = 3
    hm, om = meshes((8, 8, 8), k, False)
    H = hmg.Hierarchy(hm, "p", pseq=1)
    L = hmg.Level(hm)
    b = L.rhs_sine(2 * np.pi)
    x, st = H.solve(b, rtol=1e-10)
    A = sipg.assemble(om, k)
    bn = to_np(b)
    res = np.linalg.norm(bn - A @ to_np(x)) / np.linalg.norm(bn)
    print("cube_k3_8:", st, "oracle residual", res)
    assert res <= 1.05e-10
    oh = solver.Hierarchy(om, k, "p", pseq=1, lmax=[l["lmax"] for l in H.levels()[:-1]])
    _, hist = solver.pcg(A, bn, precond=oh.vcycle, rtol=1e-10)
    assert abs(st["iters"] - (len(hist) - 1)) <= 1
    # discretization error of the solve against the manufactured solution
    u = lambda X: np.prod(np.sin(2 * np.pi * X), axis=-1)
    assert sipg.l2_error(om, k, to_np(x), u) < 2e-3


@pytest.mark.parametrize("mg_prec", [hmg.F64, hmg.F32])
def test_pcg_curved_cph(mg_prec):
    import torch
    k = 4
    hm, om = meshes((8, 8, 8), k, True)
    H = hmg.Hierarchy(hm, "cph", pseq=1, mg_prec=mg_prec)
    b = torch.as_tensor(uniform(32, H.n_dofs), device="cuda")
    x, st = H.solve(b, rtol=1e-10)
    bn = to_np(b)
    res = np.linalg.norm(bn - sipg.apply(om, k, to_np(x)).ravel()) / np.linalg.norm(bn)
    print("curved cph", mg_prec, st, res)
    assert res <= 1.05e-10
    assert st["iters"] <= 12


def test_pcg_failure_paths():
    import torch
    hm, _ = meshes((4, 4, 4), 2, False)
    H = hmg.Hierarchy(hm, "cph", h_min=1)
    b = torch.as_tensor(uniform(33, H.n_dofs), device="cuda")
    _, st = H.solve(b, maxit=1, allow_not_converged=True)
    assert st["status"] == "HMG_NOT_CONVERGED" and st["iters"] == 1
    bad = b.clone()
    bad[5] = float("nan")
    with pytest.raises(hmg.HmgError) as ei:
        H.solve(bad)
    assert ei.value.code == -5
    # warm start from a converged solution: zero iterations
    x, st = H.solve(b)
    x2, st2 = H.solve(b, x=x.clone(), rtol=1e-6)
    assert st2["iters"] == 0 or st2["rn"] / st2["r0"] <= 1e-6
    # a misaligned vector of the right length is rejected by the library
    buf = torch.zeros(H.n_dofs + 32, dtype=torch.float64, device="cuda")
    with pytest.raises(hmg.HmgError) as ei:
        H.vcycle(buf[1:1 + H.n_dofs])
    assert ei.value.code in (-1,)


def test_binding_rejects_wrong_vectors_before_any_launch():
    """The binding checks precision and length against the handle before
    calling the library, whose kernels trust the pointers: an FP32 vector
    for an FP64 solve, a vector shorter than the level, a wrongly shaped
    batch."""
    import torch
    hm, _ = meshes((4, 4, 4), 2, False)
    H = hmg.Hierarchy(hm, "cph", h_min=1)
    L = hmg.Level(hm, prec=hmg.F32)
    b = torch.as_tensor(uniform(34, H.n_dofs), device="cuda")
    x = torch.full_like(b, 7.0)
    with pytest.raises(ValueError):
        H.solve(b.float())
    with pytest.raises(ValueError):
        H.solve(b, x=x[:-1])
    with pytest.raises(ValueError):
        H.vcycle(b[: H.n_dofs // 2], x)
    assert bool((x == 7.0).all())  # nothing ran
    u32 = L.vector(uniform(35, L.n_dofs))
    with pytest.raises(ValueError):
        L.apply(u32.double())
    with pytest.raises(ValueError):
        L.apply(u32, torch.zeros(L.n_dofs - 1, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        L.residual(u32, u32, torch.zeros(L.n_dofs, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        L.apply_batched(L.vectors(2).double())
    with pytest.raises(ValueError):
        L.chebyshev(u32[:10], L.vector(), 2, 1.5)
    with pytest.raises(ValueError):
        H.coarse_solve_batch(torch.zeros(2, H.coarse_info()["n"] + 1, dtype=torch.float64, device="cuda"))


def test_pcg_with_exact_mapping():
    """PCG + cph V-cycle on the exactly mapped curvilinear mesh (mapping
    degree 0 on every level): the final residual recomputed with the
    oracle's operator of the same geometry."""
    import torch
    k = 3
    hm, om = meshes((4, 4, 4), k, True, amp=0.08, waves=2, mapping=0)
    H = hmg.Hierarchy(hm, "cph", pseq=1, h_min=1, mg_prec=hmg.F32)
    b = torch.as_tensor(uniform(36, H.n_dofs), device="cuda")
    x, st = H.solve(b, rtol=1e-10)
    bn = to_np(b)
    res = np.linalg.norm(bn - sipg.apply(om, k, to_np(x)).ravel()) / np.linalg.norm(bn)
    print("exact mapping cph:", st, res)
    assert res <= 1.05e-10
