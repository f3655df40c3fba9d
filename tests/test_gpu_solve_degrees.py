"""GPU parity at the degrees of the large workloads (k = 4 on 64^3, k = 5 and
k = 7 on 48^3): componentwise bounds of the operator, the residual and Chebyshev
epilogues fused into the operator kernel (Alg. 2 residual, Alg. 3 update,
including the variant that keeps the input in LDS), in FP64 and FP32, on
curvilinear meshes with per-element penalty scales, against the oracle's
assembled SIPG matrix; and the mixed-precision solve of the k = 7 workload
at reduced size against the oracle's PCG.

Bounds (per result i; u the input, A the oracle matrix, |A| its entrywise
absolute value, eps32 = 2^-24):
  * FP64 operator: |y_i - (A u)_i| <= 1e-12 (|A||u|)_i.
  * FP32 operator (inputs rounded to FP32 first): |y_i - (A u)_i| <=
    16 (k+1) Lambda_n eps32 (|A||u|)_i.  Each result is a sum over at most 7
    n-point sweep chains of about 4 n rounded operations (16 n), and the
    curvilinear kernels evaluate an element's own face traces by
    extrapolating its Gauss-point values to the element end (and inject the
    face test functions back the same way): rounding errors of those values
    enter the face terms multiplied by up to Lambda_n = sum_q |l_q(0)|, the
    Gauss-point Lagrange basis at the end point (3.32 at n = 5, 4.51 at
    n = 8).  |A||u| does not see this factor, which belongs to the
    factorized evaluation, not to the matrix.
  * residual r = b - A u: the operator's bound plus one rounding of b:
    |r_i - (b - A u)_i| <= c (|A||u|)_i + eps |b_i| (c as above).
  * one fused Chebyshev step x' = x + sigma (x - x_old) + theta D^{-1}(b - A x):
    the residual bound scaled by |theta D^{-1}_i| plus the rounding of the
    update, c_u eps (|x_i| + |sigma| |x_i - x_old_i| + |theta D^{-1}_i (b - A x)_i|)
    with c_u = 4, plus c |theta D^{-1}_i (b - A x)_i| for the inverse diagonal
    (computed on the host by sum factorization, not from the assembled matrix).
"""
import functools

import numpy as np
import pytest

from gpu_helpers import fp32_bound, meshes, rel_inf, to_np
from oracle import sipg, solver
from paper_1910_01900_amd import hmg
from paper_1910_01900_amd.inputs import tau_scale, uniform

pytestmark = pytest.mark.gpu

# curvilinear meshes with penalty scales U[1, 10] and mixed boundary
# conditions; k = 4: 12 elements (1.5 workgroups of 8), k = 5: 18 elements
# in x-rows of 9 (workgroups of 7 elements: a full and a 2-element chunk
# per row), k = 7: 8 elements (2 workgroups of 4)
CASES = {4: (3, 2, 2), 5: (9, 2, 1), 7: (2, 2, 2)}
EPS32 = 2.0 ** -24


@functools.lru_cache(maxsize=None)
def oracle_case(k, bc=(0, 1, 0, 0, 1, 0)):
    nel = CASES[k]
    ts = tau_scale(5, int(np.prod(nel)))
    hm, om = meshes(nel, k, True, bc=bc, tau_scale=ts)
    A = sipg.assemble(om, k).tocsr()
    return hm, om, A, abs(A)


def _inputs(L, prec, *seeds):
    vals = [uniform(s, L.n_dofs) for s in seeds]
    if prec == hmg.F32:
        vals = [v.astype(np.float32).astype(np.float64) for v in vals]
    return vals


def lebesgue_end(n):
    """sum_q |l_q(0)| for the Lagrange basis on the n Gauss points of [0,1]."""
    z = (np.polynomial.legendre.leggauss(n)[0] + 1) / 2
    return sum(abs(np.prod([(0 - z[m]) / (z[q] - z[m]) for m in range(n) if m != q])) for q in range(n))


def _c(k, prec):
    return 1e-12 if prec == hmg.F64 else fp32_bound(k) * lebesgue_end(k + 1)


@pytest.mark.parametrize("k", [4, 5, 7])
@pytest.mark.parametrize("prec", [hmg.F64, hmg.F32])
def test_operator_componentwise(k, prec):
    hm, _, A, absA = oracle_case(k)
    print("operator k=%d prec=%d nel=%s" % (k, prec, hm.nel), flush=True)
    L = hmg.Level(hm, prec=prec)
    (u,) = _inputs(L, prec, 41)
    y = to_np(L.apply(L.vector(u)))
    ref = A @ u
    ratio = np.max(np.abs(y - ref) / (_c(k, prec) * (absA @ np.abs(u))))
    print("max componentwise ratio %.3f" % ratio)
    assert ratio <= 1.0


@pytest.mark.parametrize("k", [4, 5, 7])
@pytest.mark.parametrize("prec", [hmg.F64, hmg.F32])
def test_residual_componentwise(k, prec):
    hm, _, A, absA = oracle_case(k)
    print("residual k=%d prec=%d" % (k, prec), flush=True)
    L = hmg.Level(hm, prec=prec)
    u, b = _inputs(L, prec, 42, 43)
    r = to_np(L.residual(L.vector(b), L.vector(u)))
    ref = b - A @ u
    eps = 2.0 ** -53 if prec == hmg.F64 else EPS32
    bound = _c(k, prec) * (absA @ np.abs(u)) + eps * np.abs(b)
    ratio = np.max(np.abs(r - ref) / bound)
    print("max componentwise ratio %.3f" % ratio)
    assert ratio <= 1.0


@pytest.mark.parametrize("k", [4, 5, 7])
@pytest.mark.parametrize("prec", [hmg.F64, hmg.F32])
@pytest.mark.parametrize("x_is_zero", [False, True])
def test_chebyshev_steps(k, prec, x_is_zero):
    """Chebyshev(1) from a nonzero start is exactly one fused step with
    x_old = x (sigma_0 = 0); Chebyshev(2) adds one with sigma_1 != 0, whose
    x_old is the kept or re-read input.  Each step is compared with the
    oracle's step taken from the GPU's own previous iterate, so the bound is
    per step; the final iterate is also compared with the oracle's whole
    Chebyshev(5) smoothing normwise."""
    hm, _, A, absA = oracle_case(k)
    print("chebyshev k=%d prec=%d x_is_zero=%s" % (k, prec, x_is_zero), flush=True)
    L = hmg.Level(hm, prec=prec)
    dinv = 1.0 / A.diagonal()
    if prec == hmg.F32:  # the library stores the FP64 inverse rounded to FP32
        dinv = dinv.astype(np.float32).astype(np.float64)
    b, x0 = _inputs(L, prec, 44, 45)
    if x_is_zero:
        x0 = np.zeros_like(x0)
    lmax = 1.9
    sig, th = solver.chebyshev_coefficients(5, lmax)
    eps = 2.0 ** -53 if prec == hmg.F64 else EPS32
    c = _c(k, prec)
    xs = [x0, x0]  # x_{-1} = x_0
    for steps in range(1, 6):
        x = L.vector(x0)
        L.chebyshev(L.vector(b), x, steps, lmax, x_is_zero=x_is_zero)
        got = to_np(x)
        xp, xc = xs[-2], xs[-1]
        j = steps - 1
        res = b - A @ xc
        ref = xc + sig[j] * (xc - xp) + th[j] * dinv * res
        upd = np.abs(th[j] * dinv * res)
        bound = (abs(th[j] * dinv) * (c * (absA @ np.abs(xc)) + eps * np.abs(b)) + c * upd
                 + 4 * eps * (np.abs(xc) + abs(sig[j]) * np.abs(xc - xp) + upd))
        if j == 0 and x_is_zero:  # x_1 = theta_0 D^{-1} b: no operator apply
            bound = (4 * eps + c) * np.abs(ref) + 1e-300
        ratio = np.max(np.abs(got - ref) / bound)
        print("step %d: max componentwise ratio %.3f" % (steps, ratio))
        assert ratio <= 1.0
        xs.append(got)
    ref5 = solver.chebyshev(A, dinv, b, x0, 5, lmax)
    err = rel_inf(xs[-1], ref5)
    print("Chebyshev(5) normwise rel err %.3e" % err)
    assert err <= (1e-12 if prec == hmg.F64 else 5 * 1e-5)


def test_mixed_precision_solve_of_the_k7_workload():
    """The solve of the k = 7 curvilinear workload with penalty scales
    U[1, 10] at reduced size (2^3 elements, 4,096 DoFs): cph hierarchy with
    floor(p/2), FP32 V-cycle inside FP64 PCG to 1e-10.  The final residual
    is recomputed with the oracle's operator, and the iteration count
    matches the oracle's PCG with an FP64 V-cycle (same lambda_max values)
    within one."""
    import torch
    k = 7
    hm, om, A, absA = oracle_case(k, bc=(0,) * 6)
    H = hmg.Hierarchy(hm, "cph", pseq=1, h_min=1, mg_prec=hmg.F32)
    b = torch.as_tensor(uniform(46, H.n_dofs), device="cuda")
    x, st = H.solve(b, rtol=1e-10)
    bn, xn = to_np(b), to_np(x)
    res = np.linalg.norm(bn - sipg.apply(om, k, xn).ravel()) / np.linalg.norm(bn)
    res_a = np.linalg.norm(bn - A @ xn) / np.linalg.norm(bn)
    lv = H.levels()
    oh = solver.Hierarchy(om, k, "cph", pseq=1, h_min=1, lmax=[l["lmax"] for l in lv[:-1]])
    assert [(l["space"], l["k"], l["mesh"].nel) for l in oh.levels] == [(l["space"], l["degree"], l["nel"])
                                                                         for l in lv]
    _, hist = solver.pcg(A, bn, precond=oh.vcycle, rtol=1e-10)
    # the library stops on its own FP64 residual; the oracle's operator
    # differs from it by at most 1e-12 (|A||x|)_i per result
    allow = 1e-12 * np.linalg.norm(absA @ np.abs(xn)) / np.linalg.norm(bn)
    print("k7 mixed solve: %s, oracle residual %.3e (assembled %.3e, operator allowance %.1e), "
          "oracle PCG %d iterations" % (st, res, res_a, allow, len(hist) - 1))
    assert res <= 1.05e-10 + allow and res_a <= 1.05e-10 + allow
    assert abs(st["iters"] - (len(hist) - 1)) <= 1
