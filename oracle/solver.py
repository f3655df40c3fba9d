"""Krylov solver, multigrid V-cycle and Chebyshev-Jacobi smoother.

Alg. 1 (preconditioned CG), Alg. 2 (V-cycle), Alg. 3 (Chebyshev-accelerated
Jacobi), Sec. 3.1 (target interval [0.06, 1.2] * lambda_max, lambda_max from
20 CG iterations in the setup), Sec. 3.2 (coarsening strategies and p
sequences), Sec. 5.1 (metrics rho and n10).

Readings:
  * sigma_j, theta_j are the coefficients of the classical three-term
    Chebyshev iteration (Saad, Iterative Methods for Sparse Linear Systems,
    Alg. 12.1) applied to D^{-1}A on [a, b] = [0.06, 1.2] * lambda_max:
    c = (b+a)/2, delta = (b-a)/2, s1 = c/delta, rho_0 = 1/s1, x_1 = x_0 +
    D^{-1} r_0 / c, and for j >= 1 rho_j = 1/(2 s1 - rho_{j-1}),
    sigma_j = rho_j rho_{j-1}, theta_j = 2 rho_j / delta.  Chebyshev(n_s)
    means n_s operator applications (n_s steps of Alg. 3).
  * lambda_max: Jacobi-preconditioned CG on A x = r, x_0 = 0, r a seeded
    U[-1,1] vector; the largest eigenvalue of the Lanczos tridiagonal matrix
    built from the CG coefficients alpha_j, beta_j.
  * the coarse-level solver is an exact FP64 solve (the paper's AMG is a
    third-party library); h-coarsening stops when an N_d is odd or
    max N_d <= h_min.
"""
import numpy as np
import scipy.linalg as sla

from . import fe, rng, sipg, transfer
from .mesh import BoxMesh


def chebyshev_coefficients(n_s, lmax, lo=0.06, hi=1.2):
    """Lists (sigma_j, theta_j), j = 0..n_s-1, for Alg. 3 (reading above)."""
    a, b = lo * lmax, hi * lmax
    c, delta = 0.5 * (b + a), 0.5 * (b - a)
    s1 = c / delta
    sig, th = [0.0], [1.0 / c]
    rho_prev = 1.0 / s1
    for _ in range(1, n_s):
        rho = 1.0 / (2.0 * s1 - rho_prev)
        sig.append(rho * rho_prev)
        th.append(2.0 * rho / delta)
        rho_prev = rho
    return sig, th


def chebyshev(A, dinv, b, x0, n_s, lmax, lo=0.06, hi=1.2):
    """Alg. 3: x_{j+1} = x_j + sigma_j (x_j - x_{j-1}) + theta_j D^{-1}(b - A x_j),
    with x_{-1} = x_0."""
    sig, th = chebyshev_coefficients(n_s, lmax, lo, hi)
    x_prev = x0.copy()
    x = x0.copy()
    for j in range(n_s):
        x_new = x + sig[j] * (x - x_prev) + th[j] * dinv * (b - A @ x)
        x_prev, x = x, x_new
    return x


def lanczos_lmax(A, dinv, r0, iters=20):
    """Largest Ritz value of D^{-1}A from `iters` Jacobi-PCG iterations on
    A x = r0 (x_0 = 0): T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T_{j,j+1} = sqrt(beta_j)/alpha_j."""
    r = r0.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    for _ in range(iters):
        Ap = A @ p
        pAp = p @ Ap
        if pAp <= 0 or rz <= 0:
            break
        alpha = rz / pAp
        r = r - alpha * Ap
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        alphas.append(alpha)
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
        if rz_new <= 0:
            break
    m = len(alphas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return float(np.linalg.eigvalsh(T).max())


def next_degree(k, pseq):
    """Sec. 3.2.2 p-sequences: 0 -> k-1, 1 -> floor(k/2), 2 -> 1."""
    return {0: k - 1, 1: k // 2, 2: 1}[pseq]


def can_coarsen_h(mesh, h_min=4):
    return all(N % 2 == 0 for N in mesh.nel) and max(mesh.nel) > h_min


def level_specs(mesh, k, strategy, pseq=1, h_min=4):
    """Levels fine -> coarse as (space, k, mesh, kind-of-transfer-to-coarser).
    Each letter of the strategy string coarsens exhaustively in its turn
    (Sec. 3.2: one parameter of l = f(h, p, c) changes per level)."""
    specs = [["DG", k, mesh, None]]
    space, kk, m = "DG", k, mesh
    for letter in strategy:
        if letter == "c" and space == "DG":
            specs[-1][3] = "c"
            space = "FE"
            specs.append([space, kk, m, None])
        elif letter == "p":
            while kk > 1:
                specs[-1][3] = "p"
                kk = next_degree(kk, pseq)
                specs.append([space, kk, m, None])
        elif letter == "h":
            while can_coarsen_h(m, h_min):
                specs[-1][3] = "h"
                m = transfer.coarse_mesh(m)
                specs.append([space, kk, m, None])
    return specs


class Hierarchy:
    """Level matrices (re-discretized, Sec. 2), diagonals, lambda_max and the
    prolongations between consecutive levels.  levels[0] is the finest."""

    def __init__(self, mesh, k, strategy="cph", pseq=1, n_s=5, h_min=4, ip_factor=1.0,
                 lmax_seed=1, lmax=None):
        self.n_s = n_s
        self.levels = []
        specs = level_specs(mesh, k, strategy, pseq, h_min)
        for idx, (space, kk, m, kind) in enumerate(specs):
            if space == "DG":
                A = sipg.assemble(m, kk, ip_factor=ip_factor)
            else:
                A = fe.assemble(m, kk)
            lev = {"space": space, "k": kk, "mesh": m, "A": A, "dinv": 1.0 / A.diagonal()}
            self.levels.append(lev)
        for idx in range(len(specs) - 1):
            space, kk, m, kind = specs[idx]
            cspace, ck, cm, _ = specs[idx + 1]
            if kind == "c":
                P = transfer.c_prolongation(m, kk)
            elif kind == "p":
                P = transfer.dg_p(m, kk, ck) if space == "DG" else transfer.fe_p(m, kk, ck)
            else:
                P = transfer.dg_h(m, kk) if space == "DG" else transfer.fe_h(m, kk)
            self.levels[idx]["P"] = P
            self.levels[idx]["kind"] = kind
        for idx, lev in enumerate(self.levels[:-1]):
            if lmax is not None:
                lev["lmax"] = lmax[idx]
            else:
                r0 = rng.uniform_pm1(lmax_seed, lev["A"].shape[0])
                lev["lmax"] = lanczos_lmax(lev["A"], lev["dinv"], r0)
        coarse = self.levels[-1]
        coarse["chol"] = sla.cho_factor(coarse["A"].toarray())

    def vcycle(self, b, l=0):
        """Alg. 2 with x^{(l)} = 0 on entry."""
        lev = self.levels[l]
        if l == len(self.levels) - 1:
            return sla.cho_solve(lev["chol"], b)
        A, dinv = lev["A"], lev["dinv"]
        x = chebyshev(A, dinv, b, np.zeros_like(b), self.n_s, lev["lmax"])
        r = b - A @ x
        bc = lev["P"].T @ r
        xc = self.vcycle(bc, l + 1)
        x = x + lev["P"] @ xc
        return chebyshev(A, dinv, b, x, self.n_s, lev["lmax"])


def pcg(A, b, x0=None, precond=None, rtol=1e-10, atol=0.0, maxit=1000):
    """Alg. 1.  Stops when ||r||/||r_0|| <= rtol or ||r|| <= atol.
    Returns (x, residual-norm history [||r_0||, ||r_1||, ...])."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    M = (lambda r: r.copy()) if precond is None else precond
    r = b - A @ x
    nr = np.linalg.norm(r)
    hist = [nr]
    r0 = nr
    v = M(r)
    p = v.copy()
    delta = r @ v
    it = 0
    while nr / r0 > rtol and nr > atol and it < maxit:
        v = A @ p
        omega = delta / (p @ v)
        x = x + omega * p
        r = r - omega * v
        nr = np.linalg.norm(r)
        hist.append(nr)
        v = M(r)
        delta_old = delta
        delta = r @ v
        p = v + (delta / delta_old) * p
        it += 1
    return x, hist


def metrics(hist):
    """Sec. 5.1: rho = (||r_n||/||r_0||)^{1/n}, n10 = -10 / log10(rho)."""
    n = len(hist) - 1
    rho = (hist[-1] / hist[0]) ** (1.0 / n)
    return rho, -10.0 / np.log10(rho)
