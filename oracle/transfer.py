"""Multigrid transfer operators as explicit sparse matrices.

Sec. 3.2: prolongation P = sum_e S_e P_e G_e with the element-wise operator
P_e = (M_e^l)^{-1} M_e^{l,l-1} (L2 projection in reference space), which is a
tensor product of 1-D matrices interpolating the coarse basis at the fine
nodes; S_e weights shared nodes by their multiplicity in continuous spaces;
restriction R = P^T.  DG-to-FE (c) transfer: the element-wise operator is the
identity, prolongation injects shared values, restriction sums duplicates.
h-transfer: octree refinement, each coarse element has 2^3 children.

Readings: multiplicity weight 1/mult in the FE scatter (equivalently, the
continuous value); constrained FE nodes are excluded on both sides
(prolongation writes 0 there, restriction returns 0 there).
"""
import numpy as np
import scipy.sparse as sp

from . import basis, fe
from .mesh import BoxMesh


def p_matrix_1d(kf, kc):
    """P[i, j] = l^c_j(x^f_i): coarse GLL Lagrange basis at fine GLL nodes."""
    return basis.lagrange_values(basis.gll_nodes(kc), basis.gll_nodes(kf))


def h_matrix_1d(k, child):
    """P[i, j] = l_j((child + x_i)/2): parent basis at the child's nodes."""
    x = basis.gll_nodes(k)
    return basis.lagrange_values(x, 0.5 * (child + x))


def l2_projection_1d(kf, kc, child=None):
    """(M_f)^{-1} M_{f,c} on the reference interval of the fine element,
    with exact Gauss quadrature (used to pin that it equals interpolation)."""
    xf, xc = basis.gll_nodes(kf), basis.gll_nodes(kc)
    z, w = basis.gauss(kf + kc + 2)
    Vf = basis.lagrange_values(xf, z)
    zc = z if child is None else 0.5 * (child + z)
    Vc = basis.lagrange_values(xc, zc)
    M = Vf.T @ (w[:, None] * Vf)
    Mfc = Vf.T @ (w[:, None] * Vc)
    return np.linalg.solve(M, Mfc)


def dg_p(mesh, kf, kc):
    """DG p-prolongation (same mesh): block-diagonal kron of 1-D matrices."""
    P1 = p_matrix_1d(kf, kc)
    Pe = np.kron(P1, np.kron(P1, P1))
    return sp.kron(sp.identity(mesh.n_el), sp.csr_matrix(Pe)).tocsr()


def coarse_mesh(mesh):
    """The octree parent mesh (every N_d halved).  A per-element penalty
    factor (not part of the paper; used by the variable-penalty workload)
    is re-discretized like the rest of the operator (Sec. 2: coarser levels
    evaluate the operator for the coarse parameters): the parent's factor
    is the mean over its eight children."""
    assert all(N % 2 == 0 for N in mesh.nel)
    cn = tuple(N // 2 for N in mesh.nel)
    ts = None
    if mesh.tau_scale is not None:
        ts = np.zeros(int(np.prod(cn)))
        fine = np.asarray(mesh.tau_scale, dtype=np.float64)
        for e in range(mesh.n_el):
            ex, ey, ez = (int(c) for c in mesh.coords(e))
            ts[ex // 2 + cn[0] * (ey // 2 + cn[1] * (ez // 2))] += fine[e] / 8.0
    return BoxMesh(cn, mesh.lo, mesh.hi, mesh.deform, mesh.waves, mesh.bc, ts, mesh.mapping_degree)


def dg_h(mesh_f, k):
    """DG h-prolongation from the parent mesh to mesh_f (same degree)."""
    n = k + 1
    nd = n ** 3
    mc = coarse_mesh(mesh_f)
    rows, cols, vals = [], [], []
    H = [h_matrix_1d(k, c) for c in (0, 1)]
    for e in range(mesh_f.n_el):
        ex, ey, ez = (int(c) for c in mesh_f.coords(e))
        parent = mc.index(ex // 2, ey // 2, ez // 2)
        Pe = np.kron(H[ez % 2], np.kron(H[ey % 2], H[ex % 2]))
        R, C = np.meshgrid(e * nd + np.arange(nd), parent * nd + np.arange(nd), indexing="ij")
        rows.append(R.ravel())
        cols.append(C.ravel())
        vals.append(Pe.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(mesh_f.n_el * nd, mc.n_el * nd))


def c_prolongation(mesh, k):
    """DG <- FE at the same (h, k): injection of shared values, 0 from
    constrained nodes."""
    return (fe.gather_matrix(mesh, k) @ sp.diags(fe.free_mask(mesh, k))).tocsr()


def fe_from_dg(mesh, k, P_dg, mesh_c, kc):
    """FE prolongation built from a DG one: W_f E_f^T P_dg E_c C_c, with
    W_f = diag(free / multiplicity) (the multiplicity-weighted scatter S_e)."""
    Ef = fe.gather_matrix(mesh, k)
    Wf = sp.diags(fe.free_mask(mesh, k) / fe.multiplicity(mesh, k))
    Ec = c_prolongation(mesh_c, kc)
    return (Wf @ Ef.T @ P_dg @ Ec).tocsr()


def fe_p(mesh, kf, kc):
    return fe_from_dg(mesh, kf, dg_p(mesh, kf, kc), mesh, kc)


def fe_h(mesh_f, k):
    return fe_from_dg(mesh_f, k, dg_h(mesh_f, k), coarse_mesh(mesh_f), k)
