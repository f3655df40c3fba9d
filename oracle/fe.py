"""Continuous Q_k finite element space on the same structured meshes.

Sec. 2 (eq:WeakFormFE): the conforming space uses the form (grad v, grad u)
with no face terms; Dirichlet conditions are imposed strongly, only the
homogeneous operator is needed inside multigrid, and constrained DoFs are
kept in the system with diagonal entry 1.

Reading: constrained rows and columns act as the identity, so
A_FE = C (E^T A_cell E) C + (I - C), with E the gather from global nodes to
element-local nodes and C the diagonal projector onto unconstrained nodes.
Global node index gx + Mx*(gy + My*gz), M_d = N_d*k + 1; element-local node
(i, j, l) of element (ex, ey, ez) is global node (ex*k+i, ey*k+j, ez*k+l).
"""
import numpy as np
import scipy.sparse as sp

from . import sipg


def n_nodes(mesh, k):
    Mx, My, Mz = (N * k + 1 for N in mesh.nel)
    return Mx * My * Mz


def gather_matrix(mesh, k):
    """E (N_el*(k+1)^3 x N_fe): element-local DG layout <- global FE nodes."""
    n = k + 1
    Mx, My, _ = (N * k + 1 for N in mesh.nel)
    e = np.arange(mesh.n_el)
    ex, ey, ez = mesh.coords(e)
    loc = np.arange(n ** 3)
    i, j, l = loc % n, (loc // n) % n, loc // (n * n)
    gx = ex[:, None] * k + i[None, :]
    gy = ey[:, None] * k + j[None, :]
    gz = ez[:, None] * k + l[None, :]
    node = (gx + Mx * (gy + My * gz)).ravel()
    rows = np.arange(mesh.n_el * n ** 3)
    return sp.csr_matrix((np.ones(len(rows)), (rows, node)), shape=(len(rows), n_nodes(mesh, k)))


def free_mask(mesh, k):
    """1.0 on unconstrained nodes, 0.0 on nodes of Dirichlet box faces."""
    M = [N * k + 1 for N in mesh.nel]
    g = np.meshgrid(*[np.arange(m) for m in M], indexing="ij")
    free = np.ones(M)
    for d in range(3):
        if mesh.bc[2 * d] == 0:
            free[g[d] == 0] = 0.0
        if mesh.bc[2 * d + 1] == 0:
            free[g[d] == M[d] - 1] = 0.0
    return free.ravel(order="F")


def multiplicity(mesh, k):
    """Number of elements sharing each global node."""
    E = gather_matrix(mesh, k)
    return np.asarray(E.sum(axis=0)).ravel()


def assemble(mesh, k):
    """A_FE with constrained rows/columns replaced by the identity."""
    Acell = sipg.assemble(mesh, k, faces=False)
    E = gather_matrix(mesh, k)
    C = sp.diags(free_mask(mesh, k))
    Araw = E.T @ Acell @ E
    return (C @ Araw @ C + sp.diags(1.0 - free_mask(mesh, k))).tocsr()


def diagonal(mesh, k):
    return assemble(mesh, k).diagonal()
