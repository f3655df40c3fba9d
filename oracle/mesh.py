"""Structured hexahedral box meshes with a cubic manifold mapping.

Sec. 2: elements are images of the reference cube [0,1]^3 under a polynomial
mapping x(xi).  Sec. 5.3 (cube test case): the curvilinear mesh is a
deformed cube represented with element mappings of polynomial degree 3,
independently of the degree of the shape functions.

Readings (the paper is silent on these):
  * the degree-3 mapping interpolates the analytic deformation at the 4^3
    GLL(3) support points of each element; shared faces share their
    support points, so the mapped mesh is watertight (mapping_degree 0
    evaluates the analytic deformation itself instead);
  * the deformation is x_i += a * prod_j sin(w * pi * s_j) with
    s_j = (x_j - lo_j)/(hi_j - lo_j) the normalised undeformed coordinate
    and w half-waves per direction (w = 2 is the paper's cube deformation
    on [-1,1]^3, whose third sine factor is garbled in the text; w = 1 is
    the mild variant used by the large benchmark meshes); it vanishes on
    the boundary, so the domain stays the box;
  * face normals and surface elements follow Nanson's formula,
    n = J^{-T} n_ref / |J^{-T} n_ref|,  dGamma = |det J| |J^{-T} n_ref| w_a w_b.

Element numbering e = ex + Nx*(ey + Ny*ez).  Faces of an element are named
by direction d in {0,1,2} and side s in {0,1} (the face xi_d = s); the box
face id of a boundary face is 2*d + s.
"""
from dataclasses import dataclass, field

import numpy as np

from . import basis


@dataclass
class BoxMesh:
    nel: tuple                      # (Nx, Ny, Nz)
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    deform: float = 0.0             # amplitude a of the sine deformation
    waves: int = 1                  # half-waves per direction of the deformation
    bc: tuple = (0, 0, 0, 0, 0, 0)  # per box face: 0 Dirichlet, 1 Neumann
    tau_scale: np.ndarray = field(default=None)  # optional per-element factor
    mapping_degree: int = 3         # 3: cubic interpolant of the deformation; 0: the deformation itself

    @property
    def n_el(self):
        return int(np.prod(self.nel))

    def coords(self, e):
        Nx, Ny, _ = self.nel
        e = np.asarray(e)
        return e % Nx, (e // Nx) % Ny, e // (Nx * Ny)

    def index(self, ex, ey, ez):
        Nx, Ny, _ = self.nel
        return ex + Nx * (ey + Ny * ez)

    def neighbor(self, e, d, s):
        """Neighbour of element e across its face (d, s), or -1 on the boundary."""
        c = list(self.coords(e))
        c[d] += 1 if s == 1 else -1
        if c[d] < 0 or c[d] >= self.nel[d]:
            return -1
        return int(self.index(*c))

    def deformed(self, X):
        """Apply the analytic deformation to undeformed points X[..., 3]."""
        if self.deform == 0.0:
            return X.copy()
        lo = np.asarray(self.lo)
        hi = np.asarray(self.hi)
        s = (X - lo) / (hi - lo)
        bump = self.deform * np.prod(np.sin(self.waves * np.pi * s), axis=-1)
        return X + bump[..., None]

    def support_points(self, elems=None):
        """Q3 support points, shape (E, 64, 3), index a + 4b + 16c over the
        GLL(3) nodes in each reference direction."""
        if elems is None:
            elems = np.arange(self.n_el)
        g = basis.gll_nodes(3)
        ex, ey, ez = self.coords(np.asarray(elems))
        h = (np.asarray(self.hi) - np.asarray(self.lo)) / np.asarray(self.nel)
        ga, gb, gc = np.meshgrid(g, g, g, indexing="ij")
        # support index a + 4b + 16c  ->  flatten in Fortran order of (a,b,c)
        ref = np.stack([ga.ravel(order="F"), gb.ravel(order="F"), gc.ravel(order="F")], axis=-1)
        base = np.stack([ex, ey, ez], axis=-1).astype(np.float64)
        Xhat = np.asarray(self.lo) + (base[:, None, :] + ref[None, :, :]) * h
        return self.deformed(Xhat)

    def map(self, elems, p1, p2, p3):
        """Physical points x[E, P, 3] and Jacobians J[E, P, 3, 3]
        (J[r, s] = dx_r / dxi_s) at the reference tensor grid p1 x p2 x p3
        (first index fastest)."""
        if self.mapping_degree == 0:
            return self._map_exact(elems, p1, p2, p3)
        X = self.support_points(elems)
        V, G = basis.tabulate3(basis.gll_nodes(3), p1, p2, p3)
        x = np.einsum("pa,ear->epr", V, X)
        J = np.stack([np.einsum("pa,ear->epr", G[s], X) for s in range(3)], axis=-1)
        return x, J


def _exact_map(mesh, elems, p1, p2, p3):
    """The analytic element map: the undeformed point plus the deformation,
    J = diag(h) + grad of the deformation (chain rule, ds_d/dxi_d = 1/N_d)."""
    elems = np.asarray(elems)
    ex, ey, ez = mesh.coords(elems)
    h = (np.asarray(mesh.hi) - np.asarray(mesh.lo)) / np.asarray(mesh.nel)
    g3, g2, g1 = np.meshgrid(p3, p2, p1, indexing="ij")  # x fastest after ravel
    ref = np.stack([g1.ravel(), g2.ravel(), g3.ravel()], axis=-1)  # (P, 3)
    base = np.stack([ex, ey, ez], axis=-1).astype(np.float64)  # (E, 3)
    Xhat = np.asarray(mesh.lo) + (base[:, None, :] + ref[None, :, :]) * h  # (E, P, 3)
    E, P = Xhat.shape[0], Xhat.shape[1]
    J = np.zeros((E, P, 3, 3))
    for d in range(3):
        J[..., :, d] = 0.0
        J[..., d, d] = h[d]
    if mesh.deform == 0.0:
        return Xhat, J
    s = (Xhat - np.asarray(mesh.lo)) / (np.asarray(mesh.hi) - np.asarray(mesh.lo))
    w = mesh.waves * np.pi
    sn, cs = np.sin(w * s), np.cos(w * s)
    bump = mesh.deform * np.prod(sn, axis=-1)
    x = Xhat + bump[..., None]
    for c in range(3):
        others = np.prod(np.delete(sn, c, axis=-1), axis=-1)
        dbump = mesh.deform * w * cs[..., c] * others / mesh.nel[c]  # d bump / d xi_c
        J[..., :, c] += dbump[..., None]
    return x, J


BoxMesh._map_exact = _exact_map


def face_ref_points(n, d, s):
    """Reference tensor grids (p1, p2, p3) of the n x n Gauss points on the
    face xi_d = s, and the face weights w[qa + n*qb] over the two tangential
    directions taken in increasing order."""
    z, w = basis.gauss(n)
    pts = [z, z, z]
    pts[d] = np.array([float(s)])
    return pts, np.kron(w, w)


def cell_geometry(mesh, k, elems=None):
    """Per cell quadrature point (n = k+1 Gauss points per direction):
    J^{-T} as Jinvt[E, Q, 3, 3], JxW[E, Q] = w_q |det J_q|, and x[E, Q, 3].
    Sec. 4 (the volume integral transformed to the reference element)."""
    if elems is None:
        elems = np.arange(mesh.n_el)
    n = k + 1
    z, w = basis.gauss(n)
    x, J = mesh.map(elems, z, z, z)
    wq = np.kron(w, np.kron(w, w))
    det = np.linalg.det(J)
    Jinvt = np.linalg.inv(J).transpose(0, 1, 3, 2)
    return Jinvt, np.abs(det) * wq, x


def face_geometry(mesh, k, elems, d, s):
    """Geometry of face (d, s) of each element seen from that element:
    Jinvt[E, F, 3, 3] at the face Gauss points, outward unit normal
    normal[E, F, 3] and surface weight dA[E, F] (Nanson's formula), and the
    physical points x[E, F, 3]."""
    n = k + 1
    pts, wf = face_ref_points(n, d, s)
    x, J = mesh.map(elems, *pts)
    det = np.linalg.det(J)
    Jinvt = np.linalg.inv(J).transpose(0, 1, 3, 2)
    nref = np.zeros(3)
    nref[d] = 2.0 * s - 1.0
    m = Jinvt @ nref
    norm = np.linalg.norm(m, axis=-1)
    return Jinvt, m / norm[..., None], np.abs(det) * norm * wf, x
