"""The SIPG Laplace operator, written as its plain definition.

Sec. 2 (weak form eq:WeakFormDG, fluxes eq:InteriorPenaltyFlux1/2, mirror
boundary conditions eq:BoundaryConditions, penalty parameter) and Sec. 4
(eq:MatrixFreeAbstractNotation; the cell integral transformed to the
reference element).  The homogeneous bilinear form is

  a(v,u) = sum_e  (grad v, grad u)_e
         + sum_{interior F} ( -{dv/dn}[u] - [v]{du/dn} + tau_F [v][u] )_F
         + sum_{Dirichlet F} ( -dv/dn u - v du/dn + 2 tau_e v u )_F
         + sum_{Neumann F}   0,

with [w] = w^- - w^+ and {dw/dn} = (grad w^- + grad w^+).n^- / 2, n^- the
outward unit normal of the "-" element.  On Dirichlet faces the mirror
principle sets u^+ = -u^- and du^+/dn = du^-/dn, which yields the factor 2 on
the penalty; on homogeneous Neumann faces u^+ = u^- and du^+/dn = -du^-/dn
so the face contributes nothing.  Every integral uses the (k+1)-point Gauss
tensor rule through the element mapping.

Readings: on an interior face the "-" element is the one with the lower
coordinate along the face normal direction, and n^- and dGamma are taken
from its mapping.  tau_e = ip * s_e * (k+1)^2 (A_int/2 + A_bdry)/V with the
volume and areas computed with the same Gauss rule; tau_F = max(tau^-, tau^+)
inside and tau_e on the boundary.  DoF index of DG vectors:
e*n^3 + i + n*(j + n*l).
"""
import numpy as np
import scipy.sparse as sp

from . import basis
from .mesh import cell_geometry, face_geometry, face_ref_points


def _face_tab(k, d, s):
    n = k + 1
    pts, _ = face_ref_points(n, d, s)
    return basis.tabulate3(basis.gll_nodes(k), *pts)


def _cell_tab(k):
    z, _ = basis.gauss(k + 1)
    return basis.tabulate3(basis.gll_nodes(k), z, z, z)


def penalty(mesh, k, ip_factor=1.0, elems=None):
    """tau_e per element (Sec. 2, penalty parameter of Hillewaert):
    (k+1)^2 * (A(interior faces)/2 + A(boundary faces)) / V(element),
    times ip_factor and the optional per-element scale.  With `elems`, only
    those entries are computed (the others are NaN)."""
    sel = np.arange(mesh.n_el) if elems is None else np.unique(np.asarray(elems))
    elems = sel
    _, JxW, _ = cell_geometry(mesh, k, elems)
    vol = JxW.sum(axis=1)
    area = np.zeros(len(elems))
    for d in range(3):
        for s in range(2):
            _, _, dA, _ = face_geometry(mesh, k, elems, d, s)
            a = dA.sum(axis=1)
            interior = np.array([mesh.neighbor(e, d, s) >= 0 for e in elems])
            area += np.where(interior, 0.5 * a, a)
    t = ip_factor * (k + 1) ** 2 * area / vol
    if mesh.tau_scale is not None:
        t = t * np.asarray(mesh.tau_scale, dtype=np.float64)[elems]
    tau = np.full(mesh.n_el, np.nan)
    tau[elems] = t
    return tau


def _grad_phys(Jinvt, G):
    """Physical gradients of all basis functions: B[E, P, 3, i] =
    sum_s Jinvt[E, P, r, s] G_s[P, i]."""
    Gs = np.stack(G, axis=1)  # (P, 3, i)
    return np.einsum("eprs,psi->epri", Jinvt, Gs)


def assemble(mesh, k, tau=None, ip_factor=1.0, faces=True):
    """Assembled sparse SIPG matrix A (CSR), row = test, column = trial.
    Cell blocks and face blocks (--, -+, +-, ++) built from full 3-D basis
    tabulations, i.e. the weak form with no factorization.  For tiny meshes.
    faces=False returns the block-diagonal cell part only (grad v, grad u)_e,
    the element matrices of the continuous FE form eq:WeakFormFE."""
    n = k + 1
    nd = n ** 3
    if tau is None and faces:
        tau = penalty(mesh, k, ip_factor)
    rows, cols, vals = [], [], []

    def add_block(ri, ci, blk):
        R, C = np.meshgrid(ri, ci, indexing="ij")
        rows.append(R.ravel())
        cols.append(C.ravel())
        vals.append(blk.ravel())

    elems = np.arange(mesh.n_el)
    # cell integrals (grad v, grad u)_e
    _, G = _cell_tab(k)
    Jinvt, JxW, _ = cell_geometry(mesh, k, elems)
    B = _grad_phys(Jinvt, G)
    Ae = np.einsum("epri,ep,eprj->eij", B, JxW, B)
    for e in elems:
        dofs = e * nd + np.arange(nd)
        add_block(dofs, dofs, Ae[e])

    for d in (range(3) if faces else ()):
        # interior faces: "-" = left element (face s=1), "+" = right (face s=0)
        left = np.array([e for e in elems if mesh.neighbor(e, d, 1) >= 0], dtype=np.int64)
        if len(left):
            right = np.array([mesh.neighbor(e, d, 1) for e in left], dtype=np.int64)
            JL, nrm, dA, _ = face_geometry(mesh, k, left, d, 1)
            JR, _, _, _ = face_geometry(mesh, k, right, d, 0)
            VL, GL = _face_tab(k, d, 1)
            VR, GR = _face_tab(k, d, 0)
            dnL = np.einsum("efr,efri->efi", nrm, _grad_phys(JL, GL))
            dnR = np.einsum("efr,efri->efi", nrm, _grad_phys(JR, GR))
            for idx, (eL, eR) in enumerate(zip(left, right)):
                jump = np.concatenate([VL, -VR], axis=1)                    # [phi]
                avg = 0.5 * np.concatenate([dnL[idx], dnR[idx]], axis=1)    # {dphi/dn}
                tF = max(tau[eL], tau[eR])
                w = dA[idx][:, None]
                blk = (-(avg * w).T @ jump - (jump * w).T @ avg + tF * (jump * w).T @ jump)
                dofs = np.concatenate([eL * nd + np.arange(nd), eR * nd + np.arange(nd)])
                add_block(dofs, dofs, blk)
        # Dirichlet boundary faces (mirror principle)
        for s in range(2):
            if mesh.bc[2 * d + s] != 0:
                continue
            bnd = np.array([e for e in elems if mesh.neighbor(e, d, s) < 0], dtype=np.int64)
            if not len(bnd):
                continue
            Jb, nrm, dA, _ = face_geometry(mesh, k, bnd, d, s)
            Vb, Gb = _face_tab(k, d, s)
            dn = np.einsum("efr,efri->efi", nrm, _grad_phys(Jb, Gb))
            for idx, e in enumerate(bnd):
                w = dA[idx][:, None]
                blk = (-(dn[idx] * w).T @ Vb - (Vb * w).T @ dn[idx]
                       + 2.0 * tau[e] * (Vb * w).T @ Vb)
                dofs = e * nd + np.arange(nd)
                add_block(dofs, dofs, blk)

    N = mesh.n_el * nd
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A.tocsr()


def apply(mesh, k, u, tau=None, elems=None, ip_factor=1.0, batch=4096):
    """(A u) on the requested elements, element by element (each element's
    test functions against its cell and its six faces).  Dense tabulations,
    O(n^6) per element: usable on large meshes and on sampled elements.
    Returns v[len(elems), n^3]."""
    n = k + 1
    nd = n ** 3
    if elems is None:
        elems = np.arange(mesh.n_el)
    elems = np.asarray(elems, dtype=np.int64)
    if tau is None:
        near = [elems] + [np.array([mesh.neighbor(e, d, s) for e in elems]) for d in range(3) for s in range(2)]
        near = np.concatenate(near)
        tau = penalty(mesh, k, ip_factor, elems=near[near >= 0] if len(elems) < mesh.n_el else None)
    U = np.asarray(u, dtype=np.float64).reshape(mesh.n_el, nd)
    out = np.zeros((len(elems), nd))
    _, Gc = _cell_tab(k)
    Gc = np.stack(Gc, axis=1)  # (Q, 3, i)
    for b0 in range(0, len(elems), batch):
        eb = elems[b0:b0 + batch]
        ue = U[eb]
        Jinvt, JxW, _ = cell_geometry(mesh, k, eb)
        gref = np.einsum("qsi,ei->eqs", Gc, ue)
        gphys = np.einsum("eqrs,eqs->eqr", Jinvt, gref)
        flux = gphys * JxW[..., None]
        v = np.einsum("eqrs,eqr->eqs", Jinvt, flux)
        out[b0:b0 + batch] = np.einsum("qsi,eqs->ei", Gc, v)
        for d in range(3):
            for s in range(2):
                out[b0:b0 + batch] += _face_apply(mesh, k, U, tau, eb, d, s)
    return out


def _face_apply(mesh, k, U, tau, eb, d, s):
    """Contribution of face (d, s) of each element in eb to its own test
    functions: sum_q dA [ (-{du/dn} + tau [u]) phi_i - [u]/2 dphi_i/dn ]
    with jump and average taken from the element's own side (own outward
    normal); Dirichlet faces use the mirror values, Neumann faces add 0."""
    nd = (k + 1) ** 3
    res = np.zeros((len(eb), nd))
    nb = np.array([mesh.neighbor(e, d, s) for e in eb], dtype=np.int64)
    Vo, Go = _face_tab(k, d, s)
    Vn, Gn = _face_tab(k, d, 1 - s)
    Jo, nrm_o, dA_o, _ = face_geometry(mesh, k, eb, d, s)
    inner = nb >= 0
    if inner.any():
        ei = eb[inner]
        ni = nb[inner]
        # geometry of the face from its "-" (left) element
        if s == 1:
            Jown, nrm, dA = Jo[inner], nrm_o[inner], dA_o[inner]
            Jnb, _, _, _ = face_geometry(mesh, k, ni, d, 0)
            n_own = nrm
        else:
            Jnb, nrm, dA, _ = face_geometry(mesh, k, ni, d, 1)
            Jown = Jo[inner]
            n_own = -nrm
        uo, un = U[ei], U[ni]
        Bo = _grad_phys(Jown, Go)
        Bn = _grad_phys(Jnb, Gn)
        dphi = np.einsum("efr,efri->efi", n_own, Bo)
        u_o = uo @ Vo.T
        u_n = un @ Vn.T
        dn_o = np.einsum("efi,ei->ef", dphi, uo)
        dn_n = np.einsum("efr,efri,ei->ef", n_own, Bn, un)
        jump = u_o - u_n
        avg = 0.5 * (dn_o + dn_n)
        tF = np.maximum(tau[ei], tau[ni])[:, None]
        vt = (-avg + tF * jump) * dA
        gt = -0.5 * jump * dA
        res[inner] = vt @ Vo + np.einsum("ef,efi->ei", gt, dphi)
    if mesh.bc[2 * d + s] == 0 and (~inner).any():
        eo = eb[~inner]
        uo = U[eo]
        dphi = np.einsum("efr,efri->efi", nrm_o[~inner], _grad_phys(Jo[~inner], Go))
        u_o = uo @ Vo.T
        dn_o = np.einsum("efi,ei->ef", dphi, uo)
        dA = dA_o[~inner]
        jump = 2.0 * u_o
        avg = dn_o
        vt = (-avg + tau[eo][:, None] * jump) * dA
        gt = -0.5 * jump * dA
        res[~inner] = vt @ Vo + np.einsum("ef,efi->ei", gt, dphi)
    return res


def diagonal(mesh, k, tau=None, ip_factor=1.0):
    """diag(A) from a(phi_i, phi_i): cell term |grad phi_i|^2 and, per face,
    the own-side terms with the neighbour trace zero (interior:
    tau phi^2 - phi dphi/dn) or mirrored (Dirichlet: 2 tau phi^2 - 2 phi dphi/dn).
    Sec. 3.1: the diagonal needed by the Chebyshev-Jacobi smoother."""
    n = k + 1
    if tau is None:
        tau = penalty(mesh, k, ip_factor)
    elems = np.arange(mesh.n_el)
    _, G = _cell_tab(k)
    Jinvt, JxW, _ = cell_geometry(mesh, k, elems)
    B = _grad_phys(Jinvt, G)
    diag = np.einsum("epri,ep,epri->ei", B, JxW, B)
    for d in range(3):
        for s in range(2):
            nb = np.array([mesh.neighbor(e, d, s) for e in elems])
            V, Gf = _face_tab(k, d, s)
            J, nrm, dA, _ = face_geometry(mesh, k, elems, d, s)
            if s == 0:
                # interior faces take normal and surface weight from the left element
                inner = nb >= 0
                if inner.any():
                    _, nrmL, dAL, _ = face_geometry(mesh, k, nb[inner], d, 1)
                    nrm = nrm.copy()
                    dA = dA.copy()
                    nrm[inner] = -nrmL
                    dA[inner] = dAL
            dphi = np.einsum("efr,efri->efi", nrm, _grad_phys(J, Gf))
            for e in elems:
                if nb[e] >= 0:
                    tF = max(tau[e], tau[nb[e]])
                    diag[e] += dA[e] @ (tF * V ** 2 - V * dphi[e])
                elif mesh.bc[2 * d + s] == 0:
                    diag[e] += dA[e] @ (2.0 * tau[e] * V ** 2 - 2.0 * V * dphi[e])
    return diag.ravel()


def rhs(mesh, k, f, g=None, h=None, tau=None, ip_factor=1.0):
    """Right-hand side with the inhomogeneous boundary data moved over (Sec. 2,
    splitting a = a_hom + a_inhom):
      b_i = (phi_i, f) - sum_{Dirichlet F} (dphi_i/dn - 2 tau phi_i, g)_F
                       + sum_{Neumann F} (phi_i, h)_F.
    f, g, h take points x[..., 3] and return values."""
    n = k + 1
    if tau is None:
        tau = penalty(mesh, k, ip_factor)
    elems = np.arange(mesh.n_el)
    V, _ = _cell_tab(k)
    _, JxW, xq = cell_geometry(mesh, k, elems)
    b = (f(xq) * JxW) @ V
    for d in range(3):
        for s in range(2):
            bnd = np.array([e for e in elems if mesh.neighbor(e, d, s) < 0], dtype=np.int64)
            if not len(bnd):
                continue
            Vf, Gf = _face_tab(k, d, s)
            J, nrm, dA, xf = face_geometry(mesh, k, bnd, d, s)
            if mesh.bc[2 * d + s] == 0 and g is not None:
                dphi = np.einsum("efr,efri->efi", nrm, _grad_phys(J, Gf))
                gv = g(xf) * dA
                b[bnd] += -np.einsum("ef,efi->ei", gv, dphi) + 2.0 * tau[bnd][:, None] * (gv @ Vf)
            elif mesh.bc[2 * d + s] == 1 and h is not None:
                b[bnd] += (h(xf) * dA) @ Vf
    return b.ravel()


def interpolate(mesh, k, func):
    """Nodal DG vector of func at the mapped GLL nodes of each element."""
    g = basis.gll_nodes(k)
    x, _ = mesh.map(np.arange(mesh.n_el), g, g, g)
    return func(x).ravel()


def l2_error(mesh, k, u, func, extra=2):
    """|| u_h - func ||_{L2} with a (k+1+extra)-point Gauss rule."""
    n = k + 1
    m = n + extra
    z, w = basis.gauss(m)
    V, _ = basis.tabulate3(basis.gll_nodes(k), z, z, z)
    x, J = mesh.map(np.arange(mesh.n_el), z, z, z)
    JxW = np.abs(np.linalg.det(J)) * np.kron(w, np.kron(w, w))
    uh = np.asarray(u).reshape(mesh.n_el, n ** 3) @ V.T
    return float(np.sqrt(np.sum((uh - func(x)) ** 2 * JxW)))
