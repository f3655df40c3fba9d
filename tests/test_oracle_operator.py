"""Pins of the oracle's SIPG operator against facts the mathematics fixes
(Sec. 2 weak form, fluxes, mirror boundary conditions, penalty; Sec. 4
reference-element integrals).  None of these re-types the oracle's formulas:
the 1-D SIPG matrices below are assembled independently on a 1-D mesh."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import basis, fe, sipg
from oracle.mesh import BoxMesh, cell_geometry, face_geometry


def sipg_1d(N, h, k, tau, bc_lo, bc_hi):
    """Independent 1-D SIPG stiffness K and DG mass M on N elements of size h
    (textbook interior penalty in 1-D: the 'face' is a point, the normal of
    the left element is +1)."""
    n = k + 1
    x = basis.gll_nodes(k)
    z, w = basis.gauss(n)
    S = basis.lagrange_values(x, z)
    Dp = basis.lagrange_derivatives(x, z) / h
    Ke = Dp.T @ (w[:, None] * Dp) * h
    Me = S.T @ (w[:, None] * S) * h
    v0 = basis.lagrange_values(x, [0.0])[0]
    v1 = basis.lagrange_values(x, [1.0])[0]
    d0 = basis.lagrange_derivatives(x, [0.0])[0] / h
    d1 = basis.lagrange_derivatives(x, [1.0])[0] / h
    K = np.zeros((N * n, N * n))
    M = np.zeros((N * n, N * n))
    for e in range(N):
        sl = slice(e * n, (e + 1) * n)
        K[sl, sl] += Ke
        M[sl, sl] += Me
    for e in range(N - 1):
        # left element e (value v1, derivative d1), right element e+1 (v0, d0)
        jump = np.concatenate([v1, -v0])
        avg = 0.5 * np.concatenate([d1, d0])
        blk = -np.outer(avg, jump) - np.outer(jump, avg) + tau * np.outer(jump, jump)
        sl = slice(e * n, (e + 2) * n)
        K[sl, sl] += blk
    if bc_lo == 0:   # outward normal -1 at x = 0
        K[:n, :n] += -np.outer(-d0, v0) - np.outer(v0, -d0) + 2 * tau * np.outer(v0, v0)
    if bc_hi == 0:
        sl = slice((N - 1) * n, N * n)
        K[sl, sl] += -np.outer(d1, v1) - np.outer(v1, d1) + 2 * tau * np.outer(v1, v1)
    return K, M


@pytest.mark.parametrize("k", [1, 2, 3])
def test_kronecker_structure_cartesian(k):
    """P2: on a Cartesian box with a uniform penalty the SIPG matrix is
    K_x (x) M_y (x) M_z + M_x (x) K_y (x) M_z + M_x (x) M_y (x) K_z."""
    nel = (3, 2, 2)
    lo, hi = (0.0, -1.0, 0.5), (1.5, 1.0, 1.0)
    bc = (1, 0, 0, 0, 0, 1)
    mesh = BoxMesh(nel, lo, hi, bc=bc)
    n = k + 1
    tau = 7.3
    A = sipg.assemble(mesh, k, tau=np.full(mesh.n_el, tau)).toarray()
    h = [(hi[d] - lo[d]) / nel[d] for d in range(3)]
    KM = [sipg_1d(nel[d], h[d], k, tau, bc[2 * d], bc[2 * d + 1]) for d in range(3)]
    (Kx, Mx), (Ky, My), (Kz, Mz) = KM
    Akron = np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx))
    # permutation DG element-major -> grid order (gx fastest)
    perm = np.zeros(mesh.n_el * n ** 3, dtype=int)
    Gx, Gy = nel[0] * n, nel[1] * n
    for e in range(mesh.n_el):
        ex, ey, ez = mesh.coords(e)
        for l in range(n):
            for j in range(n):
                for i in range(n):
                    perm[e * n ** 3 + i + n * (j + n * l)] = (ex * n + i) + Gx * ((ey * n + j) + Gy * (ez * n + l))
    Aperm = np.zeros_like(A)
    Aperm[np.ix_(perm, perm)] = A
    assert np.abs(Aperm - Akron).max() < 1e-12 * np.abs(Akron).max()


@pytest.mark.parametrize("deform", [0.0, 0.12])
@pytest.mark.parametrize("ip", [1.0, 10.0, 1000.0])
def test_symmetric_positive_definite(deform, ip):
    """P3 + P4: A = A^T and lambda_min(A) > 0, Cartesian and curved."""
    mesh = BoxMesh((2, 2, 3), deform=deform, waves=2, bc=(0, 1, 0, 0, 1, 0))
    A = sipg.assemble(mesh, 2, ip_factor=ip)
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


@pytest.mark.parametrize("deform", [0.0, 0.1])
@pytest.mark.parametrize("k", [1, 3])
def test_neumann_null_space(deform, k):
    """P5: with Neumann conditions everywhere, constants are in the kernel."""
    mesh = BoxMesh((2, 3, 2), deform=deform, waves=2, bc=(1,) * 6)
    A = sipg.assemble(mesh, k)
    one = np.ones(A.shape[0])
    ref = abs(A) @ one
    assert np.abs(A @ one).max() < 1e-13 * ref.max()


@pytest.mark.parametrize("poly", ["x", "xy", "x2-y2", "xyz"])
def test_harmonic_consistency(poly):
    """P5: for a harmonic polynomial u in Q_k, rows of elements with no
    boundary face vanish (Galerkin consistency of the interior fluxes)."""
    k = 3
    mesh = BoxMesh((3, 3, 3), lo=(0, 0, 0), hi=(1.5, 1.2, 0.9))
    f = {"x": lambda X: X[..., 0],
         "xy": lambda X: X[..., 0] * X[..., 1],
         "x2-y2": lambda X: X[..., 0] ** 2 - X[..., 1] ** 2,
         "xyz": lambda X: X[..., 0] * X[..., 1] * X[..., 2]}[poly]
    u = sipg.interpolate(mesh, k, f)
    v = sipg.apply(mesh, k, u)
    centre = mesh.index(1, 1, 1)
    assert np.abs(v[centre]).max() < 1e-12 * np.abs(v).max()
    assert np.abs(v).max() > 1e-3


def test_patch_test_reproduces_polynomial():
    """P6: u in Q_k with its Dirichlet data and f = -lap u is reproduced."""
    k = 2
    mesh = BoxMesh((2, 3, 2), lo=(0, 0, 0), hi=(1.0, 1.5, 0.8), bc=(0, 1, 0, 0, 0, 1))
    uex = lambda X: X[..., 0] ** 2 + X[..., 1] * X[..., 2] - 0.5 * X[..., 2] ** 2 + 1.0
    f = lambda X: -(2.0 - 1.0) + 0 * X[..., 0]
    # Neumann data h = grad u . n on x=hi (n=+x) and z=hi (n=+z)
    def hfun(X):
        out = np.zeros(X.shape[:-1])
        on_x = np.isclose(X[..., 0], 1.0)
        on_z = np.isclose(X[..., 2], 0.8)
        out[on_x] = 2 * X[..., 0][on_x]
        out[on_z] = X[..., 1][on_z] - X[..., 2][on_z]
        return out
    A = sipg.assemble(mesh, k)
    b = sipg.rhs(mesh, k, f, g=uex, h=hfun)
    u = spla.spsolve(A.tocsc(), b)
    assert np.abs(u - sipg.interpolate(mesh, k, uex)).max() < 1e-10


@pytest.mark.parametrize("k,deform", [(2, 0.0), (2, 0.05), (3, 0.0), (3, 0.05)])
def test_convergence_order(k, deform):
    """P7: manufactured u = prod sin(2 pi x_j): L2 error order >= k+1-0.3."""
    uex = lambda X: np.prod(np.sin(2 * np.pi * X), axis=-1)
    f = lambda X: 12 * np.pi ** 2 * uex(X)
    errs = []
    Ns = (2, 4, 8) if k == 2 else (2, 4)
    for N in Ns:
        mesh = BoxMesh((N, N, N), deform=deform)
        A = sipg.assemble(mesh, k)
        b = sipg.rhs(mesh, k, f, g=uex)
        u = spla.spsolve(A.tocsc(), b)
        errs.append(sipg.l2_error(mesh, k, u, uex))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] >= k + 1 - 0.3, (errs, rates)


def test_curved_geometry_invariants():
    """P8: watertight Q3 mapping, unit boundary normals along the axes,
    total volume 1 for the deformed unit cube."""
    mesh = BoxMesh((3, 3, 3), deform=0.05)
    k = 4
    elems = np.arange(mesh.n_el)
    _, JxW, _ = cell_geometry(mesh, k, elems)
    assert abs(JxW.sum() - 1.0) < 1e-12
    for d in range(3):
        left = np.array([e for e in elems if mesh.neighbor(e, d, 1) >= 0])
        right = np.array([mesh.neighbor(e, d, 1) for e in left])
        _, nL, dAL, xL = face_geometry(mesh, k, left, d, 1)
        _, nR, dAR, xR = face_geometry(mesh, k, right, d, 0)
        assert np.abs(xL - xR).max() < 1e-14
        assert np.abs(nL + nR).max() < 1e-13
        assert np.abs(dAL - dAR).max() < 1e-13
        for s in range(2):
            bnd = np.array([e for e in elems if mesh.neighbor(e, d, s) < 0])
            _, nb, _, _ = face_geometry(mesh, k, bnd, d, s)
            ref = np.zeros(3)
            ref[d] = 2 * s - 1
            assert np.abs(nb - ref).max() < 1e-13


def test_zero_amplitude_is_affine():
    """P8: amplitude 0 gives the Cartesian operator (constant Jacobian)."""
    k = 2
    a = sipg.assemble(BoxMesh((2, 2, 2), deform=0.0), k)
    b = sipg.assemble(BoxMesh((2, 2, 2), deform=1e-30), k)
    assert abs(a - b).max() < 1e-12 * abs(a).max()
    Jinvt, JxW, _ = cell_geometry(BoxMesh((2, 2, 2)), k)
    assert np.allclose(Jinvt, np.broadcast_to(2 * np.eye(3), Jinvt.shape), atol=1e-13)


@pytest.mark.parametrize("deform", [0.0, 0.1])
def test_diagonal_and_elementwise_apply_match_assembly(deform):
    """P9 and O5/O6: diag and the element-wise apply equal the assembled
    matrix (cell-based view vs face-loop assembly), per-element tau scale."""
    mesh = BoxMesh((3, 2, 2), deform=deform, waves=2, bc=(0, 1, 0, 0, 1, 0),
                   tau_scale=np.linspace(1, 10, 12))
    k = 3
    A = sipg.assemble(mesh, k)
    u = np.random.default_rng(3).uniform(-1, 1, A.shape[0])
    assert np.abs(A @ u - sipg.apply(mesh, k, u).ravel()).max() < 1e-13 * np.abs(A @ u).max()
    assert np.abs(A.diagonal() - sipg.diagonal(mesh, k)).max() < 1e-13 * A.diagonal().max()
    sub = np.array([4, 7])
    vs = sipg.apply(mesh, k, u, elems=sub)
    nd = (k + 1) ** 3
    for r, e in enumerate(sub):
        assert np.abs(vs[r] - (A @ u)[e * nd:(e + 1) * nd]).max() < 1e-13 * np.abs(A @ u).max()


def test_penalty_closed_form():
    """tau_e on a Cartesian cube of size h: 3(k+1)^2/h inside, 3.5(k+1)^2/h
    with one boundary face, 4(k+1)^2/h with two, 4.5(k+1)^2/h with three."""
    k = 3
    mesh = BoxMesh((4, 4, 4))
    tau = sipg.penalty(mesh, k)
    h = 0.25
    c = (k + 1) ** 2 / h
    assert abs(tau[mesh.index(1, 2, 1)] - 3.0 * c) < 1e-12 * c
    assert abs(tau[mesh.index(0, 2, 1)] - 3.5 * c) < 1e-12 * c
    assert abs(tau[mesh.index(0, 3, 1)] - 4.0 * c) < 1e-12 * c
    assert abs(tau[mesh.index(0, 0, 3)] - 4.5 * c) < 1e-12 * c


def test_fe_operator_properties():
    """Continuous Q_k operator: symmetric, identity on constrained rows,
    kernel of constants under all-Neumann, and equal to the DG cell form on
    continuous functions (a(phi,u) summed over shared nodes)."""
    k = 2
    mesh = BoxMesh((2, 3, 2), deform=0.08, waves=2, bc=(0, 1, 0, 0, 1, 0))
    A = fe.assemble(mesh, k)
    assert abs(A - A.T).max() < 1e-13 * abs(A).max()
    free = fe.free_mask(mesh, k)
    Ad = A.toarray()
    assert np.allclose(Ad[free == 0][:, free == 0], np.eye(int((free == 0).sum())))
    assert np.abs(Ad[free == 0][:, free == 1]).max() == 0
    assert np.linalg.eigvalsh(Ad).min() > 0
    An = fe.assemble(BoxMesh((2, 2, 2), deform=0.08, waves=2, bc=(1,) * 6), k)
    assert np.abs(An @ np.ones(An.shape[0])).max() < 1e-12 * abs(An).max()


def test_exact_mapping_geometry():
    """mapping_degree 0 (the analytic deformation instead of its cubic
    interpolant): the Jacobian equals central differences of the map; the
    map equals the cubic one at the 4^3 support points and is watertight
    with unit axis normals on the boundary; the deformed box keeps volume 1
    (to quadrature accuracy: det J is not a polynomial); amplitude 0 gives
    the Cartesian geometry."""
    m0 = BoxMesh((3, 2, 2), deform=0.08, waves=2, mapping_degree=0)
    m3 = BoxMesh((3, 2, 2), deform=0.08, waves=2)
    el = np.arange(m0.n_el)
    g = basis.gll_nodes(3)
    assert np.abs(m0.map(el, g, g, g)[0] - m3.map(el, g, g, g)[0]).max() < 1e-15
    z = np.array([0.1, 0.37, 0.8])
    _, J = m0.map(el, z, z, z)
    for c in range(3):
        zp, zm = [z, z, z], [z, z, z]
        zp[c], zm[c] = z + 1e-6, z - 1e-6
        fd = (m0.map(el, *zp)[0] - m0.map(el, *zm)[0]) / 2e-6
        assert np.abs(fd - J[..., :, c]).max() < 1e-8
    _, JxW, _ = cell_geometry(BoxMesh((3, 3, 3), deform=0.05, mapping_degree=0), 9)
    assert abs(JxW.sum() - 1.0) < 1e-9
    mesh = BoxMesh((3, 3, 3), deform=0.05, mapping_degree=0)
    for d in range(3):
        left = np.array([e for e in range(mesh.n_el) if mesh.neighbor(e, d, 1) >= 0])
        right = np.array([mesh.neighbor(e, d, 1) for e in left])
        _, nL, dAL, xL = face_geometry(mesh, 3, left, d, 1)
        _, nR, dAR, xR = face_geometry(mesh, 3, right, d, 0)
        assert np.abs(xL - xR).max() < 1e-14 and np.abs(nL + nR).max() < 1e-13
        bnd = np.array([e for e in range(mesh.n_el) if mesh.neighbor(e, d, 0) < 0])
        _, nb, _, _ = face_geometry(mesh, 3, bnd, d, 0)
        ref = np.zeros(3)
        ref[d] = -1
        assert np.abs(nb - ref).max() < 1e-13
    a = sipg.assemble(BoxMesh((2, 2, 2)), 2)
    b = sipg.assemble(BoxMesh((2, 2, 2), mapping_degree=0), 2)
    assert abs(a - b).max() < 1e-12 * abs(a).max()


def test_exact_mapping_operator_properties():
    """The SIPG matrix on the exactly mapped curvilinear mesh: symmetric,
    positive definite with Dirichlet faces, A 1 = 0 with all-Neumann faces
    (P3-P5 for mapping_degree 0), and h^(k+1) convergence (P7)."""
    mesh = BoxMesh((2, 2, 2), deform=0.08, mapping_degree=0)
    A = sipg.assemble(mesh, 2).toarray()
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T))[0] > 0
    An = sipg.assemble(BoxMesh((2, 2, 2), deform=0.08, mapping_degree=0, bc=(1,) * 6), 2)
    one = np.ones(An.shape[0])
    assert np.abs(An @ one).max() <= 1e-12 * (abs(An) @ one).max()
    uex = lambda X: np.prod(np.sin(2 * np.pi * X), axis=-1)
    f = lambda X: 12 * np.pi ** 2 * uex(X)
    errs = []
    for N in (2, 4, 8):
        m = BoxMesh((N, N, N), deform=0.05, mapping_degree=0)
        u = spla.spsolve(sipg.assemble(m, 2).tocsc(), sipg.rhs(m, 2, f, g=uex))
        errs.append(sipg.l2_error(m, 2, u, uex))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] >= 3 - 0.3, (errs, rates)
