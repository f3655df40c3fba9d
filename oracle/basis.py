"""1-D bases and quadrature on the reference interval [0, 1].

Sec. 2 of the paper: shape functions are tensor products of 1-D Lagrange
polynomials of degree p on the Gauss-Lobatto-Legendre (GLL) nodes, the
reference element is [0,1]^d, and integrals use Gauss quadrature with p+1
points per direction.
"""
import numpy as np
from numpy.polynomial import legendre as L


def gll_nodes(k):
    """GLL nodes of degree k on [0,1]: the end points plus the roots of P'_k
    (the derivative of the Legendre polynomial of degree k), mapped from
    [-1,1].  Sec. 2 (nodal basis on Gauss-Lobatto-Legendre points)."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    interior = np.array([]) if k == 1 else np.sort(L.legroots(L.legder([0] * k + [1])).real)
    t = np.concatenate([[-1.0], interior, [1.0]])
    return 0.5 * (t + 1.0)


def gauss(n):
    """n-point Gauss-Legendre rule on [0,1] (points ascending, weights sum
    to 1).  Sec. 2: p+1 points per direction on cells and faces."""
    t, w = L.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """V[q, i] = l_i(x_q) for the Lagrange polynomials of ``nodes``, by the
    product formula l_i(x) = prod_{m != i} (x - x_m) / (x_i - x_m)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    for i in range(n):
        for m in range(n):
            if m != i:
                V[:, i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
    return V


def lagrange_derivatives(nodes, x):
    """D[q, i] = l_i'(x_q), by differentiating the product formula:
    l_i'(x) = sum_{r != i} 1/(x_i - x_r) prod_{m != i, r} (x - x_m)/(x_i - x_m)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for i in range(n):
        for r in range(n):
            if r == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[r]))
            for m in range(n):
                if m != i and m != r:
                    term *= (x - nodes[m]) / (nodes[i] - nodes[m])
            D[:, i] += term
    return D


def tabulate3(nodes, p1, p2, p3):
    """Values and reference gradients of the 3-D tensor basis
    N_{i1 i2 i3}(xi) = l_{i1}(xi_1) l_{i2}(xi_2) l_{i3}(xi_3) at the tensor grid
    p1 x p2 x p3 (Sec. 2, tensor-product shape functions).

    Point index = a + len(p1)*(b + len(p2)*c); basis index = i1 + n*(i2 + n*i3)
    (first coordinate fastest).  Returns (V, [G1, G2, G3]) with
    V[pt, i] = N_i and Gs[pt, i] = dN_i / dxi_s.
    """
    V1, V2, V3 = (lagrange_values(nodes, p) for p in (p1, p2, p3))
    D1, D2, D3 = (lagrange_derivatives(nodes, p) for p in (p1, p2, p3))
    V = np.kron(V3, np.kron(V2, V1))
    G = [np.kron(V3, np.kron(V2, D1)),
         np.kron(V3, np.kron(D2, V1)),
         np.kron(D3, np.kron(V2, V1))]
    return V, G
