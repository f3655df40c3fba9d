"""Pins of the oracle's 1-D bases against closed forms (Sec. 2: GLL nodal
basis, (k+1)-point Gauss quadrature)."""
import numpy as np
import pytest

from oracle import basis
from oracle.rng import splitmix64, uniform_pm1


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_exactness_closed_form(n):
    z, w = basis.gauss(n)
    # exact for x^m, m <= 2n-1: integral over [0,1] = 1/(m+1)
    for m in range(2 * n):
        assert abs(np.sum(w * z ** m) - 1.0 / (m + 1)) < 1e-14
    # the error for x^(2n) is the classical closed form (n!)^4 / ((2n+1) ((2n)!)^2)
    from math import factorial
    err = 1.0 / (2 * n + 1) - np.sum(w * z ** (2 * n))
    assert abs(err - factorial(n) ** 4 / ((2 * n + 1) * factorial(2 * n) ** 2)) < 1e-14


def test_gll_textbook_values():
    s5 = 1.0 / np.sqrt(5.0)
    s37 = np.sqrt(3.0 / 7.0)
    assert np.allclose(basis.gll_nodes(1), [0, 1], atol=1e-15)
    assert np.allclose(basis.gll_nodes(2), [0, 0.5, 1], atol=1e-15)
    assert np.allclose(basis.gll_nodes(3), [0, (1 - s5) / 2, (1 + s5) / 2, 1], atol=1e-15)
    assert np.allclose(basis.gll_nodes(4), [0, (1 - s37) / 2, 0.5, (1 + s37) / 2, 1], atol=1e-15)


@pytest.mark.parametrize("k", range(1, 9))
def test_gll_quadrature_exactness(k):
    # GLL weights 2/(k(k+1) P_k(t)^2) on [-1,1]; rule exact to degree 2k-1.
    x = basis.gll_nodes(k)
    t = 2 * x - 1
    Pk = np.polynomial.legendre.legval(t, [0] * k + [1])
    w = 2.0 / (k * (k + 1) * Pk ** 2) / 2.0
    for m in range(2 * k):
        assert abs(np.sum(w * x ** m) - 1.0 / (m + 1)) < 1e-13


@pytest.mark.parametrize("k", range(1, 9))
def test_lagrange_identities(k):
    x = basis.gll_nodes(k)
    z, _ = basis.gauss(k + 1)
    assert np.allclose(basis.lagrange_values(x, x), np.eye(k + 1), atol=1e-14)
    S = basis.lagrange_values(x, z)
    D = basis.lagrange_derivatives(x, z)
    assert np.allclose(S.sum(axis=1), 1.0, atol=1e-13)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-11)
    # exact differentiation of monomials of degree <= k
    for m in range(k + 1):
        assert np.allclose(D @ x ** m, m * z ** max(m - 1, 0) if m else 0 * z, atol=1e-11)
    # even-odd symmetry of the point sets
    n = k + 1
    assert np.allclose(S[::-1, ::-1], S, atol=1e-13)
    assert np.allclose(D[::-1, ::-1], -D, atol=1e-11)


def test_tabulate3_tensor_structure():
    k = 2
    x = basis.gll_nodes(k)
    p = np.array([0.1, 0.7])
    V, G = basis.tabulate3(x, p, p, p)
    # point (a,b,c) = (1,0,1), basis (i1,i2,i3) = (2,1,0)
    pt = 1 + 2 * (0 + 2 * 1)
    bi = 2 + 3 * (1 + 3 * 0)
    l = basis.lagrange_values(x, p)
    dl = basis.lagrange_derivatives(x, p)
    assert abs(V[pt, bi] - l[1, 2] * l[0, 1] * l[1, 0]) < 1e-15
    assert abs(G[0][pt, bi] - dl[1, 2] * l[0, 1] * l[1, 0]) < 1e-14
    assert abs(G[2][pt, bi] - l[1, 2] * l[0, 1] * dl[1, 0]) < 1e-14


def test_splitmix64_published_outputs():
    # SplitMix64 seeded with 1234567: first outputs as published with the
    # reference implementation (Vigna, prng.di.unimi.it/splitmix64.c).
    z = splitmix64(1234567, 3)
    assert [int(v) for v in z] == [6457827717110365317, 3203168211198807973, 9817491932198370423]
    u = uniform_pm1(7, 1000)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.1
