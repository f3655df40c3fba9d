"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
comparisons.  Random numbers only: nothing here computes any part of the
method.  Seeds follow numpy.random.default_rng(20191004 + i).

Workloads (the paper's cube test case, Sec. 5.3, on [0,1]^3 with Dirichlet
conditions; curvilinear meshes move every coordinate by
amp * prod_j sin(pi s_j) and use a degree-3 mapping):
  cube_k3_8      Cartesian 8^3, k = 3 (32,768 DoFs)
  curved_k4_64   curvilinear 64^3, k = 4 (32,768,000 DoFs), amp 0.05
  curved_k7_48   curvilinear 48^3, k = 7 (56,623,104 DoFs), amp 0.05,
                 per-element penalty scale ~ U[1, 10] (stream 5), 8 right-hand
                 sides U[-1,1] solved together (streams 200..207)
  multi_64       64 Cartesian unit cubes of N_i^3 elements, N_i ~ U{4..24},
                 degree k_i ~ U{2..7} (stream 4), 4 vectors U[-1,1] each
"""
import numpy as np

BASE_SEED = 20191004


def rng(i):
    return np.random.default_rng(BASE_SEED + i)


def uniform(i, n, lo=-1.0, hi=1.0):
    """n FP64 values ~ U[lo, hi) from stream i."""
    return rng(i).uniform(lo, hi, int(n))


WORKLOADS = {
    "cube_k3_8": dict(nel=(8, 8, 8), degree=3, deformed=False, amp=0.0, tau_scale_seed=None, nrhs=1),
    "curved_k4_64": dict(nel=(64, 64, 64), degree=4, deformed=True, amp=0.05, tau_scale_seed=None, nrhs=1),
    "curved_k7_48": dict(nel=(48, 48, 48), degree=7, deformed=True, amp=0.05, tau_scale_seed=5, nrhs=8),
    "curved_k5_48": dict(nel=(48, 48, 48), degree=5, deformed=True, amp=0.05, tau_scale_seed=None, nrhs=1),
    # Cartesian meshes of the same sizes (no stored geometry): the affine
    # kernels that the batches of unit cubes run
    "cartesian_k4_64": dict(nel=(64, 64, 64), degree=4, deformed=False, amp=0.0, tau_scale_seed=None, nrhs=1),
    "cartesian_k7_48": dict(nel=(48, 48, 48), degree=7, deformed=False, amp=0.0, tau_scale_seed=None, nrhs=1),
}


def rhs_block(n, nrhs, first=200):
    """nrhs right-hand sides of n values ~ U[-1,1] from streams first, first+1, ..."""
    return [uniform(first + q, n) for q in range(nrhs)]


def tau_scale(seed_index, n_el):
    """Per-element penalty factors ~ U[1, 10]."""
    return rng(seed_index).uniform(1.0, 10.0, int(n_el))


def multi_meshes(count=64, seed_index=4, n_range=(4, 24), k_range=(2, 7)):
    """(N_i, k_i) of a batch of unit cubes: N_i ~ U{n_range}, k_i ~ U{k_range}."""
    g = rng(seed_index)
    N = g.integers(n_range[0], n_range[1] + 1, int(count))
    k = g.integers(k_range[0], k_range[1] + 1, int(count))
    return [(int(a), int(b)) for a, b in zip(N, k)]
