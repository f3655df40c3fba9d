"""Parity at the benchmark sizes: the full operator runs on the GPU in the
launch configuration the benchmark times; the oracle recomputes sampled
elements one by one (corners, edges, faces, interior, random)."""
import numpy as np
import pytest

from gpu_helpers import meshes, to_np
from oracle import sipg
from paper_1910_01900_amd import hmg
from paper_1910_01900_amd.inputs import WORKLOADS, tau_scale, uniform

pytestmark = pytest.mark.gpu


def _samples(nel, count, seed):
    Nx, Ny, Nz = nel
    n = Nx * Ny * Nz
    corners = [0, Nx - 1, Nx * Ny - 1, n - 1, n - Nx * Ny, (Nz // 2) * Nx * Ny + (Ny // 2) * Nx + Nx // 2]
    rnd = np.random.default_rng(seed).choice(n, count, replace=False)
    return np.unique(np.concatenate([corners, rnd]))


@pytest.mark.parametrize("name,prec", [("cube_k3_8", hmg.F64), ("curved_k4_64", hmg.F64),
                                       ("curved_k4_64", hmg.F32), ("curved_k7_48", hmg.F64),
                                       ("curved_k7_48", hmg.F32)])
def test_fullsize_apply_sampled(name, prec):
    w = WORKLOADS[name]
    k = w["degree"]
    n_el = int(np.prod(w["nel"]))
    ts = tau_scale(w["tau_scale_seed"], n_el) if w["tau_scale_seed"] is not None else None
    hm, om = meshes(w["nel"], k, w["deformed"], amp=w["amp"], tau_scale=ts)
    print("fullsize", name, "prec", prec, flush=True)
    L = hmg.Level(hm, prec=prec)
    u = uniform(1, L.n_dofs)
    if prec == hmg.F32:
        u = u.astype(np.float32).astype(np.float64)
    v = L.apply(L.vector(u))
    import torch
    torch.cuda.synchronize()
    sel = _samples(w["nel"], 24, 3)
    nd = (k + 1) ** 3
    idx = (sel[:, None] * nd + np.arange(nd)[None, :]).ravel()
    got = to_np(v[torch.as_tensor(idx, device="cuda")]).reshape(len(sel), nd)
    ref = sipg.apply(om, k, u, elems=sel)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("sampled rel err %.3e" % err)
    assert err < (1e-12 if prec == hmg.F64 else 1e-5)
    assert np.isfinite(to_np(v)).all()
