"""Benchmark: PCG + hybrid multigrid solve on one MI355X.

Workload (default): the curvilinear cube of 48^3 elements, degree k = 7
(56,623,104 DoFs, x_i += 0.05 prod sin(pi x_j), cubic mapping), per-element
penalty scale ~ U[1, 10], Dirichlet boundary, seeded U[-1,1] right-hand
side.  One step = one full solve from x_0 = 0 to ||r||/||r_0|| <= 1e-10:
FP64 preconditioned CG (Alg. 1) with one V-cycle per iteration (Alg. 2) over
the hybrid hierarchy cph (DG7 -> FE7 -> FE3 -> FE1 -> h-coarsening to 3^3)
in FP32, Chebyshev(5) smoothing (Alg. 3) and an exact FP64 coarse solve;
PCG iterations are replayed from recorded HIP graphs (--no-graph: eager
launches, the same results bit for bit).  `value` is DoFs solved per second
(N * steps / time).  The FP64 and FP32 operator applies are timed on their
own with HIP events on the launch stream (operator_apply, roofline).

The plain FP64 solve (the same hierarchy with an FP64 V-cycle) is timed
after the timed region and reported beside it.  `roofline.traffic` (HBM
bytes per launch) and `roofline.fp64_flops` (executed FP64 arithmetic per
launch, timed with the same live launch duration) are read from the
committed counter summary of the workload's FP64 apply kernel
(profiles/op_kernel_<workload>_f64_pmc.md) when that summary was taken on
the current kernel source; else traffic is null and fp64_flops absent.

After the timed region, the workloads named by --also (default: the
curvilinear 64^3 mesh at k = 4, 32.8M DoFs) are reported as sub-blocks
(best of three solves), and the 64-mesh batch multi_64 (64 Cartesian unit
cubes with N_i^3 elements, N_i ~ U{4..24}, degree k_i ~ U{2..7}, 4 vectors
each) is applied under several launch schedules and reported as multi_mesh.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--also NAMES] [--no-cpu-baseline] [--no-plain-fp64]
                       [--no-multi] [--multi-only] [--learned-only] [--tables]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoF/s of SIPG operator apply (FP64/FP32); solve time per DoF at 1e-10 rel. residual"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6  # MI355X vector FP64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def apply_bytes(nel, k, prec_bytes, curved):
    """Algorithmic HBM bytes of one DG operator apply: read u, write v, the
    stored geometry (6 metric values per cell quadrature point, 7 values
    per face quadrature point on every face once) and tau per element."""
    Nx, Ny, Nz = nel
    n = k + 1
    ne = Nx * Ny * Nz
    dofs = ne * n ** 3
    b = 2 * dofs * prec_bytes + ne * prec_bytes
    if curved:
        faces = (Nx + 1) * Ny * Nz + Nx * (Ny + 1) * Nz + Nx * Ny * (Nz + 1)
        b += ne * 6 * n ** 3 * prec_bytes + faces * 7 * n * n * prec_bytes
    return b


# the sources the FP64 apply kernel is compiled from (hashed together)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1910_01900_amd", "csrc", f)
                  for f in ("op_body.h", "op_kernels.hip", "hmg_internal.h")]


def pmc_summary(workload):
    return os.path.join(ROOT, "profiles", "op_kernel_%s_f64_pmc.md" % workload)


def kernel_source_sha():
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _pmc_field(workload, name):
    """A per-launch figure of the FP64 apply kernel from the committed counter
    summary of this workload (profiles/op_kernel_<workload>_f64_pmc.md), or
    None when there is none or it was taken on a different kernel source."""
    path = pmc_summary(workload)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_sha256") != kernel_source_sha():
        return None
    try:
        return float(fields[name])
    except (KeyError, ValueError):
        return None


def measured_traffic(workload):
    """HBM bytes per launch (FETCH_SIZE / WRITE_SIZE passes)."""
    return _pmc_field(workload, "traffic_bytes_per_launch")


def measured_fp64_flops(workload):
    """Executed FP64 VALU flops per launch (SQ_INSTS_VALU_{FMA,MUL,ADD}_F64
    passes, times the active lanes per wavefront)."""
    return _pmc_field(workload, "fp64_flops_per_launch")


def time_applies(L, u, v, reps):
    import torch
    s = torch.cuda.current_stream()
    for _ in range(3):
        L.apply(u, v)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        L.apply(u, v)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps  # ms per apply


def time_applies_batched(L, nrhs, reps):
    """ms per batched launch of nrhs vectors (HIP events on the launch stream)."""
    import torch
    from paper_1910_01900_amd.inputs import uniform
    U = L.vectors(nrhs)
    for r in range(nrhs):
        U[r, :L.n_dofs] = torch.as_tensor(uniform(100 + r, L.n_dofs), dtype=L.dtype)
    V = L.vectors(nrhs)
    s = torch.cuda.current_stream()
    for _ in range(2):
        L.apply_batched(U, V)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        L.apply_batched(U, V)
    e1.record(s)
    e1.synchronize()
    del U, V
    return e0.elapsed_time(e1) / reps


def _event_ms(fn, reps, warm=2):
    """ms per call of fn() (HIP events on the current stream)."""
    import torch
    s = torch.cuda.current_stream()
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def multi_mesh_bench(prec, nrhs=4, reps=10, cheb_degree=5):
    """The multi_64 batch (64 Cartesian unit cubes, N ~ U{4..24}, k ~ U{2..7},
    nrhs vectors each): one batch apply under the default schedule (one
    launch per degree), the single launch over all meshes, the autotuned
    schedule, one batched launch per mesh and one launch per mesh and
    vector; the batched Chebyshev smoother against per-vector smoothing."""
    import ctypes as C
    import torch
    from paper_1910_01900_amd import hmg
    from paper_1910_01900_amd.inputs import multi_meshes
    spec = multi_meshes()
    levels = [hmg.Level(hmg.Mesh((N, N, N), k), prec=prec) for N, k in spec]
    B = hmg.Batch(levels, nrhs)
    g = torch.Generator(device="cuda").manual_seed(4)
    U = B.vector().uniform_(-1, 1, generator=g)
    V = B.vector()
    dofs = nrhs * sum(L.n_dofs for L in levels)
    lib, st = hmg.lib(), hmg.stream()
    es = U.element_size()
    out = {"meshes": len(levels), "nrhs": nrhs, "dofs": dofs}
    B.apply(U, V)
    out["default_ms"] = _event_ms(lambda: B.apply(U, V), reps)
    B.set_schedule(single=True)
    out["single_launch_ms"] = _event_ms(lambda: B.apply(U, V), reps)
    B.autotune(U, V, reps=3)
    out["autotuned_ms"] = _event_ms(lambda: B.apply(U, V), reps)
    out["schedule"] = B.schedule()

    def per_mesh():
        for i, L in enumerate(levels):
            o = B.offset[i] * es
            hmg.check(lib.hmg_operator_apply_batched(L._h, nrhs, C.c_void_p(U.data_ptr() + o),
                                                     C.c_void_p(V.data_ptr() + o), B.ld[i], st))

    def per_vector():
        for i, L in enumerate(levels):
            for r in range(nrhs):
                L.apply(B.view(U, i, r), B.view(V, i, r))
    out["per_mesh_batched_ms"] = _event_ms(per_mesh, reps)
    out["per_vector_ms"] = _event_ms(per_vector, max(2, reps // 2))
    for key in ("default_ms", "single_launch_ms", "autotuned_ms", "per_mesh_batched_ms", "per_vector_ms"):
        out[key.replace("_ms", "_dofs_per_s")] = dofs / (out[key] * 1e-3)
    # Chebyshev(degree) smoothing of every vector: batch vs per-vector calls
    lmax = [L.lambda_max() for L in levels]
    B.set_chebyshev(lmax, cheb_degree)
    X, T = B.vector(), B.vector()
    out["chebyshev_degree"] = cheb_degree
    out["chebyshev_batch_ms"] = _event_ms(lambda: B.chebyshev(U, X, T), max(2, reps // 2))

    def cheb_per_vector():
        for i, L in enumerate(levels):
            for r in range(nrhs):
                L.chebyshev(B.view(U, i, r), B.view(X, i, r), cheb_degree, lmax[i])
    out["chebyshev_per_vector_ms"] = _event_ms(cheb_per_vector, 2, warm=1)
    del B, U, V, X, T, levels
    torch.cuda.empty_cache()
    return out


def multi_solve_bench(nrhs=4, count=64):
    """The 64-mesh batch as a solve (multi_64: Cartesian unit cubes N_i^3,
    N_i ~ U{4..24}, k_i ~ U{2..7}, nrhs right-hand sides U[-1,1] each,
    streams 300 + 4 i + q): per mesh an FP64 PCG with an FP32 cph V-cycle to
    1e-10, the nrhs vectors solved together against one after another."""
    import torch
    from paper_1910_01900_amd import hmg
    from paper_1910_01900_amd.inputs import multi_meshes, uniform
    spec = multi_meshes(count)
    t0 = time.time()
    work = []
    for i, (N, k) in enumerate(spec):
        H = hmg.Hierarchy(hmg.Mesh((N, N, N), k), "cph", pseq=1, h_min=4, mg_prec=hmg.F32, max_rhs=nrhs)
        B = H.vectors(nrhs)
        for q in range(nrhs):
            B[q, :H.n_dofs] = torch.as_tensor(uniform(300 + 4 * i + q, H.n_dofs))
        work.append((H, B, H.vectors(nrhs)))
    log("multi_64 solve: %d hierarchies in %.1f s" % (len(work), time.time() - t0))
    dofs = nrhs * sum(H.n_dofs for H, _, _ in work)

    def batched():
        its = []
        for H, B, X in work:
            X.zero_()
            _, st = H.solve_batched(B, X, rtol=1e-10, maxit=200)
            its.append(max(s["iters"] for s in st))
        return its

    def sequential():
        for H, B, X in work:
            for q in range(nrhs):
                X[q].zero_()
                H.solve(B[q, :H.n_dofs], X[q, :H.n_dofs], rtol=1e-10, maxit=200)

    out = {"meshes": len(work), "nrhs": nrhs, "dofs": dofs}
    for name, fn in (("batched", batched), ("sequential", sequential)):
        fn()
        best = 1e30
        for _ in range(2):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t1)
            if name == "batched":
                out["max_iterations"] = max(r)
        out[name + "_ms"] = 1e3 * best
        out[name + "_ns_per_dof"] = 1e9 * best / dofs
    # every vector's final residual with the FP64 operator of its mesh
    worst = 0.0
    for H, B, X in work:
        L = hmg.Level(H.mesh, prec=hmg.F64)
        for q in range(nrhs):
            r = L.residual(B[q, :H.n_dofs], X[q, :H.n_dofs])
            worst = max(worst, float(torch.linalg.norm(r) / torch.linalg.norm(B[q, :H.n_dofs])))
    out["max_final_rel_residual"] = worst
    out["batched_vs_sequential_speedup"] = out["sequential_ms"] / out["batched_ms"]
    del work
    torch.cuda.empty_cache()
    return out


def tables_bench():
    """The paper's printed n10 tables (Tables 5-8, p = 1..7; the cited values
    in tests/golden/paper_tables_n10.json) re-run with the library's solver:
    per table, how many cases agree within 5% (continuous FE coarsest level)
    or stay at most 5% above the printed value (DG coarsest level, exact
    coarse solve against the paper's CG + AMG to 1e-3)."""
    from paper_1910_01900_amd import hmg
    path = os.path.join(ROOT, "tests", "golden", "paper_tables_n10.json")
    cases = [c for c in json.load(open(path))["cases"] if c["compare"] != "skip"]
    per = {}
    t0 = time.time()
    for i, c in enumerate(cases):
        N, k = c["N"], c["k"]
        mesh = hmg.Mesh((N, N, N), k, (-1.0,) * 3, (1.0,) * 3, c["curved"], 0.15 if c["curved"] else 0.0, 2,
                        (0,) * 6, c["ip"], None)
        H = hmg.Hierarchy(mesh, c["strategy"], pseq=c["pseq"], h_min=2, smoother_degree=5, mg_prec=hmg.F64)
        _, st = H.solve(hmg.Level(mesh).rhs_sine(3 * np.pi), rtol=1e-10, maxit=600)
        dev = (st["n10"] - c["n10"]) / c["n10"]
        ok = abs(dev) <= 0.05 if c["compare"] == "band" else dev <= 0.05
        t = per.setdefault(c["cite"].split("(")[0].strip(), {"cases": 0, "ok": 0, "max_abs_rel_dev_band": 0.0,
                                                             "min_rel_dev_upper": 0.0})
        t["cases"] += 1
        t["ok"] += int(ok)
        if c["compare"] == "band":
            t["max_abs_rel_dev_band"] = max(t["max_abs_rel_dev_band"], abs(dev))
        else:
            t["min_rel_dev_upper"] = min(t["min_rel_dev_upper"], dev)
        if (i + 1) % 50 == 0:
            log("tables: %d of %d cases (%.0f s)" % (i + 1, len(cases), time.time() - t0))
    return {"cases": len(cases), "ok": sum(t["ok"] for t in per.values()), "per_table": per,
            "seconds": time.time() - t0}


def learned_bench(samples=20480, steps=3000, batch=64, lr=1e-3, grid=16, h_min=12):
    """Learned coarse-grid correction on the curvilinear 48^3 mesh, k = 5
    (23.9M DoFs), hierarchy cph down to Q1 on h_min^3, FP32 V-cycle.
    h_min = 12 (2,197 coarse nodes): PCG with the exact (dense) coarse
    solve; h_min = 24 (15,625 nodes, no dense inverse): flexible CG with the
    iterative (Jacobi-PCG, 1e-3, at most 50 iterations) coarse solve.
    Against both: Chebyshev smoothing only on the coarsest level, and
    flexible CG with the learned correction (accepted while the coarse residual <= 0.5,
    else the exact or iterative solve).  Training pairs: the coarse
    right-hand sides of the V-cycles of seeded solves and their exact (FP64
    dense or CG to 1e-12) solves."""
    import torch
    from paper_1910_01900_amd import hmg
    from paper_1910_01900_amd.inputs import uniform
    mesh = hmg.Mesh((48, 48, 48), 5, deformed=True, amp=0.05)
    t0 = time.time()
    H = hmg.Hierarchy(mesh, "cph", pseq=1, h_min=h_min, smoother_degree=5, mg_prec=hmg.F32, max_rhs=8)
    info = H.coarse_info()
    log("learned: hierarchy in %.1f s, coarse nodes %s" % (time.time() - t0, info["nodes"]))
    N = H.n_dofs
    b = torch.as_tensor(uniform(3, N), device="cuda")

    def solve_ms(reps=3):
        x = torch.zeros_like(b)
        H.solve(b, x, rtol=1e-10, maxit=200)
        best, st = 1e30, None
        for _ in range(reps):
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, st = H.solve(b, x, rtol=1e-10, maxit=200)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        return 1e3 * best, st

    def vcycle_ms(reps=10):
        x = torch.zeros_like(b)
        return _event_ms(lambda: H.vcycle(b, x), reps)

    out = {"workload": "curved_k5_48", "dofs": N, "coarse_nodes": list(info["nodes"]), "coarse_unknowns": info["n"]}
    res = {}
    base = hmg.COARSE_EXACT if info["n"] <= 8192 else hmg.COARSE_CG
    for name, mode in (("exact" if base == hmg.COARSE_EXACT else "cg", base), ("smooth", hmg.COARSE_SMOOTH)):
        H.set_coarse(mode)
        ms, st = solve_ms()
        res[name] = {"solve_ms": ms, "iterations": st["iters"], "vcycle_ms": vcycle_ms()}
        log("learned: %s coarse solve: %.1f ms, %d iterations" % (name, ms, st["iters"]))
    H.set_coarse(base)
    # training pairs from the method's own V-cycles and exact coarse solves:
    # the coarse right-hand sides of batched solves of 8 seeded U[-1,1]
    # right-hand sides (drawn on the GPU, generator seed 1000 + solve)
    t0 = time.time()
    R = torch.zeros((samples, info["n"]), dtype=torch.float64, device="cuda")
    H.capture(R)
    k = 0
    B = H.vectors(8)
    while H.captured() < samples:
        g = torch.Generator(device="cuda").manual_seed(1000 + k)
        B[:, :N].uniform_(-1.0, 1.0, generator=g)
        H.solve_batched(B, rtol=1e-10, maxit=200)
        k += 1
        if k % 25 == 0:
            log("learned: %d of %d training pairs captured (%.0f s)" % (min(H.captured(), samples), samples,
                                                                       time.time() - t0))
    H.capture(None)
    del B
    t_capture = time.time() - t0
    E = torch.empty_like(R)
    for c0 in range(0, samples, 512):  # exact coarse solves (dense inverse, or FP64 CG to 1e-12)
        E[c0:c0 + 512] = H.coarse_solve_batch(R[c0:c0 + 512].contiguous())
        torch.cuda.synchronize()
        log("learned: exact coarse solves %d of %d (%.0f s)" % (min(c0 + 512, samples), samples, time.time() - t0))
    inp, tgt = H.learned_data(grid, R, E)
    torch.cuda.synchronize()
    t_data = time.time() - t0
    net = hmg.Net(grid=grid, max_batch=batch, seed=1)
    g = torch.Generator(device="cuda").manual_seed(2)
    ntrain = samples * 7 // 8
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        if i % 500 == 0:
            log("learned: training step %d of %d" % (i, steps))
        idx = torch.randint(0, ntrain, (batch,), device="cuda", generator=g)
        net.train_step(inp[idx].contiguous(), tgt[idx].contiguous(), lr if i < steps * 3 // 4 else lr / 4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    val, _ = net.gradient(inp[ntrain:ntrain + batch].contiguous(), tgt[ntrain:ntrain + batch].contiguous())
    one = inp[:1].contiguous()
    infer = _event_ms(lambda: net.forward(one), 20)
    H.set_coarse(hmg.COARSE_LEARNED, net, accept=0.5)
    f0 = H.coarse_stats()
    ms, st = solve_ms()
    fb = H.coarse_stats() - f0
    res["learned"] = {"solve_ms": ms, "iterations": st["iters"], "vcycle_ms": vcycle_ms(),
                      "fallbacks_in_timed_solves": fb, "solves": 4}
    log("learned: learned coarse solve: %.1f ms, %d iterations, %d fallbacks over 4 solves"
        % (ms, st["iters"], fb))
    out.update(res)
    out["training"] = {"pairs": samples, "data_s": t_data, "capture_s": t_capture, "capture_solves": k,
                       "steps": steps, "batch": batch,
                       "ms_per_step": 1e3 * t_train / steps, "validation_loss": val,
                       "inference_ms": infer}
    del H, net, R, E, inp, tgt
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, u_host, budget_s=15.0):
    """The oracle's element-wise apply (O(n^6) dense tabulations) on a
    bounded sample of elements of the same mesh, timed on the host."""
    from threadpoolctl import threadpool_info
    from oracle import sipg
    from oracle.mesh import BoxMesh
    k = w["degree"]
    from paper_1910_01900_amd.inputs import tau_scale
    n_el = int(np.prod(w["nel"]))
    ts = tau_scale(w["tau_scale_seed"], n_el) if w["tau_scale_seed"] is not None else None
    om = BoxMesh(tuple(w["nel"]), deform=w["amp"] if w["deformed"] else 0.0, tau_scale=ts)
    n_el = int(np.prod(w["nel"]))
    # probe on 64 elements, then one run sized to about budget_s seconds
    probe = np.arange(64) * (n_el // 64)
    t0 = time.perf_counter()
    sipg.apply(om, k, u_host, elems=probe)
    per_elem = (time.perf_counter() - t0) / 64
    count = int(min(n_el, max(64, budget_s / per_elem)))
    sel = np.arange(count) * (n_el // count)
    t0 = time.perf_counter()
    sipg.apply(om, k, u_host, elems=sel)
    elapsed = time.perf_counter() - t0
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    dofs = len(sel) * (k + 1) ** 3
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": dofs / elapsed, "unit": "DoF/s", "cores": int(min(threads, avail)), "kind": "oracle",
            "cpu_model": model, "host_cpus_available": int(avail), "blas_threads": int(threads),
            "sample": "FP64 operator apply (the oracle's dense element-wise quadrature) of %d elements spread "
                      "over the %s k=%d mesh (%d DoFs), %.1f s" % (len(sel), "x".join(map(str, w["nel"])), k, dofs,
                                                                   elapsed)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="curved_k7_48")
    ap.add_argument("--also", default="curved_k4_64",
                    help="comma-separated workloads reported as sub-blocks after the timed one ('' for none)")
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--rhs", type=int, default=None,
                    help="right-hand sides solved together per step (default: the workload's, 8 for curved_k7_48)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-fp64", action="store_true", help="skip the plain FP64 V-cycle solve")
    ap.add_argument("--nrhs", type=int, default=8, help="vectors per batched apply (0: skip)")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="launch every kernel eagerly instead of replaying recorded PCG iterations and V-cycles")
    ap.add_argument("--no-multi", action="store_true", help="skip the 64-mesh batch (multi_64)")
    ap.add_argument("--multi-only", action="store_true", help="only time the 64-mesh batch (multi_64)")
    ap.add_argument("--tables", action="store_true",
                    help="only re-run the paper's printed n10 tables (Tables 5-8, p <= 7) and summarise")
    ap.add_argument("--learned-only", action="store_true",
                    help="only the learned coarse-grid correction on curved_k5_48")
    ap.add_argument("--solve-only", action="store_true",
                    help="only the warm-up and timed solve steps of the workload (for kernel traces of the solve)")
    ap.add_argument("--learned-case", choices=["both", "12", "24"], default="both",
                    help="coarse level of the learned correction: Q1 on 12^3 (dense exact solve) or 24^3 (iterative)")
    ap.add_argument("--apply-only", choices=["f64", "f32"], default=None,
                    help="only time the operator apply (and a 1 GiB copy used to calibrate "
                         "HBM counters); for profiling")
    a = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (a.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_01900_amd import hmg
    from paper_1910_01900_amd.inputs import WORKLOADS, tau_scale, uniform

    w = WORKLOADS[a.workload]
    k = w["degree"]
    n_el = int(np.prod(w["nel"]))
    ts = tau_scale(w["tau_scale_seed"], n_el) if w["tau_scale_seed"] is not None else None
    mesh = hmg.Mesh(tuple(w["nel"]), k, deformed=w["deformed"], amp=w["amp"], tau_scale=ts)
    torch.cuda.set_device(0)

    if a.tables:
        print(json.dumps(tables_bench()), flush=True)
        return

    if a.learned_only:
        res = {}
        if a.learned_case in ("both", "12"):
            res["coarse_12"] = learned_bench()
        if a.learned_case in ("both", "24"):
            res["coarse_24"] = learned_bench(samples=4096, steps=3000, batch=32, grid=32, h_min=24)
        print(json.dumps(res), flush=True)
        return

    if a.multi_only:
        res = {}
        for name, prec in (("fp64", hmg.F64), ("fp32", hmg.F32)):
            res[name] = multi_mesh_bench(prec)
            log("multi_64 %s:" % name, json.dumps(res[name]))
        res["solve"] = multi_solve_bench()
        log("multi_64 solve:", json.dumps(res["solve"]))
        print(json.dumps({"workload": "multi_64", **res}), flush=True)
        return

    if a.apply_only:
        prec = hmg.F64 if a.apply_only == "f64" else hmg.F32
        L = hmg.Level(mesh, prec=prec)
        u = L.vector(uniform(1, L.n_dofs))
        v = L.vector()
        ms = time_applies(L, u, v, a.apply_reps)
        msb = time_applies_batched(L, a.nrhs, max(3, a.apply_reps // 4)) if a.nrhs > 1 else None
        src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)  # the first copy is the one the counter calibration reads
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(5):
            dst.copy_(src)
        c1.record()
        c1.synchronize()
        copy_gbs = 2 * (1 << 30) * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
        nb = apply_bytes(w["nel"], k, 8 if prec == hmg.F64 else 4, w["deformed"])
        print(json.dumps({"workload": a.workload, "prec": a.apply_only, "ms_per_apply": ms,
                          "dofs_per_s": L.n_dofs / (ms * 1e-3), "algorithmic_bytes": nb,
                          "achieved_GBs": nb / (ms * 1e-3) / 1e9, "calibration_copy_bytes": 1 << 30,
                          "device_copy_GBs": copy_gbs, "nrhs": a.nrhs,
                          "batched_ms": msb, "batched_dofs_per_s": (a.nrhs * L.n_dofs / (msb * 1e-3)) if msb else None}))
        return

    res = run_workload(a, a.workload, hmg, timed=True)
    if a.solve_only:
        print(json.dumps({"workload": a.workload, **res}), flush=True)
        return
    out = {
        "metric": METRIC,
        "value": res["value"],
        "value_is": "solve throughput: DoFs solved to 1e-10 relative residual per second (FP64 PCG, FP32 "
                    "V-cycle; a step solves the workload's right-hand sides together, 8 for curved_k7_48), "
                    "over the timed steps; operator-apply DoF/s in operator_apply",
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (outer CG) / f32 (V-cycle)",
        "data": "synthetic",
        "config": res["config"],
    }
    for key in ("solve_batched", "solve", "solve_plain_fp64", "operator_apply", "operator_apply_batched", "roofline"):
        if key in res:
            out[key] = res[key]
    if a.also:
        for name in a.also.split(","):
            if name and name != a.workload:
                log("sub-block", name)
                sub = run_workload(a, name, hmg, timed=False)
                out.setdefault("other_workloads", {})[name] = sub
    if not a.no_multi:
        torch.cuda.empty_cache()
        multi = {}
        for name, prec in (("fp64", hmg.F64), ("fp32", hmg.F32)):
            multi[name] = multi_mesh_bench(prec)
            m = multi[name]
            log("multi_64 %s: %d meshes x %d vectors, %.1f M DoFs: default %.2f ms, single launch %.2f ms, "
                "autotuned %.2f ms (%.1f GDoF/s), per mesh %.2f ms, per vector %.2f ms; Chebyshev(%d) batch "
                "%.2f ms vs per vector %.2f ms"
                % (name, m["meshes"], m["nrhs"], m["dofs"] / 1e6, m["default_ms"], m["single_launch_ms"],
                   m["autotuned_ms"], m["autotuned_dofs_per_s"] / 1e9, m["per_mesh_batched_ms"],
                   m["per_vector_ms"], m["chebyshev_degree"], m["chebyshev_batch_ms"],
                   m["chebyshev_per_vector_ms"]))
        out["multi_mesh"] = {"workload": "multi_64", **multi}
        out["multi_mesh"]["solve"] = multi_solve_bench()
        log("multi_64 solve:", json.dumps(out["multi_mesh"]["solve"]))
    if not a.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(WORKLOADS[a.workload], res["u_host"])
    print(json.dumps(out), flush=True)


def coarse_description(levels):
    """'exact FP64, FE1 3^3' style text from the hierarchy's coarsest level."""
    c = levels[-1]
    nel = c["nel"]
    mesh = ("%d^3" % nel[0]) if nel[0] == nel[1] == nel[2] else "x".join(map(str, nel))
    solver = "exact FP64 (dense inverse)" if c["n_dofs"] <= 8192 else "FP64 Jacobi-PCG to 1e-3"
    return "%s, %s%d %s (%d unknowns)" % (solver, c["space"], c["degree"], mesh, c["n_dofs"])


def run_workload(a, name, hmg, timed):
    """Setup, solves and operator applies of one workload.  timed: the
    contract's timed region (warm-up solves, then exactly `steps` solves
    bracketed by synchronisations); otherwise the best of three solves."""
    import torch
    from paper_1910_01900_amd.inputs import WORKLOADS, rhs_block, tau_scale, uniform
    w = WORKLOADS[name]
    k = w["degree"]
    n_el = int(np.prod(w["nel"]))
    ts = tau_scale(w["tau_scale_seed"], n_el) if w["tau_scale_seed"] is not None else None
    mesh = hmg.Mesh(tuple(w["nel"]), k, deformed=w["deformed"], amp=w["amp"], tau_scale=ts)
    nrhs = w["nrhs"] if a.rhs is None else a.rhs
    t0 = time.time()
    log("setup: hierarchy cph (FP32 V-cycle) for", name)
    H = hmg.Hierarchy(mesh, "cph", pseq=1, h_min=4, smoother_degree=5, mg_prec=hmg.F32, graph=a.graph,
                      max_rhs=nrhs)
    levels = H.levels()
    log("setup done in %.1f s; levels:" % (time.time() - t0), [(l["space"], l["degree"], l["nel"][0]) for l in levels])
    N = H.n_dofs
    b = torch.as_tensor(uniform(3, N), device="cuda")
    x = torch.zeros_like(b)
    steps, warmup = (a.steps, a.warmup) if timed else (3, 1)
    if nrhs > 1:  # the step: nrhs right-hand sides solved together
        B = H.vectors(nrhs)
        for q, v in enumerate(rhs_block(N, nrhs)):
            B[q, :N] = torch.as_tensor(v)
        X = H.vectors(nrhs)

        def step():
            X.zero_()
            _, sts = H.solve_batched(B, X, rtol=1e-10, maxit=100)
            return sts
    else:
        def step():
            x.zero_()
            _, st = H.solve(b, x, rtol=1e-10, maxit=100)
            return [st]
    for i in range(warmup):
        sts = step()
        log("warmup step %d: iterations %s" % (i, [st["iters"] for st in sts]))
    torch.cuda.synchronize()
    times, stats = [], None
    t_start = time.perf_counter()
    for i in range(steps):
        t1 = time.perf_counter()
        stats = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        log("step %d: %.1f ms, iterations %s" % (i, times[-1] * 1e3, [st["iters"] for st in stats]))
    total = time.perf_counter() - t_start
    if not timed:
        total = min(times) * steps
    res = {"value": nrhs * N * steps / total, "ms_per_step": 1e3 * total / steps}
    if a.solve_only:
        res["iterations"] = [st["iters"] for st in stats]
        return res
    if nrhs > 1:
        # the same right-hand sides one after another, and the single solve of stream 3
        Xs = H.vectors(nrhs)
        seq = []
        for rep in range(2):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for q in range(nrhs):
                Xs[q].zero_()
                H.solve(B[q, :N], Xs[q, :N], rtol=1e-10, maxit=100)
            torch.cuda.synchronize()
            seq.append(time.perf_counter() - t1)
        r64 = hmg.Level(mesh, prec=hmg.F64)
        rel = []
        for q in range(nrhs):
            r = r64.residual(B[q, :N], X[q, :N])
            rel.append(float(torch.linalg.norm(r) / torch.linalg.norm(B[q, :N])))
        del r64, r
        res["solve_batched"] = {
            "nrhs": nrhs, "ms": res["ms_per_step"], "ns_per_dof_per_rhs": 1e6 * res["ms_per_step"] / (nrhs * N),
            "sequential_ms": 1e3 * min(seq), "batched_vs_sequential_speedup": 1e3 * min(seq) / res["ms_per_step"],
            "iterations": [st["iters"] for st in stats], "n10": [st["n10"] for st in stats],
            "final_rel_residual": rel, "rhs": "U[-1,1], streams 200..%d" % (199 + nrhs)}
        log("batched %d RHS: %.1f ms, sequential %.1f ms, residuals max %.2e"
            % (nrhs, res["ms_per_step"], 1e3 * min(seq), max(rel)))
        del B, X, Xs
        x.zero_()
        t1 = time.perf_counter()
        _, st1 = H.solve(b, x, rtol=1e-10, maxit=100)
        torch.cuda.synchronize()
        single_s = time.perf_counter() - t1
        x.zero_()
        t1 = time.perf_counter()
        _, st1 = H.solve(b, x, rtol=1e-10, maxit=100)
        torch.cuda.synchronize()
        single_s = min(single_s, time.perf_counter() - t1)
        stats = [st1]
    else:
        single_s = total / steps
    res["single_ms"] = 1e3 * single_s
    del H
    torch.cuda.empty_cache()
    res["config"] = {"workload": name, "mesh": "x".join(map(str, w["nel"])), "degree": k,
                     "curved": w["deformed"], "penalty_scale": "U[1,10] per element" if ts is not None else "1",
                     "dofs": N, "strategy": "cph", "p_sequence": "floor(p/2)",
                     "levels": ["%s%d %s" % (l["space"], l["degree"], "x".join(map(str, l["nel"]))) for l in levels],
                     "smoother": "Chebyshev(5)", "coarse": coarse_description(levels), "rtol": 1e-10,
                     "rhs_per_step": nrhs,
                     "parallelism": "single GPU", "graph": a.graph}
    if not a.no_plain_fp64:
        # plain FP64: the same hierarchy with every level in FP64
        H64 = hmg.Hierarchy(mesh, "cph", pseq=1, h_min=4, smoother_degree=5, mg_prec=hmg.F64, graph=a.graph)
        x64 = torch.zeros_like(b)
        _, st64 = H64.solve(b, x64, rtol=1e-10, maxit=100)  # warm-up
        torch.cuda.synchronize()
        t64 = []
        for _ in range(max(1, min(steps, 3))):
            x64.zero_()
            t1 = time.perf_counter()
            _, st64 = H64.solve(b, x64, rtol=1e-10, maxit=100)
            torch.cuda.synchronize()
            t64.append(time.perf_counter() - t1)
        res["solve_plain_fp64"] = {"ns_per_dof": 1e9 * min(t64) / N, "ms": 1e3 * min(t64),
                                   "iterations": st64["iters"], "n10": st64["n10"]}
        log("plain FP64 solve: %.1f ms, %d iterations" % (1e3 * min(t64), st64["iters"]))
        del H64, x64
        torch.cuda.empty_cache()

    # final residual recomputed with the FP64 operator
    L64 = hmg.Level(mesh, prec=hmg.F64)
    r = L64.residual(b, x)
    rel = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    log("final relative residual %.3e" % rel)
    st = stats[0]
    res["solve"] = {"ms": res["single_ms"], "ns_per_dof": 1e6 * res["single_ms"] / N, "rhs": "U[-1,1], stream 3",
                    "iterations": st["iters"], "n10": st["n10"], "rho": st["rho"], "final_rel_residual": rel}
    if "solve_plain_fp64" in res:
        res["solve"]["mixed_vs_plain_fp64_speedup"] = res["solve_plain_fp64"]["ms"] / res["single_ms"]

    # operator applies, timed with HIP events on the launch stream
    u = L64.vector(uniform(1, L64.n_dofs))
    v = L64.vector()
    ms64 = time_applies(L64, u, v, a.apply_reps)
    res["u_host"] = u.cpu().numpy() if (timed and not a.no_cpu_baseline) else None
    del u, v, r, b, x
    L32 = hmg.Level(mesh, prec=hmg.F32)
    u32 = L32.vector(uniform(1, L32.n_dofs))
    v32 = L32.vector()
    ms32 = time_applies(L32, u32, v32, a.apply_reps)
    del u32, v32
    if a.nrhs > 1:
        msb32 = time_applies_batched(L32, a.nrhs, 5)
        del L32
        torch.cuda.empty_cache()
        msb64 = time_applies_batched(L64, a.nrhs, 5)
        res["operator_apply_batched"] = {
            "nrhs": a.nrhs, "fp64_ms": msb64, "fp32_ms": msb32,
            "fp64_dofs_per_s": a.nrhs * N / (msb64 * 1e-3), "fp32_dofs_per_s": a.nrhs * N / (msb32 * 1e-3)}
        log("batched apply, %d vectors: FP64 %.3f ms, FP32 %.3f ms" % (a.nrhs, msb64, msb32))
    else:
        del L32
    del L64
    torch.cuda.empty_cache()
    bytes64 = apply_bytes(w["nel"], k, 8, w["deformed"])
    achieved = bytes64 / (ms64 * 1e-3) / 1e9
    log("apply FP64 %.3f ms (%.2f GDoF/s, %.0f GB/s), FP32 %.3f ms (%.2f GDoF/s)"
        % (ms64, N / ms64 / 1e6, achieved, ms32, N / ms32 / 1e6))
    res["operator_apply"] = {"fp64_dofs_per_s": N / (ms64 * 1e-3), "fp32_dofs_per_s": N / (ms32 * 1e-3),
                             "fp64_ms": ms64, "fp32_ms": ms32,
                             "fp32_achieved_GBs": apply_bytes(w["nel"], k, 4, w["deformed"]) / (ms32 * 1e-3) / 1e9}
    res["roofline"] = {"kernel": "op_kernel<%d,double,%s,DG,APPLY>" % (k + 1, "curved" if w["deformed"] else "affine"),
                       "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": achieved / PEAK_HBM_GBS, "traffic": measured_traffic(name),
                       "algorithmic_bytes_per_launch": bytes64}
    flops = measured_fp64_flops(name)
    if flops is not None:  # executed FP64 arithmetic of the same kernel, same live timing
        tf = flops / (ms64 * 1e-3) / 1e12
        res["roofline"]["fp64_flops"] = {"achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                         "frac": tf / PEAK_FP64_TFLOPS, "per_launch": flops}
    if not timed:
        res.pop("u_host", None)
    return res

if __name__ == "__main__":
    main()
