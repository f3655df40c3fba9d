"""Host logic of bench.py: the algorithmic byte count of the curvilinear
apply, the source-gated reading of the committed counter summary, and the
refusal of more than one GPU."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_apply_bytes_curved_k4_64():
    # u and v (2 x 32,768,000 x 8 B), tau per element, 6 metric values per
    # cell point (125 per element), 7 values per face point (25 per face) on
    # the 3 x 65 x 64 x 64 faces
    nel, k = (64, 64, 64), 4
    ne, dofs, faces = 64 ** 3, 64 ** 3 * 125, 3 * 65 * 64 * 64
    expect = 2 * dofs * 8 + ne * 8 + ne * 6 * 125 * 8 + faces * 7 * 25 * 8
    assert bench.apply_bytes(nel, k, 8, True) == expect == 3217457152
    assert bench.apply_bytes(nel, k, 4, True) * 2 == expect
    # Cartesian: only u, v and tau
    assert bench.apply_bytes(nel, k, 8, False) == 2 * dofs * 8 + ne * 8


def _summary(path, sha, traffic="4255016947", flops="10542489600"):
    with open(path, "w") as f:
        f.write("# summary\n\n| quantity | value |\n|---|---|\n| x | 1 |\n\n")
        f.write("- traffic_bytes_per_launch: %s\n" % traffic)
        if flops is not None:
            f.write("- fp64_flops_per_launch: %s\n" % flops)
        f.write("- kernel_source_sha256: `%s`\n" % sha)


def test_counter_summary_is_read_only_for_the_current_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "pmc_summary", lambda w: str(tmp_path / ("op_kernel_%s_f64_pmc.md" % w)))
    p = bench.pmc_summary("curved_k7_48")
    _summary(p, bench.kernel_source_sha())
    assert bench.measured_traffic("curved_k7_48") == 4255016947.0
    assert bench.measured_fp64_flops("curved_k7_48") == 10542489600.0
    # each workload reads its own summary: none for this one
    assert bench.measured_traffic("curved_k4_64") is None
    # a summary taken on another kernel source is ignored
    _summary(p, "0" * 64)
    assert bench.measured_traffic("curved_k7_48") is None
    assert bench.measured_fp64_flops("curved_k7_48") is None
    # missing or malformed fields
    _summary(p, bench.kernel_source_sha(), traffic="n/a", flops=None)
    assert bench.measured_traffic("curved_k7_48") is None
    assert bench.measured_fp64_flops("curved_k7_48") is None


def test_summary_path_is_keyed_by_workload():
    assert bench.pmc_summary("curved_k7_48").endswith(os.path.join("profiles", "op_kernel_curved_k7_48_f64_pmc.md"))


def test_coarse_description_from_the_hierarchy():
    lv = [{"space": "DG", "degree": 7, "nel": (48, 48, 48), "n_dofs": 56623104},
          {"space": "FE", "degree": 1, "nel": (3, 3, 3), "n_dofs": 64}]
    assert bench.coarse_description(lv) == "exact FP64 (dense inverse), FE1 3^3 (64 unknowns)"
    lv[-1] = {"space": "FE", "degree": 1, "nel": (24, 24, 24), "n_dofs": 15625}
    assert bench.coarse_description(lv).startswith("FP64 Jacobi-PCG")


def test_kernel_source_sha_tracks_the_kernel_sources():
    names = sorted(os.path.basename(p) for p in bench.KERNEL_SOURCES)
    assert names == ["hmg_internal.h", "op_body.h", "op_kernels.hip"]
    assert all(os.path.exists(p) for p in bench.KERNEL_SOURCES)
    assert len(bench.kernel_source_sha()) == 64


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr
