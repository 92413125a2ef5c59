"""Host-side behaviour of bench.py (no GPU): the one-GPU rule and the
traffic lookup that ties counter summaries to the kernel sources and plan."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_for_the_profiled_sources_and_plan(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    h = bench.kernel_source_hash()
    (prof / "traffic_k_fused_staged_d3q19_256_fp32.md").write_text(
        "# HBM traffic: k_fused_staged, d3q19_256, fp32 storage, plan rows:64:4:86:10\n"
        f"traffic_bytes_per_launch: 2.5e+09\nsource_hash: {h}\n")
    (prof / "traffic_k_fused_staged_d3q19_512_fp16.md").write_text(
        "# HBM traffic: k_fused_staged, d3q19_512_fp16, fp16 storage, plan rows:64:4:86:10\n"
        "traffic_bytes_per_launch: 1e+10\nsource_hash: 0000000000000000\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    rows = {"kernel": 3, "tile_x": 64, "tile_y": 4, "tile_z": 86, "graph_steps": 20}
    assert bench.read_traffic("k_fused_staged", "d3q19_256", "fp32", rows) == 2.5e9
    # another tile, another kernel or other sources: no traffic
    assert bench.read_traffic("k_fused_staged", "d3q19_256", "fp32", dict(rows, tile_z=43)) is None
    assert bench.read_traffic("k_fused_staged", "d3q19_256", "fp32", dict(rows, kernel=2)) is None
    assert bench.read_traffic("k_fused_staged", "d3q19_512_fp16", "fp16", rows) is None
    assert bench.read_traffic("k_fused", "d3q19_256", "fp32", rows) is None


def test_source_hash_ignores_comments_only():
    a = "int f(int x) { // twice\n  return 2 * x; /* doubled */ }\n"
    b = "int f(int x) {\n    // the double of x\n    return 2 * x;\n}\n"
    c = "int f(int x) { return 3 * x; }\n"
    assert bench.code_of(a) == bench.code_of(b)
    assert bench.code_of(a) != bench.code_of(c)


def test_paper_model_traffic_only_for_its_own_sources(tmp_path, monkeypatch):
    """The per-step traffic of the paper's-model workloads is keyed by the
    hash of that model's kernel sources (not the force model's) and, on
    D3Q19, by the plan it was measured on."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    h_eq = bench.kernel_source_hash(names=bench.PAPER_MODEL_SOURCES["eq"])
    h_2d = bench.kernel_source_hash(names=bench.PAPER_MODEL_SOURCES["d2q9"])
    assert len({h_eq, h_2d, bench.kernel_source_hash()}) == 3
    rows = {"kernel": 3, "tile_x": 64, "tile_y": 4, "tile_z": 86, "graph_steps": 20}
    split = {"kernel": 0, "tile_x": 0, "tile_y": 0, "tile_z": 0, "graph_steps": 20}
    assert bench.paper_model_kernels("eq", rows) == ("k_meq_staged",)
    assert bench.paper_model_kernels("eq", split) == ("k_density", "k_meq_collide")
    (prof / "traffic_k_meq_staged_d3q19_256_eq.md").write_text(
        f"# HBM traffic: plan rows:64:4:86\ntraffic_bytes_per_step: 2.9e+09\nsource_hash: {h_eq}\n")
    (prof / "traffic_k_meq_collide_d3q19_256_eq.md").write_text(
        f"# HBM traffic: plan split:0:0:0\ntraffic_bytes_per_step: 4.1e+09\nsource_hash: {h_eq}\n")
    (prof / "traffic_k2_step_tiled_d2q9_2048.md").write_text(
        f"traffic_bytes_per_step: 5.2e+08\nsource_hash: {h_eq}\n")  # another model's hash
    real = bench.kernel_source_hash
    csrc = os.path.join(ROOT, "paper_1202_4748_amd", "csrc")
    monkeypatch.setattr(bench, "kernel_source_hash",
                        lambda csrc_=None, names=bench.STEP_KERNEL_SOURCES: real(csrc, names))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    k_rows, k_split = bench.paper_model_kernels("eq", rows), bench.paper_model_kernels("eq", split)
    assert bench.read_step_traffic("eq", "d3q19_256_eq", k_rows, rows) == 2.9e9
    assert bench.read_step_traffic("eq", "d3q19_256_eq", k_rows, dict(rows, tile_z=43)) is None
    assert bench.read_step_traffic("eq", "d3q19_256_eq", k_split, split) == 4.1e9
    k2 = bench.paper_model_kernels("d2q9", None)
    assert bench.read_step_traffic("d2q9", "d2q9_2048", k2) is None
    assert bench.read_step_traffic("d2q9", "d2q9_256", k2) is None  # no summary


def test_paper_model_workloads_are_complete():
    import workloads
    for name, wl in workloads.WORKLOADS.items():
        if "model" in wl:
            assert wl["model"] in bench.PAPER_MODEL, name
            assert {"L", "steps", "a", "b", "kappa", "rho_c", "kT", "tau", "init_sigma"} <= set(wl), name


def test_valu_busy_only_for_the_profiled_sources_and_plan(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    real = bench.kernel_source_hash
    csrc = os.path.join(ROOT, "paper_1202_4748_amd", "csrc")
    h = real(csrc, bench.STEP_KERNEL_SOURCES)
    (prof / "valu_k_fused_staged_d3q19_256_fp32.md").write_text(
        f"# VALU use: k_fused_staged, plan rows:64:4:86\nvalu_busy: 0.5756\nsource_hash: {h}\n")
    (prof / "valu_k2_step_tiled_d2q9_2048.md").write_text(f"valu_busy: 0.83\nsource_hash: {h}\n")
    monkeypatch.setattr(bench, "kernel_source_hash",
                        lambda csrc_=None, names=bench.STEP_KERNEL_SOURCES: real(csrc, names))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rows = {"kernel": 3, "tile_x": 64, "tile_y": 4, "tile_z": 86, "graph_steps": 10}
    assert bench.read_valu_busy("k_fused_staged", "d3q19_256_fp32", bench.STEP_KERNEL_SOURCES, rows) == 0.5756
    assert bench.read_valu_busy("k_fused_staged", "d3q19_256_fp32", bench.STEP_KERNEL_SOURCES,
                                dict(rows, tile_z=43)) is None
    # another model's sources, or no summary
    assert bench.read_valu_busy("k2_step_tiled", "d2q9_2048", bench.PAPER_MODEL_SOURCES["d2q9"]) is None
    assert bench.read_valu_busy("k_meq_staged", "d3q19_256_eq", bench.PAPER_MODEL_SOURCES["eq"], rows) is None
