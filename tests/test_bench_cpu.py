"""CPU: the benchmark's output contract. The compact stdout record keeps the
required keys (metric, value, unit, roofline, cpu_baseline, ...) and stays
under the line cap whatever the extra sections hold; --gpus above 1 exits
with a message (one GPU per run); the traffic lookup refuses counters taken
on other kernel sources."""
import json
import pathlib
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def _result(n_extra):
    kern = lambda us, b: dict(avg_us=us, algorithmic_bytes=b, gbs=b / (us * 1e-6) / 1e9,
                              elements_per_s=2**20 / (us * 1e-6), model_gflops=1e4)
    res = {key: None for key in ("vs_baseline",)}
    res.update(metric=bench.METRIC, value=6.1e10, unit="elements/s", n_gpus=1, steps=100, warmup=5,
               ms_per_step=0.0171, higher_is_better=True, scaling="weak", dtype="f32", data="synthetic",
               config={"workload": "3D variable-coefficient Laplacian, P1 tetrahedra, 2^20 elements",
                       "n_elem": 2**20, "n_vert": 274625},
               model_gflops=4.9e4,
               kernels={"fem_integrate_residual_mesh": kern(16.8, 73699864.0),
                        "fem_integrate_residual": kern(17.1, 92274688.0),
                        "fem_geometry": kern(16.7, 65000000.0)},
               roofline={"bound": "hbm", "kernel": "fem_integrate_residual_mesh", "achieved": 4390.0,
                         "peak": 8000.0, "unit": "GB/s", "frac": 0.549, "traffic": 72364921,
                         "algorithmic_bytes_per_launch": 73699864.0, "achievable_gbs": 6428.0,
                         "frac_of_achievable": 0.68, "achievable_gbs_same_bytes": 5317.0},
               two_call_step={"elements_per_s": 3.0e10, "ms_per_step": 0.0349},
               hot_step={"elements_per_s": 6.9e10, "ms_per_step": 0.0152, "note": "information only"},
               cpu_baseline={"value": 8.7e7, "unit": "elements/s", "cores": 16, "kind": "oracle",
                             "sample": "all elements of the step workload on 16 threads",
                             "single_thread": {"value": 6.6e6}})
    extra = {"fp64_step": dict(elements_per_s=4.2e10, ms_per_step=0.0248, fused_us=24.3, fused_gbs=5100.0,
                               integrate_us=33.9, integrate_gbs=5440.0),
             "adjoint_laplace3d_2p21_f32": dict(us=46.9, frac_of_peak=0.67),
             "batched_64_meshes_f32": dict(graph_replay_us=162.7, graph_replay_elements_per_s=5.5e10,
                                           graph_replay_gbs=5057.0, separate_launches_in_a_graph_us=305.7,
                                           speedup_vs_separate=1.88)}
    for tag in ("elasticity2d_2p22_f32", "elasticity3d_2p21_f32", "elasticity2d_2p22_f64",
                "elasticity3d_2p21_f64"):
        extra[f"{tag}_integrate"] = dict(elements_per_s=3e10, frac_of_peak=0.68)
    for i in range(n_extra):   # many strategy and P3 sections, to exercise the size cap
        extra[f"strategies_workload{i}"] = dict(lane_us=17.5, transpose_us=28.9, shuffle_us=24.5)
        extra[f"w{i}_p3_f32_integrate"] = dict(us=50.0, mfma_us=80.0, copy_same_bytes_us=41.7)
    res["extra"] = extra
    res["extra_file"] = "gpurun_out/bench_extra.json"
    return res


@pytest.mark.parametrize("n_extra", [0, 2, 200])
def test_compact_line_contract(n_extra):
    line = bench.compact(_result(n_extra))
    text = json.dumps(line)
    assert len(text) <= bench.MAX_LINE
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in line, key
    assert line["config"]["workload"].startswith("3D variable-coefficient Laplacian")
    rf = line["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in rf, key
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], rel=1e-3)
    cb = line["cpu_baseline"]
    assert (cb["kind"], cb["unit"], cb["cores"]) == ("oracle", "elements/s", 16) and cb["sample"]
    assert line["n_gpus"] == 1 and line["higher_is_better"] is True and line["vs_baseline"] is None


def test_compact_line_carries_the_yardsticks():
    """The rows-streamed yardsticks (fused kernel, geometry, adjoint) and a
    strategy section without the quad-permutation form reach the compact
    line with their ratios; absent, they are left out."""
    res = _result(0)
    res["roofline"].update(same_rows_us=15.7, frac_of_rows=15.7 / 16.8)
    res["kernels"]["fem_geometry"].update(stream_rows=[6, 10], stream_rows_us=14.5)
    res["extra"]["adjoint_laplace3d_2p21_f32"].update(stream_rows_us=48.0, frac_of_stream_rows=48.0 / 46.9)
    res["extra"]["strategies_elasticity3d_2p21_f32"] = dict(lane_us=62.4, transpose_us=67.7)
    line = bench.compact(res)
    assert line["roofline"]["same_rows_us"] == 15.7
    assert line["roofline"]["frac_of_rows"] == pytest.approx(15.7 / 16.8, rel=1e-3)
    assert line["geometry_only"]["frac_of_rows"] == pytest.approx(14.5 / 16.7, rel=1e-3)
    assert line["adjoint"]["frac_of_rows"] == pytest.approx(48.0 / 46.9, rel=1e-3)
    el = line["transposition"]["elasticity3d_2p21_f32"]
    assert el == {"lane_us": 62.4, "lds_us": 67.7}
    plain = bench.compact(_result(0))
    assert "frac_of_rows" not in plain["roofline"] and "frac_of_rows" not in plain["geometry_only"]
    assert "frac_of_rows" not in plain["adjoint"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_needs_matching_sources(monkeypatch):
    rec = json.loads((ROOT / "profiles" / "traffic.json").read_text())
    key = "fem_integrate_residual_mesh:laplace3d_2p20_f32"
    assert key in rec
    want = rec[key]
    got = bench.measured_traffic("fem_integrate_residual_mesh", "laplace3d_2p20_f32")
    if want["source_hash"] == bench.source_hash(bench.KERNEL_SOURCES["fem_integrate_residual_mesh"]):
        assert got == want["bytes_per_launch"]
    else:
        assert got is None
    # counters taken on other kernel sources are not used, matching ones are
    monkeypatch.setattr(bench, "source_hash", lambda files: "0" * 16)
    assert bench.measured_traffic("fem_integrate_residual_mesh", "laplace3d_2p20_f32") is None
    monkeypatch.setattr(bench, "source_hash", lambda files: want["source_hash"])
    assert bench.measured_traffic("fem_integrate_residual_mesh", "laplace3d_2p20_f32") == want["bytes_per_launch"]
    assert bench.measured_traffic("fem_integrate_residual_mesh", "no_such_workload") is None
