"""CPU: bench.py's host-side bookkeeping -- the measured-traffic file is
used only for the workload and the kernel sources it was measured on, and
the --gpus guard refuses more than one GPU."""
import json
import os
import subprocess
import sys

import bench
from paper_2311_15439_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_tied_to_workload_and_sources(tmp_path, monkeypatch):
    # a traffic file written for the image workload with the current sources
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic{}.json"))
    path = tmp_path / "trafficimage2d.json"
    rec = {"sources_sha256": bench._sources_digest(), "workload": inputs.IMAGE_2D.name,
           "kernels": {"bin_accum_adam": {"bytes": 123.0}}}
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("bin_accum_adam", inputs.IMAGE_2D.name) == 123.0
    assert bench.measured_traffic("bin_accum_adam", inputs.VOLUME_3D.name) is None
    assert bench.measured_traffic("bin_scatter", inputs.IMAGE_2D.name) is None
    # sources changed since the counters were taken
    rec["sources_sha256"] = "0" * 64
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("bin_accum_adam", inputs.IMAGE_2D.name) is None
    # no file
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing{}.json"))
    assert bench.measured_traffic("bin_accum_adam", inputs.IMAGE_2D.name) is None


def test_write_traffic_from_request_sizes(tmp_path, monkeypatch):
    hdr = "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
    acc = '"void spx::bin_accum_kernel<2, 2, true>(x)"'
    # the accum kernel of two steps, then the calibration copy
    rd = hdr
    for d, n128 in ((5, 100), (9, 200)):
        rd += f"{d},{acc},TCC_EA0_RDREQ_128B_sum,{n128}\n{d},{acc},TCC_EA0_RDREQ_64B_sum,3\n" \
              f"{d},{acc},TCC_EA0_RDREQ_32B_sum,1\n"
    rd += f'12,"spx::cast_kernel(y)",TCC_EA0_RDREQ_128B_sum,{bench.COPY_ELEMS * 4 // 128}\n'
    wr = hdr + f"5,{acc},WRITE_SIZE,50\n9,{acc},WRITE_SIZE,60\n" \
        + f'12,"spx::cast_kernel(y)",WRITE_SIZE,{bench.COPY_ELEMS * 2 / 1024.0}\n'
    (tmp_path / "r.csv").write_text(rd)
    (tmp_path / "w.csv").write_text(wr)
    out = tmp_path / "timage2d.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "t{}.json"))
    bench.write_traffic(str(tmp_path / "r.csv"), str(tmp_path / "w.csv"), inputs.IMAGE_2D.name)
    t = json.loads(out.read_text())
    k = t["kernels"]["bin_accum_adam"]
    # the last dispatch: 128-, 64- and 32-byte requests; WRITE_SIZE in KiB
    assert k["read_bytes"] == 200 * 128 + 3 * 64 + 32 and k["written_bytes"] == 60 * 1024
    assert k["bytes"] == k["read_bytes"] + k["written_bytes"]
    c = t["copy_check"]
    assert c["read_bytes"] == c["read_expected"] and c["written_bytes"] == c["written_expected"]
    assert t["workload"] == inputs.IMAGE_2D.name


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_expected_unique_and_wave_lines():
    import numpy as np
    assert bench.expected_unique(1, 64) == 1.0
    assert abs(bench.expected_unique(1e12, 64) - 64.0) < 1e-6
    # 2 lines, 2 draws: 1 + 1/2 expected distinct
    assert abs(bench.expected_unique(2, 2) - 1.5) < 1e-12
    # one wave of 64 points, 2 levels, 3 vertices; 4-byte rows, 32 rows per 128-byte line
    idx = np.zeros((64, 2, 3), np.uint32)
    idx[:, 0, :] = 5                                   # level 0: one line for the whole wave
    idx[:, 1, 0] = np.arange(64) * 32                  # level 1: vertex 0 on 64 lines,
    idx[:, 1, 1] = np.arange(64) * 32 + 1              # vertex 1 on the same lines,
    idx[:, 1, 2] = 64 * 32 + np.arange(64) * 32        # vertex 2 on 64 others
    u = bench.wave_unique_lines(idx, 20, 4)
    assert list(u) == [1.0, 128.0]


def test_line_rate_and_ceiling():
    probe = {1 << 12: 4e11, 1 << 20: 2e11, 1 << 28: 1e11}
    # beyond the measured range the end values hold; large buffers: every gather its own line
    assert abs(bench.line_rate(probe, 2.0 ** 30) - 1e11 * bench.expected_unique(2 ** 28 / 128, 64) / 64) < 1
    # interpolation in log2 of the size
    mid = bench.line_rate(probe, 2.0 ** 24)
    assert abs(mid - 1.5e11 * bench.expected_unique(2 ** 24 / 128, 64) / 64) < 1e3
    # a 4 KiB buffer has 32 lines: a wave's 64 gathers hit about 28 of them
    small = bench.line_rate(probe, 2.0 ** 12)
    assert abs(small - 4e11 * bench.expected_unique(32, 64) / 64) < 1
    ms = bench.gather_ceiling_ms(6400, [64.0, 32.0], [2.0 ** 28, 2.0 ** 28], probe)
    r = bench.line_rate(probe, 2.0 ** 28)
    assert abs(ms - 1e3 * 100 * 96 / r) < 1e-9


def test_footprints():
    # a coarse level whose 18^2 box is far below T: ~324 lines; a fine level: every line of T
    f = bench.level_footprints([16.0, 1e6], 1.0, 2, 20, 4, False)
    assert abs(f[0] / bench.LINE_BYTES - bench.expected_unique((1 << 20) * 4 / 128, 18 ** 2)) < 1e-9
    assert abs(f[1] - (1 << 20) * 4 * (1 - (1 - 128 / ((1 << 20) * 4)) ** (1 << 20))) < 1.0


def _fake_detail():
    cell = {"fwd": {"median_ms": 0.35}, "fwd_bwd": {"median_ms": 1.1}, "fwd_points_per_s": 3.0e9,
            "fwd_bwd_points_per_s": 9.1e8, "fwd_gather_frac": 0.61, "fwd_bwd_gather_frac": 0.4}
    sweep = {w: {"simplex": dict(cell), "grid": dict(cell)} for w in
             [inputs.IMAGE_2D.name, inputs.VOLUME_3D.name] + [inputs.sweep_workload(n).name for n in range(2, 7)]}
    acc = {"simplex": {"psnr_db": 22.8}, "simplex_equal_memory": {"psnr_db": 22.9}, "grid": {"psnr_db": 23.1},
           "simplex_minus_grid_db": -0.3, "simplex_equal_memory_minus_grid_db": -0.2}
    return {
        "ms_per_step": 1.652,
        "config": {"workload": inputs.IMAGE_2D.name},
        "roofline": {"bound": "hbm", "kernel": "bin_accum_adam", "achieved": 5150.123456, "peak": 8000.0,
                     "unit": "GB/s", "frac": 0.6437654, "traffic": 3.943e9, "avg_ms": 0.766, "bytes_per_launch": 3.94e9},
        "cpu_baseline": {"value": 5960.0, "unit": "points/s", "cores": 16, "kind": "oracle", "sample": "x" * 300,
                         "cpu_model": "AMD EPYC 9575F 64-Core Processor", "build": "gcc -O3 -march=native"},
        "grid_baseline_step": {"points_per_s": 5.7e8, "ms_per_step": 1.827, "kernels_ms": {}},
        "encode_sweep": sweep,
        "equal_accuracy": {inputs.IMAGE_2D.name: acc},
        "volume_step": {"simplex": {"points_per_s": 8.5e8}, "simplex_speedup": 1.94, "equal_accuracy": acc},
        "nd_accuracy": {inputs.nd_workload(n).name: dict(acc, simplex={"psnr_db": 30.0, "ms_per_step": 1.0},
                                                         simplex_equal_memory={"psnr_db": 29.0, "ms_per_step": 1.0},
                                                         grid={"psnr_db": 30.5, "ms_per_step": 4.0},
                                                         simplex_speedup=4.0)
                        for n in range(3, 7)},
        "layout_accuracy": {w.name: {"hashed": {"psnr_db": 22.9, "ms_per_step": 1.6},
                                     "sized": {"psnr_db": 22.8, "ms_per_step": 1.4},
                                     "grid": {"psnr_db": 23.0, "ms_per_step": 1.8},
                                     "sized_memory_fraction": 0.43, "sized_minus_hashed_db": -0.1,
                                     "sized_minus_grid_db": -0.2, "sized_speedup_vs_grid": 1.29}
                            for w in (inputs.IMAGE_2D, inputs.VOLUME_3D)},
        "fused_network_backward": {"ms_per_step": 1.716, "vs_separate": 0.955},
        "serving": {"saturation_points_per_s": 4.2e8,
                    "loads": [{"load": 0.5, "p50_ms": 1.4, "p99_ms": 5.2, "points_per_s": 2e8},
                              {"load": 0.8, "p50_ms": 2.1, "p99_ms": 5.2, "points_per_s": 3.3e8}]},
    }


def test_headline_is_compact_json():
    d = _fake_detail()
    line = bench.headline(d, (1 << 20) / 1.652e-3, 20, 5, "results/bench_detail.json")
    text = json.dumps(line, separators=(",", ":"))
    assert len(text) < 4096, len(text)
    back = json.loads(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in back
    assert back["config"]["workload"].startswith("image-2d training step") and "bf16" in back["dtype"]
    d["config"]["workload"] = "volume-3d n=3 L=16 T=2^19 F=2 f16"
    assert bench.headline(d, 8e8, 20, 5, "x")["config"]["workload"].startswith("volume-3d training step")
    r = back["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and 0 < r["frac"] <= 1
    assert back["cpu_baseline"]["cores"] == 16 and back["cpu_baseline"]["cpu_model"]
    assert back["fused_network_backward"]["vs_separate"] == 0.955
    assert all(ln.startswith("# ") for ln in bench.summary_lines(d))
