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
    path = tmp_path / "traffic.json"
    rec = {"sources_sha256": bench._sources_digest(), "workload": inputs.IMAGE_2D.name,
           "kernels": {"bin_accum_adam": {"bytes": 123.0}}}
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic("bin_accum_adam", inputs.IMAGE_2D.name) == 123.0
    assert bench.measured_traffic("bin_accum_adam", inputs.VOLUME_3D.name) is None
    assert bench.measured_traffic("bin_scatter", inputs.IMAGE_2D.name) is None
    # sources changed since the counters were taken
    rec["sources_sha256"] = "0" * 64
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("bin_accum_adam", inputs.IMAGE_2D.name) is None
    # no file
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("bin_accum_adam", inputs.IMAGE_2D.name) is None


def test_write_traffic_scales_by_the_copy(tmp_path, monkeypatch):
    hdr = "Kernel_Name,Counter_Value\n"
    # the accum kernel of two steps, then the calibration copy
    fetch = hdr + '"void spx::bin_accum_kernel<2, 2, true>(x)",100\n"void spx::bin_accum_kernel<2, 2, true>(x)",200\n' \
        + f'"spx::cast_kernel(y)",{bench.COPY_ELEMS * 4 / 1024.0 * 0.5}\n'
    write = hdr + '"void spx::bin_accum_kernel<2, 2, true>(x)",50\n"void spx::bin_accum_kernel<2, 2, true>(x)",60\n' \
        + f'"spx::cast_kernel(y)",{bench.COPY_ELEMS * 2 / 1024.0}\n'
    (tmp_path / "f.csv").write_text(fetch)
    (tmp_path / "w.csv").write_text(write)
    out = tmp_path / "t.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    bench.write_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), inputs.IMAGE_2D.name)
    t = json.loads(out.read_text())
    k = t["kernels"]["bin_accum_adam"]
    assert abs(t["factor"]["FETCH_SIZE"] - 0.5) < 1e-12 and abs(t["factor"]["WRITE_SIZE"] - 1.0) < 1e-12
    # the last dispatch, in bytes, each counter divided by its factor
    assert k["FETCH_SIZE_bytes"] == 200 * 1024 / 0.5 and k["WRITE_SIZE_bytes"] == 60 * 1024
    assert k["bytes"] == k["FETCH_SIZE_bytes"] + k["WRITE_SIZE_bytes"]
    assert t["workload"] == inputs.IMAGE_2D.name


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
