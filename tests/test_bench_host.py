"""Host checks of bench.py (no GPU): the one-GPU refusal, and the committed
HBM-traffic summary that the bench line reports as roofline.traffic.

* `bench.py --gpus 2` exits with status 2 and says why, before touching the GPU;
* the traffic summary is parsed into the P2P kernel's bytes per launch when
  its source digest matches the P2P kernel's sources, else None; the figure
  is FETCH_SIZE x fetch_scale + WRITE_SIZE x write_scale in bytes, with the
  scales taken from the plain-copy calibration in the same file;
* the shader-clock reader returns a number or None without starting any
  program.
"""
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


def _summary():
    vals = {}
    with open(bench.TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    return vals


def test_traffic_summary_is_consistent():
    v = _summary()
    copy = float(v["copy_bytes"])
    fs = copy / (1024 * float(v["copy_fetch_kib"]))
    ws = copy / (1024 * float(v["copy_write_kib"]))
    assert abs(fs - float(v["fetch_scale"])) < 1e-3 and abs(ws - float(v["write_scale"])) < 1e-3
    for k in ("p2p", "m2l", "l2p_combine", "p2m", "gather"):
        want = 1024 * (float(v[k + "_fetch_kib_per_dispatch"]) * fs +
                       float(v[k + "_write_kib_per_dispatch"]) * ws)
        assert abs(float(v[k + "_traffic_bytes_per_launch"]) - want) <= 0.01 * want, k
    got = bench.measured_traffic("uniform-1e6-p4")
    if v["p2p_source_sha256"] == bench.p2p_source_digest():
        assert got == float(v["p2p_traffic_bytes_per_launch"])
    else:
        assert got is None
    assert bench.measured_traffic("plummer-1e6-p6") is None


def test_shader_clock_reader_runs_without_a_gpu():
    v = bench.gpu_sclk_mhz()
    assert v is None or v > 0
