"""Host logic of bench.py that runs without a GPU: the gating of the committed
HBM counter summaries by workload, launch length and source digest, the
cluster step's work counts, and the single-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads  # noqa: E402


def _summary(name):
    with open(os.path.join(ROOT, "profiles", name)) as f:
        return json.load(f)


def test_sweep_traffic_follows_the_recorded_digest(monkeypatch):
    d = _summary("traffic_k_sweep_stream_uneven512.json")
    name = workloads.uneven_512().name
    spl = next(iter(d["by_sweeps_per_launch"]))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda *a, **k: d["kernel_source_sha256"])
    got, algo = bench.measured_traffic("k_sweep_stream", name, int(spl))
    assert got == d["by_sweeps_per_launch"][spl]["traffic_bytes_per_launch"]
    assert algo == d["by_sweeps_per_launch"][spl]["algorithmic_bytes_per_launch"]
    # another workload, another launch length, an unknown kernel: no figure
    assert bench.measured_traffic("k_sweep_stream", "some-other-workload", int(spl)) == (None, None)
    assert bench.measured_traffic("k_sweep_stream", name, 12345) == (None, None)
    assert bench.measured_traffic("k_no_such_kernel", name, int(spl)) == (None, None)
    # sources changed since the counters were taken: no figure
    monkeypatch.setattr(bench, "kernel_source_digest", lambda *a, **k: "0" * 64)
    assert bench.measured_traffic("k_sweep_stream", name, int(spl)) == (None, None)


def test_cluster_traffic_follows_the_recorded_digest(monkeypatch):
    d = _summary("traffic_cluster_sw_batch256x1024.json")
    assert d["kernel_sources"] == list(bench.CLUSTER_SOURCES)
    name = workloads.batch_256x1024().name
    monkeypatch.setattr(bench, "kernel_source_digest", lambda *a, **k: d["kernel_source_sha256"])
    assert bench.measured_cluster_traffic(name) == d["traffic_bytes_per_step"]
    assert bench.measured_cluster_traffic("some-other-workload") is None
    monkeypatch.setattr(bench, "kernel_source_digest", lambda *a, **k: "0" * 64)
    assert bench.measured_cluster_traffic(name) is None


def test_cluster_summary_adds_up():
    """The per-step bytes are the calibrated sum of the four kernels' counters."""
    d = _summary("traffic_cluster_sw_batch256x1024.json")
    cal = d["copy_calibration"]
    total = sum((p["fetch_size_kib_per_dispatch"] * cal["fetch_scale"] +
                 p["write_size_kib_per_dispatch"] * cal["write_scale"]) * 1024 for p in d["parts"])
    assert total == pytest.approx(d["traffic_bytes_per_step"], rel=1e-12)
    assert [p["kernel"] for p in d["parts"]] == ["k_cl_local", "k_cl_cross<false>", "k_cl_cross<true>",
                                                   "k_cl_flip<0>"]


def test_cluster_work_counts():
    # half a Philox call per site for its two bonds (four words per call serve
    # two sites), at most 1/128 call for flip bits; a 32-bit label written and
    # read back and the spin bits read twice (1.5x for neighbour rows) and
    # written once
    assert bench.SW_OPS_PER_SITE == pytest.approx((0.5 + 1 / 128) * 40)
    assert bench.SW_BYTES_PER_SITE == pytest.approx(8 + 3.5 / 8)
    peak_alu = bench.lane_ops_peak() / bench.SW_OPS_PER_SITE
    peak_hbm = bench.HBM_BYTES_PER_S / bench.SW_BYTES_PER_SITE
    assert peak_hbm < peak_alu  # the step's counted bound is its traffic


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env=dict(os.environ, WORLD_SIZE="1"))
    assert r.returncode == 2
    assert "one GPU" in r.stderr
