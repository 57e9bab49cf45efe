"""Host-side checks of bench.py: the algorithmic operation models behind the
roofline figures, the published peaks they are divided by, the traffic
lookup's source-hash guard, and the one-GPU contract of --gpus."""
import json
import math
import os
import subprocess
import sys

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, REPO)

import bench  # noqa: E402


def test_lattice_model_per_chain():
    # sum over steps i = 1..63 of 4 floor(i/2) + 18
    assert bench.lattice_alg_ops_per_chain(64) == 4 * 992 + 18 * 63 == 5102
    assert bench.lattice_alg_ops_per_chain(1) == 0
    assert bench.lattice_alg_ops_per_chain(2) == 18


def test_lattice26_model_per_chain():
    # sum over steps i = 1..63 of 6 (i - 1) + 28
    assert bench.lattice26_alg_ops_per_chain(64) == 6 * 1953 + 28 * 63 == 13482
    assert bench.lattice26_alg_ops_per_chain(2) == 28


def test_real_model_per_chain():
    k, N = 8, 64
    per_dir = 60 * 4 / math.pi + 20
    expect = sum(k * 9 * (i - 1) + k * per_dir + 10 for i in range(1, N))
    assert bench.real_alg_ops_per_chain(N, k) == pytest.approx(expect, rel=1e-15)
    assert round(bench.real_alg_ops_per_chain(N, k)) == 189829


def test_peaks_follow_unit_counts():
    # 256 CUs at 2.4 GHz; 128 lanes per CU per clock for 32-bit (fp32 vector
    # 157.3 TFLOP/s counting an FMA as 2), 64 for binary64 (78.6 TFLOP/s)
    assert bench.VALU_PEAK_INT32_TOPS == pytest.approx(157.3 / 2, rel=2e-3)
    assert bench.VALU_PEAK_FP64_TOPS == pytest.approx(78.6 / 2, rel=2e-3)
    assert bench.ATTAINABLE_INT_PATH_TOPS == bench.VALU_PEAK_FP64_TOPS


def test_traffic_needs_matching_source_hash(tmp_path, monkeypatch):
    rec = {"lattice_n64": {"kernel": "grow_lattice_reg",
                           "source_sha256": bench.kernel_source_hash("grow_lattice.hip"),
                           "bytes_per_launch": 123}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("grow_lattice_reg", "grow_lattice.hip", "lattice_n64") == 123
    rec["lattice_n64"]["source_sha256"] = "0" * 64
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic("grow_lattice_reg", "grow_lattice.hip", "lattice_n64") is None
    assert bench.measured_traffic("grow_lattice_reg", "grow_lattice.hip", "real_n64") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(REPO, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_lds_models():
    import bench
    # hard spheres: steps 1, 2, 3 move 24, 48 and 72 bytes (write; one near
    # bead; two near beads), step 4 also culls bead 0
    assert bench.real_lds_bytes_per_chain(2) == 24
    assert bench.real_lds_bytes_per_chain(4) == 24 + 48 + 72
    assert bench.real_lds_bytes_per_chain(5) == 24 + 48 + 72 + 96
    # 26-neighbour lattice: (i - 1) words read and one written per step
    assert bench.lattice26_lds_bytes_per_chain(4) == 4 + 8 + 12
    N = 64
    assert bench.lattice26_lds_bytes_per_chain(N) == 4 * (N - 1) * N // 2
    assert abs(bench.LDS_PEAK_TBS - 78.6432) < 1e-9
    o = bench.lds_object(1e12, 1000.0, "x")
    assert abs(o["achieved"] - 1.0) < 1e-12 and abs(o["frac"] - 1.0 / bench.LDS_PEAK_TBS) < 1e-12


def test_cpu_baseline_reports_one_thread_and_all_cores():
    """The CPU baseline times the oracle on one thread and on every core the
    job may use, and states the host's CPU model and counts."""
    from paper_1704_04381_amd.workloads import WORKLOADS

    cb = bench.cpu_baseline(WORKLOADS["real_n64"], 200, 800)
    assert cb["kind"] == "oracle" and cb["unit"] == "monomer-steps/s"
    assert cb["value"] > 0 and cb["single_thread"]["value"] > 0 and cb["single_thread"]["cores"] == 1
    cpu = cb["host_cpu"]
    assert cpu["nproc"] == os.cpu_count() and cpu["affinity"] >= 1
    assert cb["cores"] == min(cpu["affinity"], cpu["job_share"] or cpu["affinity"])
    assert isinstance(cpu["model"], str)
