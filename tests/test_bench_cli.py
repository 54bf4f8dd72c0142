"""Host checks of the benchmark script (no GPU): the one-GPU contract, the
HBM-traffic lookup that the roofline uses, and the compressed-memory
accounting of the TLR record."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_lookup_follows_the_kernel_source():
    """The committed counter summary counts only while the kernel's source
    has the hash the counters were taken on; unknown workloads give None."""
    got = bench.measured_traffic("k_gemm_nt_sub_lds", "tlr_n100000_nb1200")
    assert got is not None and 1e9 < got < 2e10
    assert bench.measured_traffic("k_gemm_nt_sub_lds", "no_such_workload") is None
    assert bench.measured_traffic("no_such_kernel", "tlr_n100000_nb1200") is None


def test_traffic_lookup_rejects_a_changed_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "k.hip"
    src.write_text("// kernel\n")
    rec = {"kernel": "k", "source": "k.hip", "source_sha256": "0" * 64,
           "fetch_bytes_per_launch": 1.0, "write_bytes_per_launch": 2.0, "workload": "w"}
    (prof / "k_w_hbm_traffic.md").write_text("traffic_json: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k", "w") is None
    import hashlib
    rec["source_sha256"] = hashlib.sha256(src.read_bytes()).hexdigest()
    (prof / "k_w_hbm_traffic.md").write_text("traffic_json: " + json.dumps(rec) + "\n")
    assert bench.measured_traffic("k", "w") == 3.0


def test_tlr_memory_accounting():
    """Dense diagonal tiles, 2 nb k per low-rank tile and nb^2 per dense
    fall-back tile (rank < 0), against the dense lower tiles and the full
    matrix."""
    nb, T = 4, 3
    ranks = np.zeros((T, T), dtype=np.int64)
    ranks[1, 0], ranks[2, 0], ranks[2, 1] = 1, -1, 2
    m = bench.tlr_memory(ranks, nb, T * nb)
    comp = T * nb * nb + 2 * nb * 1 + nb * nb + 2 * nb * 2
    assert abs(m["compressed_gb"] - 8.0 * comp / 1e9) < 1e-18
    assert abs(m["ratio_lower_tiles_over_tlr"] - 6 * nb * nb / comp) < 1e-12
    assert abs(m["ratio_full_over_tlr"] - (T * nb) ** 2 / comp) < 1e-12
