"""Host-side logic of the benchmark (no GPU): the one-GPU guard, and the
lookup that ties stored HBM counters to the final-step kernel sources."""
import os
import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_lookup_follows_the_kernel_sources(tmp_path, monkeypatch):
    sha = bench.source_sha()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "root_gemm_qaoa32_fp16x3_traffic.md").write_text(
        f"header\nsource_sha: {sha}\nfetch_bytes: 100\nwrite_bytes: 23\n")
    (prof / "root_gemm_qaoa32_bf16x6_traffic.md").write_text(
        "source_sha: 0000000000000000\nfetch_bytes: 1\nwrite_bytes: 2\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_sha", lambda: sha)
    assert bench.measured_traffic("fp16x3") == 123.0   # taken on these sources
    assert bench.measured_traffic("bf16x6") is None    # taken on other sources
    assert bench.measured_traffic("fp32") is None      # never taken


def test_committed_traffic_summaries_carry_their_keys():
    for form in ("fp16x3", "bf16x6"):
        path = os.path.join(bench.ROOT, "profiles", f"root_gemm_qaoa32_{form}_traffic.md")
        keys = {line.split(":", 1)[0].strip() for line in open(path) if ":" in line}
        assert {"source_sha", "fetch_bytes", "write_bytes"} <= keys, form
