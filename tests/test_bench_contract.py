"""Host-side checks of bench.py's contract (no GPU): the one-GPU refusal and the
committed rocprofv3 traffic summaries it reads."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_traffic_summaries_parse_and_exceed_the_algorithmic_bytes():
    """Each fused-step summary names its kernel source hash and order and gives
    HBM bytes per launch; the traffic can only be at least the algorithmic bytes
    (operands once plus the epilogue's reads and writes)."""
    algorithmic = {"gemm_bf16": 4831838208, "gemm_fp32": 5368709120}
    for kind, info in bench.KERNELS.items():
        vals = {}
        for line in open(info["traffic"]):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
        assert int(vals["n"]) == 16384
        assert len(vals["kernel_source_sha256_16"]) == 16
        hbm = float(vals["hbm_bytes_per_launch"])
        assert hbm == float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
        assert hbm >= algorithmic[kind]
