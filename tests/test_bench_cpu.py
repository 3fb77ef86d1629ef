"""CPU checks of the benchmark's contract and byte model (no GPU)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_byte_model_matches_field_passes():
    import bench
    np_, ncol, nz, N = 2686976, 65536, 41, 4
    kb = dict(bench.kernel_bytes(np_, ncol, nz, N))
    f = 8 * np_
    F = nz * (4 * N + 1) * 8  # one factor set shared by the identical columns
    assert sum(kb.values()) == 65 * f + 2 * F
    assert kb["colsolve_stage3"] - kb["colsolve_stage2"] == 4 * f
    # 1.397 GB per step on the benchmark grid
    assert abs(sum(kb.values()) / 1e9 - 1.397) < 0.001


def test_precision_form_byte_model():
    """R1 in FP32: its 14 field passes (5 written, 9 read) move 4 bytes per
    value, the other 51 passes 8: 464 bytes per node against 520."""
    import bench
    np_, ncol, nz, N = 2686976, 65536, 41, 4
    k64 = dict(bench.kernel_bytes(np_, ncol, nz, N))
    k32 = dict(bench.kernel_bytes(np_, ncol, nz, N, r1=4))
    F = nz * (4 * N + 1) * 8
    assert sum(k32.values()) == 464 * np_ + 2 * F
    assert sum(k64.values()) - sum(k32.values()) == 14 * 4 * np_
    assert k32["rhs_stage3"] == k64["rhs_stage3"]
