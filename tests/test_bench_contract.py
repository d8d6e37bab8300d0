"""Host-side parts of bench.py: the one-GPU guard and the algorithmic byte
counts its roofline figures divide by (the operator's 1484 B per P3 triangle
in FP64, the Jacobian apply's 1804 B)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_element():
    import bench
    # operator: read W (7 x 10) and b_old (3 x 10), write R (7 x 10), 4 metric
    # entries, |J|, 3 normals (2 each), 3 half lengths; 3 int32 neighbour codes
    assert bench.bytes_per_element(2, 3, 8) == 8 * (2 * 70 + 30 + 4 + 1 + 6 + 3) + 4 * 3 == 1484
    # Jacobian apply: read W and x, write y, the same geometry and codes
    assert bench.jac_bytes_per_element(2, 3, 8) == 8 * (3 * 70 + 14) + 12 == 1804
    # FP32 halves the floating-point part only
    assert bench.bytes_per_element(2, 3, 4) == 4 * (2 * 70 + 30 + 14) + 12
