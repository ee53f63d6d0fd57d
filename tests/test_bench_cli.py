"""bench.py's command line on the host: one GPU per process."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_kernel_bytes_of_the_dominant_family():
    """The algorithmic bytes of the fused update at 128^3 with 5 sites and a
    full history of 5 pairs: 4 n_v N (2 m + 4) + 8 P N."""
    sys.path.insert(0, ROOT)
    import bench
    N = 128 ** 3
    assert bench.kernel_bytes(5, N, 5, 5.0, "update_fftx_f32") == 4 * 5 * N * 14 + 8 * 3 * N
    assert bench.kernel_bytes(5, N, 5, 5.0, "zfft_contract_f32") == 16 * 3 * N
