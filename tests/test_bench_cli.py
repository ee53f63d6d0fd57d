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
    """The method's bytes of the fused update + closure + forward x transform
    at 128^3 with 5 sites: read m tau_i, m R_i and w, write tau and the packed
    spectra, 4 n_v N (2 m + 2) + 8 P N; at the headline solve's mean of 4.94
    stored pairs 548 MB.  The increment scheme's closure-increment write
    (4 n_v N; it reads the anchor's closure argument in place of w) is
    reported apart."""
    sys.path.insert(0, ROOT)
    import bench
    N = 128 ** 3
    assert bench.kernel_bytes(5, N, 5, 5.0, "update_fftx_f32") == 4 * 5 * N * 12 + 8 * 3 * N
    assert abs(bench.kernel_bytes(5, N, 5, 4.94, "update_fftx_f32") / 1e6 - 548.2) < 0.5
    assert bench.increment_overhead_bytes(5, N, "update_fftx_f32") == 4 * 5 * N
    assert bench.increment_overhead_bytes(5, N, "fftx_residual_f32") == 0.0
    assert bench.kernel_bytes(5, N, 5, 5.0, "zfft_contract_f32") == 16 * 3 * N
