"""Host-side contracts of bench.py (no GPU): the single-GPU guard, the gating
of measured HBM traffic on the kernel sources, and the accuracy form's
metrics against the oracle's definitions."""
import os
import subprocess
import sys

import numpy as np

import bench
from oracle import mfcim as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


def test_traffic_is_reported_only_for_the_measured_sources(tmp_path):
    h = bench.kernel_source_hash(bench.KERNEL_SOURCES)
    good = tmp_path / "good.txt"
    good.write_text(f"# comment: 1\nsource_sha256: {h}\nhbm_bytes_per_launch: 1234\n")
    assert bench.measured_traffic(str(good)) == 1234.0
    stale = tmp_path / "stale.txt"
    stale.write_text("source_sha256: " + "0" * 64 + "\nhbm_bytes_per_launch: 1234\n")
    assert bench.measured_traffic(str(stale)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt")) is None
    # a different key than the file records is no figure either
    assert bench.measured_traffic(str(good), bench.KERNEL_SOURCES, "hbm_bytes_per_step") is None


def test_accuracy_metrics_match_the_oracle():
    rng = np.random.default_rng(3)
    for _ in range(5):
        n = 500
        xi = (rng.random(n) < 0.2).astype(np.uint8)
        x = rng.standard_normal(n)
        sig = (rng.random(n) < 0.25).astype(np.uint8)
        R = rng.standard_normal(n)
        assert np.isclose(bench.acc_rmse(sig, R, x, xi), O.rmse(sig, R, x, xi), rtol=1e-14, atol=0)
        assert bench.acc_hamming(sig, xi) == O.hamming_loss(sig, xi)


def test_factored_flop_count():
    S = 128
    per_fft = 5 * S * 7 + 6 * S
    expect = 2 * (2 * S * per_fft) + 2 * 3 * (S * S // 4 + S * S // 16 + S * S // 64) * 4 + S * S + 20 * S * S
    assert bench.mri_flops_per_replica_step(S, 3) == expect
