"""CPU checks of bench.py's host-side helpers (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("p,g", [(2, 1), (3, 2), (17, 5), (64, 6), (256, 8), (1000, 14), (1023, 18),
                                  (2 ** 20 - 1, 38)])
def test_gemm_count_is_the_binary_schedule(p, g):
    # floor(log2 p) squarings and popcount(p) - 1 multiplies (section 4.3)
    assert bench.gemm_count(p) == g == (p.bit_length() - 1) + bin(p).count("1") - 1


def test_clock_sampler_reports_why_it_has_no_samples():
    # without a GPU driver (or amdsmi) the sampler reports the reason, not a number
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with bench.ClockSampler(0.01, delay=0.0) as c:
        pass
    s = c.summary()
    assert s["samples"] == 0 and s["source"] == "amdsmi" and s.get("error")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
