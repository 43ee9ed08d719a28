"""bench.py on the host: one GPU only, refused politely otherwise; the byte and
operation counts it prices its rooflines with; the oracle legs."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_algorithmic_bytes():
    """11.5 K words + 100 B per element and stage: FP32 p = 2 is 376 B, FP64 652 B."""
    b = _bench()
    assert b.stage_bytes_per_element(2, 4) == 376.0
    assert b.stage_bytes_per_element(2, 8) == 652.0
    assert b.stage_bytes_per_element(3, 4) == 11.5 * 10 * 4 + 100


def test_compute_roofline_peaks():
    """The FP64 path is priced at the FP64 vector peak; the FP32 path's peak
    lies between the FP64 and packed-FP32 peaks, and its unpacked figure
    between FP64 and the packed one's half."""
    b = _bench()
    r64 = b.compute_roofline(2, False, 1000, 1e-6)
    assert r64["peak"] == b.FP64_PEAK_TFLOPS
    r32 = b.compute_roofline(2, True, 1000, 1e-6)
    assert b.FP64_PEAK_TFLOPS < r32["peak"] < b.FP32_PEAK_TFLOPS
    assert abs(r32["achieved"] - r32["flop_per_launch"] / 1e-6 / 1e12) < 1e-9
    assert r32["frac_of_unpacked_peak"] > r32["frac"]


def test_cpu_baseline_legs():
    """The oracle on the host: one process, then one per usable core at once."""
    b = _bench()
    r = b.cpu_baseline(1, budget_s=0.3)
    assert r["kind"] == "oracle" and r["cores"] >= 1 and r["value"] > 0
    assert r["single_thread"]["value"] > 0 and r["host"]["nproc"] >= 1
