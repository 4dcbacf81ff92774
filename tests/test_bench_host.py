"""Host checks of bench.py (no GPU): it refuses more than one GPU with a message, and it
reports the committed HBM traffic of the fused step only while the counters' source
digest matches the kernel's current sources."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_traffic_follows_the_kernel_digest(monkeypatch):
    bench = _bench_module()
    with open(bench.PMC_SUMMARY) as f:
        text = f.read()
    committed = [ln.split(":", 1)[1].strip() for ln in text.splitlines()
                 if ln.strip().lstrip("- ").startswith("source_sha256")]
    assert len(committed) == 1
    t = bench._measured_traffic()
    if committed[0] == bench.kernel_source_digest():
        algorithmic = [float(ln.split(":", 1)[1].split()[0]) for ln in text.splitlines()
                       if ln.strip().lstrip("- ").startswith("algorithmic_bytes_per_launch")][0]
        assert t is not None and t > algorithmic   # counters see at least the algorithmic bytes
    else:
        assert t is None
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0" * 64)
    assert bench._measured_traffic() is None
