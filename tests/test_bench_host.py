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
    assert bench._measured_valu_insts() is None
    # with the digest the counters were taken with, the summary's figures are read: the
    # traffic above the algorithmic bytes and the VALU instructions of one launch (its table
    # row, thousands separators removed) equal to the committed row
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: committed[0])
    assert bench._measured_traffic() > 0
    row = [ln for ln in text.splitlines() if ln.startswith("| SQ_INSTS_VALU |")]
    assert len(row) == 1
    assert bench._measured_valu_insts() == float(row[0].split("|")[2].replace(",", ""))


def test_number_fluctuation_s0_of_an_ideal_gas():
    """Independent uniform points (an ideal gas) have S(0) = 1: the cube estimator and its
    1/l extrapolation find it within a few percent, in a slab of the box and in one that
    wraps around the periodic x boundary."""
    import numpy as np
    bench = _bench_module()
    rng = np.random.default_rng(3)
    L = 86.0
    frames = [rng.uniform(0.0, L, size=(3, 64000)) for _ in range(20)]
    s0, per = bench.number_fluctuation_s0(frames, (L, L, L), 30.0, 25.0)
    assert len(per) >= 3 and abs(s0 - 1.0) < 0.05, (s0, per)
    s0w, _ = bench.number_fluctuation_s0(frames, (L, L, L), 70.0, 40.0)
    assert abs(s0w - 1.0) < 0.05


def test_number_fluctuation_s0_of_a_lattice_is_small():
    """A perfect lattice (one point per unit cell, cubes of whole cells) has no number
    fluctuation at all."""
    import numpy as np
    bench = _bench_module()
    g = np.arange(40, dtype=np.float64) + 0.5
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    com = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    s0, per = bench.number_fluctuation_s0([com], (40.0, 40.0, 40.0), 0.0, 40.0, sides=(4, 5, 8))
    assert max(per.values()) == 0.0 and abs(s0) < 1e-12


def test_smooth_counts():
    """Width 0 leaves the counts alone; a constant profile and the interior of a linear ramp
    (a symmetric kernel away from the ends) come back unchanged."""
    import numpy as np
    bench = _bench_module()
    c = np.array([5, 9, 2, 7], dtype=np.int64)
    assert (bench.smooth_counts(c, 0.0, 0.5) == c).all()
    flat = np.full(14, 100000, dtype=np.int64)
    assert (bench.smooth_counts(flat, 1.5, 0.5) == flat).all()
    ramp = 100000 + 1000 * np.arange(40, dtype=np.int64)
    out = bench.smooth_counts(ramp, 1.0, 0.5)
    assert np.abs(out[10:30] - ramp[10:30]).max() <= 1
