"""Host-side logic of bench.py (CPU only): the stored counter readings are used only for
the kernel source they were taken on."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_follows_kernel_source(tmp_path, monkeypatch):
    b = _bench()
    csrc = tmp_path / "paper_2510_10529_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "apply.hip").write_text("kernel v1\n")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    h = b.kernel_source_hash()
    (tmp_path / "profiles" / "ks_apply_traffic.txt").write_text(
        "# comment\n"
        f"workload=w1 prec=f64 src={h} fetch_kib=100 write_kib=50 fetch_scale=2.0 write_scale=1.0 launches=3\n"
        f"workload=w1 prec=f64 src={h} deflate=10 fetch_kib=70 write_kib=40 fetch_scale=2.0 write_scale=1.0\n")
    assert b.read_traffic("f64", "w1") == 1024.0 * (100 * 2.0 + 50 * 1.0)
    assert b.read_traffic("f64", "w1", 10) == 1024.0 * (70 * 2.0 + 40 * 1.0)   # another launch mix
    assert b.read_traffic("f64", "w1", 6) is None
    assert b.read_traffic("f32", "w1") is None
    assert b.read_traffic("f64", "other") is None
    (csrc / "apply.hip").write_text("kernel v2\n")          # the kernel changed since the counters
    assert b.read_traffic("f64", "w1") is None


def test_multi_gpu_request_exits_with_message():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
