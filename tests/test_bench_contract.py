"""The benchmark's host-side contract, on the CPU: it refuses more than one
GPU with a message, prices the rank kernel's algorithmic bytes as 4m + 28n,
and takes the measured traffic from the committed counter summary only when
that summary was taken on the current kernel source."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    for n in (2, 8):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2
        assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes():
    b = load_bench()
    # in_offsets 4(n+1) ~ 4n, in_sources 4m, ranks read 8n, out-degrees 4n,
    # new ranks 8n, vertex permutation 4n
    assert b.algorithmic_bytes(0, 0) == 0
    assert b.algorithmic_bytes(10, 100) == 4 * 100 + 28 * 10
    n, m = 1 << 24, 280_209_285
    assert b.algorithmic_bytes(n, m) == 4 * m + 28 * n


def test_ppr_algorithmic_bytes_and_cpu_info():
    b = load_bench()
    # in_sources 4m, k contributions gathered once 8kn, k new ranks 8kn
    assert b.ppr_algorithmic_bytes(10, 100, 3) == 4 * 100 + 16 * 3 * 10
    n, m = 1 << 20, 17_134_700
    assert abs(b.ppr_algorithmic_bytes(n, m, 64) - 1.142e9) < 1e6
    info = b.cpu_info()
    assert info["nproc"] == os.cpu_count() and info["affinity_cpus"] >= 1


def test_traffic_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    b = load_bench()
    good = tmp_path / "traffic.txt"
    good.write_text("# counters\nkernel_sha256: %s\ntraffic_bytes_per_launch: 7074645403\n"
                    % b.kernel_hash())
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(good))
    assert b.read_traffic() == 7074645403.0

    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_sha256: 0000000000000000\ntraffic_bytes_per_launch: 1\n")
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(stale))
    assert b.read_traffic() is None

    broken = tmp_path / "broken.txt"
    broken.write_text("kernel_sha256: %s\ntraffic_bytes_per_launch: n/a\n" % b.kernel_hash())
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(broken))
    assert b.read_traffic() is None

    monkeypatch.setattr(b, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert b.read_traffic() is None


def test_kernel_hash_covers_the_rank_kernel_sources(tmp_path, monkeypatch):
    b = load_bench()
    h0 = b.kernel_hash()
    copies = []
    for p in b.KERNEL_SOURCES:
        q = tmp_path / os.path.basename(p)
        q.write_bytes(open(p, "rb").read())
        copies.append(str(q))
    monkeypatch.setattr(b, "KERNEL_SOURCES", copies)
    assert b.kernel_hash() == h0
    with open(copies[0], "ab") as f:
        f.write(b"\n")
    assert b.kernel_hash() != h0
