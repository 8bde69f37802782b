"""Host-side checks of bench.py's contract (no GPU needed)."""

from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    """--gpus N > 1 exits with status 2 and says why, before touching a GPU."""
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_traffic_summaries_parse(tmp_path, monkeypatch):
    """A counter summary is used only for the kernel source and workload it was
    taken on: matching hash and size give its bytes, anything else None."""
    algorithmic = 152 * 4096 * 4096
    got = bench.measured_traffic("fused_dns_fp32", 4096 * 4096)
    assert got is None or algorithmic < got < 1.5 * algorithmic
    assert bench.measured_traffic("fused_dns_fp32", 1024 * 1024) is None
    assert bench.measured_traffic("no_such_kernel", 4096 * 4096) is None
    prof = tmp_path / "profiles"
    prof.mkdir()
    text = ("kernel_source_sha256: {h}\nlups_per_launch: 100\nhbm_bytes_per_launch: 16000\n")
    (prof / "traffic_k.txt").write_text(text.format(h=bench.kernel_source_hash()))
    (prof / "traffic_old.txt").write_text(text.format(h="0" * 16))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k", 100) == 16000.0
    assert bench.measured_traffic("k", 101) is None
    assert bench.measured_traffic("old", 100) is None


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    """Editing comments or blank space keeps a counter summary valid; any
    change of code invalidates it."""
    def h(text):
        f = tmp_path / "k.hip"
        f.write_text(text)
        monkeypatch.setattr(bench, "KERNEL_SRC", str(f))
        return bench.kernel_source_hash()

    base = h("int f(int a) {\n  return a + 1;  // one\n}\n")
    assert h("/* about f */\nint f(int a) {\n\n    return a + 1;  // two\n}") == base
    assert h("int f(int a) {\n  return a + 2;  // one\n}\n") != base
    # spacing inside a line counts (conservative: a reformatting invalidates too)
    assert h("int f(int a) {\n  return a+1;\n}\n") != base


def test_correction_interval_must_be_positive():
    """--corr-every below 1 is an argument error (exit 2) before touching a GPU."""
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--corr-every", "0"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "--corr-every" in res.stderr
    assert res.stdout == ""


def test_cpu_legs_report_host_and_do_not_import_the_product():
    """The oracle legs: one thread and every usable core (bounded to two here),
    with the CPU model and core counts, and without importing the library's
    package (the oracle leg is test infrastructure only)."""
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "c = bench.cpu_baseline(1, 0, 1, max_procs=2); "
            "v = bench.variant_oracle_rates(n=32, steps=1); "
            "print(json.dumps({'c': c, 'v': sorted(v), 'product': 'paper_1705_09807_amd' in sys.modules}))" % ROOT)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert res.returncode == 0, res.stderr
    import json
    out = json.loads(res.stdout.strip().splitlines()[-1])
    c = out["c"]
    assert c["kind"] == "oracle" and c["cores"] == 1 and c["value"] > 0
    assert c["nproc"] >= 1 and c["affinity_cores"] >= 1 and "cpu_model" in c
    if c["affinity_cores"] > 1:
        assert c["cores_all"] == 2 and c["mlups_all"] > 0
    assert "les1024_learned" in out["v"]
    assert out["product"] is False
