"""bench.py's command line on the host: the options parse, and more than one GPU
is refused with a message (the benchmark is one GPU's throughput)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_help_parses():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    assert "--steps" in r.stdout and "--warmup" in r.stdout


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_traffic_record_is_dropped_when_the_kernel_source_changes(tmp_path, monkeypatch):
    """The bench reports the committed HBM-traffic record of its GEMM only while the
    kernel source hash matches the one the counters were taken with."""
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.kernel_source_sha()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel": "k_cgemm_b3<0>", "source_sha256": sha, "bytes_per_launch": 1.5e10}
    (prof / "t.md").write_text("text\n<!-- traffic " + json.dumps(rec) + " -->\n")
    csrc = tmp_path / "paper_2208_07478_amd" / "csrc"
    csrc.mkdir(parents=True)
    src = open(os.path.join(ROOT, "paper_2208_07478_amd", "csrc", "sigma.hip")).read()
    (csrc / "sigma.hip").write_text(src)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_traffic("k_cgemm_b3<0>")["bytes_per_launch"] == 1.5e10
    assert bench.stored_traffic("k_cgemm<0, float>") is None
    a = src.index("// Real arithmetic of one GEMM variant")
    (csrc / "sigma.hip").write_text(src[:a] + src[a:].replace("Prr[a][b]", "Prr[a][b] ", 1))
    assert bench.stored_traffic("k_cgemm_b3<0>") is None
