"""Host-side contract of the entry points: the bench refuses more than one GPU,
and the binding refuses to load without the built library (no fallback)."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""   # no JSON line


def test_binding_without_library_fails_loudly(tmp_path):
    src = os.path.join(ROOT, "paper_2507_21236_amd")
    dst = tmp_path / "paper_2507_21236_amd"
    dst.mkdir()
    for f in os.listdir(src):
        if f.endswith(".py"):
            shutil.copy(os.path.join(src, f), dst / f)
    assert not (dst / "libattn.so").exists()
    code = "import paper_2507_21236_amd"
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       cwd=str(tmp_path), env={**os.environ, "PYTHONPATH": str(tmp_path)})
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libattn.so is missing" in r.stderr
