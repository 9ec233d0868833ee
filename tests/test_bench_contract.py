"""Host checks of the benchmark's contract and of the binding's failure mode:
more than one GPU is refused with a message, and without the built library
the binding raises instead of computing anything on the host."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_binding_fails_loudly_without_the_library(monkeypatch):
    from paper_0711_2665_amd import lbmd
    monkeypatch.setattr(lbmd, "_lib", None)
    monkeypatch.setattr(lbmd, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "liblbmd.so"))
    with pytest.raises(RuntimeError, match="missing"):
        lbmd.lib()
