"""bench.py's command line on the CPU: a request for more than one GPU is
refused with exit status 2 and a message, before anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_legs_listed_in_help():
    """Every leg that --only selects is named in the help text, the
    paper's two synthetic inputs included."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0
    for leg in ("plain", "batched", "serving", "large", "grid3d", "randlocal"):
        assert leg in r.stdout, leg
