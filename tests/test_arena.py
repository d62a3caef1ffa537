"""The host-side arena allocator (first fit, 256-byte alignment, coalescing),
checked on the CPU by a randomised model test written in C++."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_arena_model(tmp_path):
    exe = str(tmp_path / "arena_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-o", exe,
                           os.path.join(HERE, "arena_check.cpp")])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "arena ok" in out.stdout
