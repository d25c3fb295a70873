"""Host-only C++ parts of the library, compiled with g++ and run here: the
device-arena bookkeeping of the serving loop."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_bookkeeping(tmp_path):
    exe = str(tmp_path / "arena_check")
    src = os.path.join(ROOT, "tests", "native", "arena_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-o", exe, src],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "arena ok" in r.stdout
