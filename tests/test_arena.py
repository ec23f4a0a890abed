"""The served form's device-memory arena: its first-fit bookkeeping is host
code, compiled here with g++ and checked on randomised allocation sequences."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def test_arena_first_fit_bookkeeping():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "arena_check")
        subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "arena_check.cpp")],
                       check=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
        assert "arena ok" in r.stdout
