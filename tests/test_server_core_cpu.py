"""The serving scheduler's admission and batching policy, on the CPU with a
fake executor and a fake clock (csrc/server_core.h compiled with g++)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_scheduler_policy(tmp_path):
    exe = tmp_path / "server_core_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                    os.path.join(HERE, "server_core_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout
