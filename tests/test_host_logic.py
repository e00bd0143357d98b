"""Host-side logic shared with the kernels, compiled with g++ (no GPU)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_rank_order_is_a_permutation(tmp_path):
    exe = str(tmp_path / "order_key_check")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined",
                           os.path.join(ROOT, "tests", "cpp", "order_key_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0 and "OK" in r.stdout, r.stdout + r.stderr
