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


def test_bench_flop_count_matches_the_step():
    """The bench's algorithmic flop count is the sum of the step's products:
    2N^3 + N^3 (basis change) + 2N^2 M + (q n_it - 1) 2N^3 (folded spectrum) +
    N^3 (overlap) + N^3/3 (Cholesky) + N^3 (triangular solve) + 2N^3 (Rayleigh
    quotients) + 2N^3 (back-rotation) = 19.33 N^3 + 2 N^2 M for q = 2, n_it = 3
    and 13.33 N^3 + 2 N^2 M for q = 1."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    for n, M in ((8192, 512), (2048, 512), (256, 128)):
        n3 = float(n) ** 3
        assert abs(bench.algorithmic_flops(n, M, 2, 3) - (58.0 / 3.0 * n3 + 2.0 * n * n * M)) <= 1e-9 * n3
        assert abs(bench.algorithmic_flops(n, M, 1, 3) - (40.0 / 3.0 * n3 + 2.0 * n * n * M)) <= 1e-9 * n3
    assert abs(bench.algorithmic_flops(8192, 512, 2, 3) - 1.07e13) <= 0.01e13
