"""Counter probe for the HBM traffic of the dominant kernels (run under
`rocprofv3 --pmc FETCH_SIZE` and, separately, `--pmc WRITE_SIZE`).

    python -m paper_1502_07806_amd.traffic_probe [--n 8192]

Dispatches, in order: a plain device copy of 1 GiB (calibration: 1 GiB read +
1 GiB written), then one folded-spectrum update product of each path at order
n on synthetic operands: the split-BF16 kernel (gemm_x3_kernel, FSUPD
epilogue) and the FP64 kernel (gemm_f64_kernel, FSUPD epilogue).  The counter
values per dispatch divided by the copy's give bytes per launch.  Needs
libpfsm_testhooks.so (the internal kernels' test entry points).
"""
import argparse
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=8192)
    a = ap.parse_args()
    n = a.n
    L = ctypes.CDLL(os.path.join(HERE, "libpfsm_testhooks.so"))
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.pfsm_test_gemm_x3.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, dbl, dbl, vp, i64,
                                    vp, i64, i32, vp, vp, vp]
    L.pfsm_test_gemm_f64.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, dbl, dbl, vp, vp, i64,
                                     vp, i32, vp]
    L.pfsm_test_pack_x3.argtypes = [vp, i32, i64, i64, i64, i32, vp, i64, vp]
    L.pfsm_test_x3_row_stride.argtypes = [i64]
    L.pfsm_test_x3_row_stride.restype = i64
    dev = torch.device("cuda:0")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    # calibration copy: 1 GiB
    x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    # split-BF16 folded-spectrum update, N x N x N
    ldp = L.pfsm_test_x3_row_stride(n)
    g = torch.Generator(device=dev).manual_seed(1)
    M = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
    Ap = torch.empty(n * ldp, dtype=torch.int16, device=dev)
    Bp = torch.empty(n * ldp, dtype=torch.int16, device=dev)
    assert L.pfsm_test_pack_x3(P(M), 1, n, n, n, 0, P(Ap), ldp, s) == 0
    assert L.pfsm_test_pack_x3(P(M), 1, n, n, n, 0, P(Bp), ldp, s) == 0
    Y32 = torch.randn(n, n, dtype=torch.float32, device=dev, generator=g)
    X32 = torch.randn(n, n, dtype=torch.float32, device=dev, generator=g)
    eps = torch.randn(n, dtype=torch.float64, device=dev, generator=g)
    torch.cuda.synchronize()
    assert L.pfsm_test_gemm_x3(2, -1, 0, n, n, n, P(Ap), ldp, P(Bp), ldp, P(X32), n, 0, 0.1, 0.0, P(Y32), n, P(X32),
                               n, 0, P(eps), None, s) == 0
    torch.cuda.synchronize()
    del Ap, Bp, Y32, X32
    # FP64 folded-spectrum update, N x N x N
    B = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
    C = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
    torch.cuda.synchronize()
    assert L.pfsm_test_gemm_f64(0, 0, 2, n, n, n, P(M), n, P(B), n, P(C), n, 0.1, 0.0, P(eps), P(C), n, None, 0,
                                s) == 0
    torch.cuda.synchronize()
    print("traffic probe done (n=%d)" % n, flush=True)


if __name__ == "__main__":
    main()
