"""ctypes access to libpfsm_testhooks.so (internal kernels, tests only)."""
import ctypes
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOOKS = os.path.join(ROOT, "paper_1502_07806_amd", "libpfsm_testhooks.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(HOOKS):
            raise RuntimeError("libpfsm_testhooks.so missing: run python -m paper_1502_07806_amd.build_lib")
        L = ctypes.CDLL(HOOKS)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.pfsm_test_gemm_f64.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, dbl, dbl, vp, vp,
                                         i64, vp, i32, vp]
        L.pfsm_test_gemm_f64.restype = i32
        L.pfsm_test_pack_x3.argtypes = [vp, i32, i64, i64, i64, i32, vp, i64, vp]
        L.pfsm_test_pack_x3.restype = i32
        L.pfsm_test_pack_x3_part.argtypes = [vp, i32, i64, i64, i64, i32, vp, i64, vp, i32, i32, vp, vp, vp]
        L.pfsm_test_pack_x3_part.restype = i32
        L.pfsm_test_gemm_x3.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, dbl, dbl, vp,
                                        i64, vp, i64, i32, vp, vp, vp]
        L.pfsm_test_gemm_x3.restype = i32
        L.pfsm_test_gemm_x3_ws.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, dbl, dbl, vp,
                                           i64, vp, i64, i32, vp, vp, vp, ctypes.c_size_t, vp]
        L.pfsm_test_gemm_x3_ws.restype = i32
        L.pfsm_test_gemm_x3_fs.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp,
                                           i64, vp, dbl, vp]
        L.pfsm_test_gemm_x3_fs.restype = i32
        L.pfsm_test_x3_plain_stride.argtypes = [i64]
        L.pfsm_test_x3_plain_stride.restype = i64
        L.pfsm_test_x3_split_bytes.argtypes = [i64]
        L.pfsm_test_x3_split_bytes.restype = i64
        L.pfsm_test_x3_row_stride.argtypes = [i64]
        L.pfsm_test_x3_row_stride.restype = i64
        L.pfsm_test_cholesky.argtypes = [vp, i64, i64, vp, vp, vp]
        L.pfsm_test_cholesky.restype = i32
        L.pfsm_test_trsm.argtypes = [vp, i64, vp, i64, i64, i64, vp, vp]
        L.pfsm_test_trsm.restype = i32
        L.pfsm_test_cholesky_qr_gated.argtypes = [vp, i64, vp, i64, i64, i64, vp, vp, vp, vp, vp]
        L.pfsm_test_cholesky_qr_gated.restype = i32
        L.pfsm_test_convert_gated.argtypes = [vp, i64, vp, i64, i64, i64, i32, vp, vp]
        L.pfsm_test_convert_gated.restype = i32
        L.pfsm_test_oz_split.argtypes = [vp, i64, i64, i64, i32, vp, vp, vp, vp]
        L.pfsm_test_oz_split.restype = i32
        L.pfsm_test_gemm_oz.argtypes = [i64, i64, i64, i32, vp, vp, vp, vp, vp, i64, i32, vp]
        L.pfsm_test_gemm_oz.restype = i32
        L.pfsm_test_oz_row_stride.argtypes = [i64]
        L.pfsm_test_oz_row_stride.restype = i64
        L.pfsm_test_oz_plane_bytes.argtypes = [i64, i32]
        L.pfsm_test_oz_plane_bytes.restype = i64
        L.pfsm_test_refine_slices.argtypes = []
        L.pfsm_test_refine_slices.restype = i32
        L.pfsm_test_refine_tau.argtypes = []
        L.pfsm_test_refine_tau.restype = dbl
        L.pfsm_test_refine_kmax.argtypes = []
        L.pfsm_test_refine_kmax.restype = i32
        L.pfsm_test_refine.argtypes = [i64, vp, i64, vp, i64, vp, vp, vp, vp, vp, vp, i64, vp, vp]
        L.pfsm_test_refine.restype = i32
        _lib = L
    return _lib


def bf16_round(x):
    """Round-to-nearest-even to bfloat16 (as float32 values)."""
    x = np.asarray(x, np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def split_hi_lo(x):
    x = np.asarray(x, np.float64)
    hi = bf16_round(x.astype(np.float32)).astype(np.float64)
    lo = bf16_round((x - hi).astype(np.float32)).astype(np.float64)
    return hi, lo


def oz_digits(X, s):
    """Digits of the columns of X as the int8 digit GEMM defines them: each column
    scaled by 2^-e (e the frexp exponent of its largest magnitude), then s
    round-to-nearest-even digits of the remainder, the first at weight 2^-6 and
    each next one 2^-7 smaller.  Returns (list of s float arrays, e)."""
    X = np.asarray(X, np.float64)
    mx = np.max(np.abs(X), axis=0)
    e = np.where(mx > 0, np.frexp(mx)[1], 0).astype(np.int64)
    t = np.ldexp(X, (6 - e)[None, :])
    D = []
    for _ in range(s):
        d = np.rint(t)
        D.append(d)
        t = (t - d) * 128.0
    return D, e
