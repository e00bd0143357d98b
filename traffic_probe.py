"""Measurement helpers for the profiles: HBM traffic of the dominant kernels,
and the per-kernel table of one solve from a kernel trace.

    python traffic_probe.py [--n 8192]
        dispatches the kernels; run it under `rocprofv3 --pmc FETCH_SIZE` and,
        separately, `rocprofv3 --pmc WRITE_SIZE` (CSV output)
    python traffic_probe.py --summarize FETCH.csv WRITE.csv --out profiles/traffic.json
        turns the two counter files into HBM bytes per launch
    python traffic_probe.py --trace-summary KERNEL_TRACE.csv --out OUT.md
        per-kernel table of one solve of a `rocprofv3 --kernel-trace` run of
        bench.py (the launches between the last two int8 refinement products),
        and the submatrix eigensolver's kernel time per sweep

Dispatches, in order: a plain device copy of 1 GiB (calibration: 1 GiB read +
1 GiB written), then at order n on synthetic operands: the split-BF16
folded-spectrum update (FSUPD epilogue, default tile configuration), the same
update from plain BF16 operands (one product, as the mixed path runs it), the
FP64 folded-spectrum update, and the int8 digit product of the refinement
(two digit splits with the refinement's digit count, then one launch).  Each counter value of a dispatch is
scaled by the copy's bytes over the copy's counter value.  Needs
libpfsm_testhooks.so (the internal kernels' test entry points).
"""
import argparse
import csv
import ctypes
import hashlib
import json
import os
import re

import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(ROOT, "paper_1502_07806_amd")
GEMM_SOURCES = ("gemm_f64.hip", "gemm_x3.hip", "gemm_x3.h", "gemm_oz.hip", "gemm_oz.h", "common.h", "refine.h")
OZ_PRODUCT = "gemm_oz_multi"  # the int8 digit product's default kernel


def gemm_source_hash() -> str:
    """Hash of the GEMM kernel sources: stored traffic figures apply only to the
    kernels they were measured on."""
    h = hashlib.sha256()
    for f in GEMM_SOURCES:
        p = os.path.join(PKG, "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def summarize(fetch_csv: str, write_csv: str, n: int, out: str):
    def per_dispatch(path):
        d = {}
        for r in csv.DictReader(open(path)):
            k = int(r["Dispatch_Id"])
            e = d.setdefault(k, {"name": r["Kernel_Name"], "kib": 0.0})
            e["kib"] += float(r["Counter_Value"])
        return [d[k] for k in sorted(d)]
    fe, wr = per_dispatch(fetch_csv), per_dispatch(write_csv)
    copy_f = [e for e in fe if "copyBuffer" in e["name"]][0]["kib"]
    copy_w = [e for e in wr if "copyBuffer" in e["name"]][0]["kib"]
    gib_kib = float(1 << 20)
    sf, sw = gib_kib / copy_f, gib_kib / copy_w  # true bytes per counted byte (copy of 1 GiB)

    def pick(lst, key):
        return [e for e in lst if key in e["name"]][0]["kib"]
    res = {"_calibration": {"copy_bytes": 1 << 30, "fetch_scale": sf, "write_scale": sw,
                            "note": "FETCH_SIZE and WRITE_SIZE (KiB, summed over agents) per dispatch, each scaled "
                                    "by what the same counter reads for a 1 GiB device copy"}}
    for key, name in (("gemm_x3_fsupd_n%d" % n, "gemm_x3_dl<2, true, 3>"),
                      ("gemm_x3_fsupd_plain_n%d" % n, "gemm_x3_dl<2, true, 1>"),
                      ("gemm_f64_fsupd_n%d" % n, "gemm_f64_kernel"), ("gemm_oz_n%d" % n, OZ_PRODUCT)):
        f, w = pick(fe, name) * 1024 * sf, pick(wr, name) * 1024 * sw
        res[key] = {"kernel": name, "fetch_bytes": f, "write_bytes": w, "bytes_per_launch": f + w,
                    "source_hash": gemm_source_hash()}
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


def _short(name: str) -> str:
    name = name.replace("pfsm::(anonymous namespace)::", "").replace("void ", "").replace("pfsm::", "")
    m = re.match(r"([A-Za-z_0-9]+(<[^()]*>)?)", name)
    return m.group(1) if m else name[:40]


def trace_summary(trace_csv: str, out: str):
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    idx = [i for i, r in enumerate(rows) if OZ_PRODUCT in r["Kernel_Name"]]
    seq = rows[idx[-2] + 1:idx[-1] + 1]
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in seq]
    span = (int(seq[-1]["End_Timestamp"]) - int(seq[0]["Start_Timestamp"])) / 1e6
    agg = {}
    for r, d in zip(seq, dur):
        a = agg.setdefault(_short(r["Kernel_Name"]), [0, 0.0, 1e30, 0.0])
        a[0] += 1
        a[1] += d
        a[2] = min(a[2], d)
        a[3] = max(a[3], d)
    busy = sum(dur)
    lines = ["One solve taken from the kernel trace (the launches between the last two int8 refinement "
             "products): span %.2f ms, kernels busy %.2f ms, %d launches." % (span, busy / 1e3, len(seq)), "",
             "| kernel | launches | total ms | avg us | min us | max us | share |", "|---|---|---|---|---|---|---|"]
    for name, a in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append("| `%s` | %d | %.3f | %.1f | %.1f | %.1f | %.1f%% |"
                     % (name, a[0], a[1] / 1e3, a[1] / a[0], a[2], a[3], 100.0 * a[1] / busy))
    sweeps, cur = [], None
    for r, d in zip(seq, dur):
        name = _short(r["Kernel_Name"])
        if name == "sweep_begin":
            cur = [0.0, 0]
            sweeps.append(cur)
        if cur is not None and name in ("sweep_begin", "pair_solve", "pair_apply_b", "pair_solve_apply_u"):
            cur[0] += d
            cur[1] += 1
        if name == "rank_select":
            cur = None
    lines += ["", "Submatrix eigensolver, kernel time per sweep (us / launches): "
              + ", ".join("%.0f / %d" % (t, c) for t, c in sweeps)]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--summarize", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--trace-summary", metavar="KERNEL_TRACE_CSV")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    a = ap.parse_args()
    n = a.n
    if a.trace_summary:
        trace_summary(a.trace_summary, a.out)
        return
    if a.summarize:
        summarize(a.summarize[0], a.summarize[1], n, a.out)
        return
    L = ctypes.CDLL(os.path.join(PKG, "libpfsm_testhooks.so"))
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.pfsm_test_gemm_x3.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, dbl, dbl, vp, i64,
                                    vp, i64, i32, vp, vp, vp]
    L.pfsm_test_gemm_f64.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, dbl, dbl, vp, vp, i64,
                                     vp, i32, vp]
    L.pfsm_test_pack_x3.argtypes = [vp, i32, i64, i64, i64, i32, vp, i64, vp]
    L.pfsm_test_x3_row_stride.argtypes = [i64]
    L.pfsm_test_x3_row_stride.restype = i64
    L.pfsm_test_x3_plain_stride.argtypes = [i64]
    L.pfsm_test_x3_plain_stride.restype = i64
    L.pfsm_test_gemm_x3_fs.argtypes = [i32, i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp,
                                       dbl, vp]
    L.pfsm_test_oz_split.argtypes = [vp, i64, i64, i64, i32, vp, vp, vp, vp]
    L.pfsm_test_gemm_oz.argtypes = [i64, i64, i64, i32, vp, vp, vp, vp, vp, i64, i32, vp]
    L.pfsm_test_oz_row_stride.argtypes = [i64]
    L.pfsm_test_oz_row_stride.restype = i64
    L.pfsm_test_refine_slices.restype = i32
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
    # the same update from plain BF16 operands (one product), as the mixed path runs it
    ldq = L.pfsm_test_x3_plain_stride(n)
    Aq = torch.empty(n * ldq, dtype=torch.int16, device=dev)
    Bq = torch.empty(n * ldq, dtype=torch.int16, device=dev)
    assert L.pfsm_test_pack_x3(P(M), 1, n, n, n, 32, P(Aq), ldq, s) == 0
    assert L.pfsm_test_pack_x3(P(M), 1, n, n, n, 32, P(Bq), ldq, s) == 0
    torch.cuda.synchronize()
    assert L.pfsm_test_gemm_x3_fs(2, 1, 0, n, n, n, P(Aq), ldq, P(Bq), ldq, P(X32), n, P(Y32), n, P(X32), n, P(eps),
                                  0.1, s) == 0
    torch.cuda.synchronize()
    del Ap, Bp, Aq, Bq, Y32, X32
    # FP64 folded-spectrum update, N x N x N
    B = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
    C = torch.randn(n, n, dtype=torch.float64, device=dev, generator=g)
    torch.cuda.synchronize()
    assert L.pfsm_test_gemm_f64(0, 0, 2, n, n, n, P(M), n, P(B), n, P(C), n, 0.1, 0.0, P(eps), P(C), n, None, 0,
                                s) == 0
    torch.cuda.synchronize()
    # int8 digit product with the refinement's digit count, C = M B
    s6 = L.pfsm_test_refine_slices()
    ldo = L.pfsm_test_oz_row_stride(n)
    Ad = torch.empty(s6 * n * ldo, dtype=torch.int8, device=dev)
    Bd = torch.empty(s6 * n * ldo, dtype=torch.int8, device=dev)
    ea = torch.empty(n, dtype=torch.int32, device=dev)
    eb = torch.empty(n, dtype=torch.int32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    assert L.pfsm_test_oz_split(P(M), n, n, n, s6, P(Ad), P(ea), P(info), s) == 0
    assert L.pfsm_test_oz_split(P(B), n, n, n, s6, P(Bd), P(eb), P(info), s) == 0
    assert L.pfsm_test_gemm_oz(n, n, n, s6, P(Ad), P(ea), P(Bd), P(eb), P(C), n, -1, s) == 0
    torch.cuda.synchronize()
    print("traffic probe done (n=%d)" % n, flush=True)


if __name__ == "__main__":
    main()
