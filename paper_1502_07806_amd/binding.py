"""ctypes binding of libpfsm (argument marshalling only).

Every step of the method runs inside libpfsm's HIP kernels; this module only
converts torch tensors into device pointers, leading dimensions and the
current HIP stream.  It raises if the library is missing: there is no
fallback implementation.

Layout: the library is column-major.  A torch tensor V whose strides are
(1, ld) is passed as is; any other layout is copied into column-major order
first.  Returned eigenvector matrices are column-major views (V.stride() ==
(1, n)); V[:, j] is the j-th eigenvector.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfsm.so")

PFSM_PREC = {"fp64": 0, "mixed_bf16": 1}
PFSM_SHIFT = {"fixed": 0, "rayleigh": 1}
INFO_TEXT = {0: "ok", -1: "non-finite eigenvalue",
             -2: "an eigenpair's residual exceeds the plan's threshold",
             -3: "submatrix eigensolver did not converge",
             -4: "an output vector lost its length: V_prev is not orthonormal",
             -5: "a diagonal entry of B is not a positive finite number"}
FLAG_NO_REFINE = 1
FLAG_FS_SPLIT = 2
FLAG_RESIDUALS = 4
FLAG_BACKWARD_SPLIT = 8


class PfsmDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("num_parts", ctypes.c_int32),
        ("part_offsets", ctypes.POINTER(ctypes.c_int64)),
        ("halo", ctypes.c_int64),
        ("iterations", ctypes.c_int32),
        ("fs_power", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("shift_mode", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("max_sweeps", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("resid_tol", ctypes.c_double),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpfsm.so; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libpfsm.so not found at %s: build it with "
                           "`python -m paper_1502_07806_amd.build_lib` (no fallback exists)" % path)
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    lib.pfsm_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PfsmDesc)]
    lib.pfsm_plan_create.restype = ctypes.c_int
    lib.pfsm_solve_static.argtypes = [vp, vp, i64, vp, i64, vp, vp, i64, vp, vp]
    lib.pfsm_solve_static.restype = ctypes.c_int
    lib.pfsm_residuals.argtypes = [vp, vp, sz, vp, vp]
    lib.pfsm_residuals.restype = ctypes.c_int
    lib.pfsm_refine_digit_count.argtypes = []
    lib.pfsm_refine_digit_count.restype = i32
    lib.pfsm_workspace_size.argtypes = [vp, ctypes.POINTER(sz)]
    lib.pfsm_workspace_size.restype = ctypes.c_int
    lib.pfsm_solve.argtypes = [vp, vp, i64, vp, i64, vp, vp, i64, vp, sz, vp, vp]
    lib.pfsm_solve.restype = ctypes.c_int
    lib.pfsm_backward.argtypes = [vp, vp, vp, i64, vp, vp, i64, dbl, vp, i64, vp, sz, vp, vp]
    lib.pfsm_backward.restype = ctypes.c_int
    lib.pfsm_diagnostics.argtypes = [vp, vp, i64, vp, vp, i64, vp, vp, sz, vp]
    lib.pfsm_diagnostics.restype = ctypes.c_int
    lib.pfsm_plan_destroy.argtypes = [vp]
    lib.pfsm_plan_destroy.restype = None
    lib.pfsm_plan_create_batched.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(PfsmDesc), i32]
    lib.pfsm_plan_create_batched.restype = ctypes.c_int
    lib.pfsm_solve_batched.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(vp),
                                       ctypes.POINTER(i64), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(i64), vp, sz, vp, vp]
    lib.pfsm_solve_batched.restype = ctypes.c_int
    lib.pfsm_batch_count.argtypes = [vp]
    lib.pfsm_batch_count.restype = i32
    lib.pfsm_autotune.argtypes = [vp, vp, sz, ctypes.POINTER(i32), vp]
    lib.pfsm_autotune.restype = ctypes.c_int
    lib.pfsm_set_tile_config.argtypes = [vp, i32]
    lib.pfsm_set_tile_config.restype = ctypes.c_int
    lib.pfsm_debug_stats.argtypes = [vp, vp, sz, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
    lib.pfsm_debug_stats.restype = ctypes.c_int
    lib.pfsm_timing_begin.argtypes = [vp, i32]
    lib.pfsm_timing_begin.restype = ctypes.c_int
    lib.pfsm_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(i32)]
    lib.pfsm_timing_read.restype = ctypes.c_int
    lib.pfsm_timing_end.argtypes = [vp]
    lib.pfsm_timing_end.restype = ctypes.c_int
    lib.pfsm_g2s_workspace_size.argtypes = [i64, ctypes.POINTER(sz)]
    lib.pfsm_g2s_workspace_size.restype = ctypes.c_int
    lib.pfsm_generalized_to_standard.argtypes = [i64, vp, i64, vp, i64, i32, vp, i64, vp, sz, vp, vp, vp]
    lib.pfsm_generalized_to_standard.restype = ctypes.c_int
    lib.pfsm_status_string.argtypes = [ctypes.c_int]
    lib.pfsm_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise RuntimeError(load_library().pfsm_status_string(status).decode())


def _colmajor(t: torch.Tensor) -> Tuple[torch.Tensor, int]:
    """Column-major view/copy of a 2-D float64 CUDA tensor and its leading dimension."""
    if t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2:
        raise ValueError("expected a 2-D float64 GPU tensor")
    n0, n1 = t.shape
    if t.stride(0) == 1 and t.stride(1) >= max(1, n0):
        return t, t.stride(1)
    c = t.t().contiguous().t()
    return c, max(1, n0)


def _stream_handle() -> int:
    return torch.cuda.current_stream().cuda_stream


def _desc(n, part_offsets, halo=-1, iterations=3, fs_power=2, alpha=0.0, shift_mode="fixed", precision="fp64",
          max_sweeps=0, refine=True, fs_split=False, residuals=False, resid_tol=0.0, backward_split=False):
    offs = (ctypes.c_int64 * len(part_offsets))(*[int(x) for x in part_offsets])
    flags = ((0 if refine else FLAG_NO_REFINE) | (FLAG_FS_SPLIT if fs_split else 0) |
             (FLAG_RESIDUALS if residuals else 0) | (FLAG_BACKWARD_SPLIT if backward_split else 0))
    d = PfsmDesc(int(n), len(part_offsets) - 1, offs, int(halo), int(iterations), int(fs_power), float(alpha),
                 PFSM_SHIFT[shift_mode], PFSM_PREC[precision], int(max_sweeps), flags, float(resid_tol))
    return d, offs  # keep offs alive while d is used


class Plan:
    """A PFSM plan: partition layout, submatrix policy and iteration options for order n."""

    def __init__(self, n: int, part_offsets: Sequence[int], halo: int = -1, iterations: int = 3,
                 fs_power: int = 2, alpha: float = 0.0, shift_mode: str = "fixed", precision: str = "fp64",
                 max_sweeps: int = 0, refine: bool = True, fs_split: bool = False, residuals: bool = False,
                 resid_tol: float = 0.0, backward_split: bool = False):
        lib = load_library()
        d, _keep = _desc(n, part_offsets, halo, iterations, fs_power, alpha, shift_mode, precision, max_sweeps,
                         refine, fs_split, residuals, resid_tol, backward_split)
        h = ctypes.c_void_p()
        _check(lib.pfsm_plan_create(ctypes.byref(h), ctypes.byref(d)))
        self._h = h
        self.n = int(n)
        self.part_offsets = [int(x) for x in part_offsets]
        self.precision = precision
        sz = ctypes.c_size_t()
        _check(lib.pfsm_workspace_size(h, ctypes.byref(sz)))
        self.workspace_bytes = int(sz.value)
        self._work = None
        self._info = None

    def _workspace(self, device) -> torch.Tensor:
        if self._work is None or self._work.device != device:
            self._work = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
            self._info = torch.zeros(1, dtype=torch.int32, device=device)
        return self._work

    @property
    def info(self) -> torch.Tensor:
        return self._info

    def solve(self, A: torch.Tensor, V_prev: torch.Tensor, out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None,
              check: bool = True):
        n = self.n
        if A.shape != (n, n) or V_prev.shape != (n, n):
            raise ValueError("A and V_prev must be %d x %d" % (n, n))
        Ac, lda = _colmajor(A)  # A is symmetric: row-major storage of A is A^T = A as well
        Vc, ldv = _colmajor(V_prev)
        work = self._workspace(A.device)
        if out is None:
            lam = torch.empty(n, dtype=torch.float64, device=A.device)
            Vout = torch.empty((n, n), dtype=torch.float64, device=A.device).t()
        else:
            lam, Vout = out
        if Vout.stride(0) != 1:
            raise ValueError("out V must be column-major (stride(0) == 1)")
        _check(load_library().pfsm_solve(self._h, Ac.data_ptr(), lda, Vc.data_ptr(), ldv, lam.data_ptr(),
                                          Vout.data_ptr(), Vout.stride(1), work.data_ptr(), self.workspace_bytes,
                                          self._info.data_ptr(), _stream_handle()))
        if check:
            self.check()
        return lam, Vout

    def solve_static(self, A: torch.Tensor, V_prev: torch.Tensor,
                     out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None, check: bool = True):
        """solve() through pfsm_solve_static: the library's own device workspace
        (PFSM_STATIC_SCRATCH_BYTES), no allocation inside the call."""
        n = self.n
        if A.shape != (n, n) or V_prev.shape != (n, n):
            raise ValueError("A and V_prev must be %d x %d" % (n, n))
        Ac, lda = _colmajor(A)
        Vc, ldv = _colmajor(V_prev)
        if self._info is None or self._info.device != A.device:
            self._info = torch.zeros(1, dtype=torch.int32, device=A.device)
        if out is None:
            lam = torch.empty(n, dtype=torch.float64, device=A.device)
            Vout = torch.empty((n, n), dtype=torch.float64, device=A.device).t()
        else:
            lam, Vout = out
        if Vout.stride(0) != 1:
            raise ValueError("out V must be column-major (stride(0) == 1)")
        _check(load_library().pfsm_solve_static(self._h, Ac.data_ptr(), lda, Vc.data_ptr(), ldv, lam.data_ptr(),
                                                 Vout.data_ptr(), Vout.stride(1), self._info.data_ptr(),
                                                 _stream_handle()))
        if check:
            self.check()
        return lam, Vout

    def residuals(self) -> torch.Tensor:
        """Per-column residuals ||A v_i - lambda_i v_i|| of the last solve (output order);
        the plan must have been made with residuals=True or resid_tol > 0."""
        if self._work is None:
            raise RuntimeError("no solve has run with this plan's workspace")
        r = torch.empty(self.n, dtype=torch.float64, device=self._work.device)
        _check(load_library().pfsm_residuals(self._h, self._work.data_ptr(), self.workspace_bytes, r.data_ptr(),
                                             _stream_handle()))
        return r

    def check(self):
        """Synchronise and raise if the device reported a failure."""
        code = int(self._info.item())
        if code != 0:
            text = INFO_TEXT.get(code, "overlap matrix not positive definite at column %d" % code)
            raise RuntimeError("pfsm device info %d: %s" % (code, text))

    def backward(self, lam: torch.Tensor, V: torch.Tensor, grad_lam: Optional[torch.Tensor],
                 grad_V: Optional[torch.Tensor], eta: float = 1e-8) -> torch.Tensor:
        n = self.n
        Vc, ldv = _colmajor(V)
        work = self._workspace(V.device)
        gl = grad_lam.contiguous() if grad_lam is not None else None
        if grad_V is not None:
            gVc, ldg = _colmajor(grad_V)
        else:
            gVc, ldg = None, n
        gA = torch.empty((n, n), dtype=torch.float64, device=V.device).t()
        _check(load_library().pfsm_backward(self._h, lam.contiguous().data_ptr(), Vc.data_ptr(), ldv,
                                             gl.data_ptr() if gl is not None else None,
                                             gVc.data_ptr() if gVc is not None else None, ldg, float(eta),
                                             gA.data_ptr(), n, work.data_ptr(), self.workspace_bytes,
                                             self._info.data_ptr(), _stream_handle()))
        return gA

    def diagnostics(self, A: torch.Tensor, lam: torch.Tensor, V: torch.Tensor) -> Tuple[float, float]:
        """(||AV - V diag(lam)||_F / ||A||_F, ||V^T V - I||_F), computed on the device in FP64."""
        Ac, lda = _colmajor(A)
        Vc, ldv = _colmajor(V)
        work = self._workspace(A.device)
        out = torch.empty(2, dtype=torch.float64, device=A.device)
        _check(load_library().pfsm_diagnostics(self._h, Ac.data_ptr(), lda, lam.contiguous().data_ptr(),
                                                Vc.data_ptr(), ldv, out.data_ptr(), work.data_ptr(),
                                                self.workspace_bytes, _stream_handle()))
        o = out.cpu()
        return float(o[0]), float(o[1])

    def autotune(self) -> int:
        """Pick the fastest split-BF16 tile configuration for this plan (mixed precision); returns it (-1: none)."""
        work = self._workspace(torch.device("cuda", torch.cuda.current_device()))
        c = ctypes.c_int32()
        _check(load_library().pfsm_autotune(self._h, work.data_ptr(), self.workspace_bytes, ctypes.byref(c),
                                            _stream_handle()))
        return int(c.value)

    def set_tile_config(self, cfg: int):
        _check(load_library().pfsm_set_tile_config(self._h, int(cfg)))

    def debug_stats(self):
        """Counters of the last solve: per-submatrix sweeps and rotating pair problems, refinement clusters."""
        P = len(self.part_offsets) - 1
        cap = 2 * P + 5
        buf = (ctypes.c_int32 * cap)()
        cnt = ctypes.c_int32()
        _check(load_library().pfsm_debug_stats(self._h, self._work.data_ptr(), self.workspace_bytes, buf, cap,
                                               ctypes.byref(cnt)))
        v = list(buf)
        return {"converged_sweep": v[0:2 * P:2], "rotating_pairs": v[1:2 * P:2],
                "clusters": v[2 * P], "multi_clusters": v[2 * P + 1], "max_cluster": v[2 * P + 2],
                "fs_band_products": v[2 * P + 3], "correction_band": v[2 * P + 4]}

    # -- stage timing (instrumentation for benchmarks)
    TIMING_BOUNDS = 27
    STAGES = (["basis_change", "step_length", "submatrix_eigh"]
              + [x for i in range(8) for x in ("fs_shift_%d" % i, "fs_update_%d" % i)]
              + ["overlap", "cholesky_qr", "rayleigh", "ordering", "back_rotation", "refine_product", "refine_rr"])

    def timing_begin(self, max_solves: int):
        _check(load_library().pfsm_timing_begin(self._h, int(max_solves)))

    def timing_read(self):
        """List (one entry per recorded solve) of {stage: milliseconds}."""
        per = self.TIMING_BOUNDS - 1
        cap = 4096 * per
        buf = (ctypes.c_float * cap)()
        cnt = ctypes.c_int32()
        _check(load_library().pfsm_timing_read(self._h, buf, cap, ctypes.byref(cnt)))
        out = []
        for sv in range(cnt.value):
            out.append({name: float(buf[sv * per + k]) for k, name in enumerate(self.STAGES)})
        return out

    def timing_end(self):
        _check(load_library().pfsm_timing_end(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pfsm_plan_destroy(h)
            self._h = None


class BatchedPlan:
    """Many independent PFSM instances (e.g. k-points / spins) solved by one call.

    specs: list of dicts with the Plan keyword arguments plus "n" and "part_offsets".
    The call is capturable into one CUDA/HIP graph (torch.cuda.graph)."""

    def __init__(self, specs):
        lib = load_library()
        self.count = len(specs)
        descs = (PfsmDesc * self.count)()
        keep = []
        for i, sp in enumerate(specs):
            sp = dict(sp)
            d, k = _desc(sp.pop("n"), sp.pop("part_offsets"), **sp)
            descs[i] = d
            keep.append(k)
        h = ctypes.c_void_p()
        _check(lib.pfsm_plan_create_batched(ctypes.byref(h), descs, self.count))
        self._h = h
        self.n = [int(sp["n"]) for sp in specs]
        sz = ctypes.c_size_t()
        _check(lib.pfsm_workspace_size(h, ctypes.byref(sz)))
        self.workspace_bytes = int(sz.value)
        self._work = None
        self.info = None

    def _workspace(self, device):
        if self._work is None or self._work.device != device:
            self._work = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
            self.info = torch.zeros(self.count, dtype=torch.int32, device=device)
        return self._work

    def outputs(self, device):
        """Allocate (lams, Vs) output tensors (column-major eigenvector matrices)."""
        lams = [torch.empty(n, dtype=torch.float64, device=device) for n in self.n]
        Vs = [torch.empty((n, n), dtype=torch.float64, device=device).t() for n in self.n]
        return lams, Vs

    def solve(self, As, Vprevs, out=None, check: bool = True):
        dev = As[0].device
        work = self._workspace(dev)
        cols = [_colmajor(A) for A in As]
        vcols = [_colmajor(V) for V in Vprevs]
        lams, Vs = out if out is not None else self.outputs(dev)
        for V in Vs:
            if V.stride(0) != 1:
                raise ValueError("output eigenvector matrices must be column-major")
        c = self.count
        P = ctypes.c_void_p * c
        I = ctypes.c_int64 * c
        _check(load_library().pfsm_solve_batched(
            self._h, P(*[a.data_ptr() for a, _ in cols]), I(*[l for _, l in cols]),
            P(*[v.data_ptr() for v, _ in vcols]), I(*[l for _, l in vcols]),
            P(*[x.data_ptr() for x in lams]), P(*[x.data_ptr() for x in Vs]), I(*[x.stride(1) for x in Vs]),
            work.data_ptr(), self.workspace_bytes, self.info.data_ptr(), _stream_handle()))
        self._keep = (cols, vcols)  # inputs may be temporaries; keep them alive until the next call
        if check:
            self.check()
        return lams, Vs

    def check(self):
        codes = self.info.cpu().tolist()
        bad = [(i, c) for i, c in enumerate(codes) if c != 0]
        if bad:
            raise RuntimeError("pfsm batched device info (instance, code): %s" % bad[:8])

    def autotune(self):
        work = self._workspace(torch.device("cuda", torch.cuda.current_device()))
        c = ctypes.c_int32()
        _check(load_library().pfsm_autotune(self._h, work.data_ptr(), self.workspace_bytes, ctypes.byref(c),
                                            _stream_handle()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.pfsm_plan_destroy(h)
            self._h = None


def solve(A: torch.Tensor, V_prev: torch.Tensor, plan: Plan, check: bool = True):
    """(lam, V) = PFSM step for (A, V_prev) with `plan`."""
    return plan.solve(A, V_prev, check=check)


class PFSMFunction(torch.autograd.Function):
    """(lam, V) = PFSMFunction.apply(A, V_prev, plan, eta); gradient flows to A only.

    The backward pass is the eigen-adjoint of A = V diag(lam) V^T computed by
    libpfsm (pfsm_backward); V_prev and the plan get no gradient."""

    @staticmethod
    def forward(ctx, A, V_prev, plan: Plan, eta: float = 1e-8):
        lam, V = plan.solve(A, V_prev)
        ctx.plan = plan
        ctx.eta = eta
        ctx.save_for_backward(lam, V)
        return lam, V

    @staticmethod
    def backward(ctx, grad_lam, grad_V):
        lam, V = ctx.saved_tensors
        gA = ctx.plan.backward(lam, V, grad_lam, grad_V, ctx.eta)
        return gA, None, None, None


def generalized_to_standard(A: torch.Tensor, B: torch.Tensor, iterations: int, out: Optional[torch.Tensor] = None,
                            residuals: bool = False, check: bool = True):
    """Z = B^{-1} A for A x = lambda B x (Implementation section, Eqs. 13-15):
    `iterations` steps of Z_{k+1} = (I - D^{-1} B) Z_k + D^{-1} A from Z_0 = A,
    D = diag(B), each one FP64 product on the GPU (pfsm_generalized_to_standard).

    A and B are n x n float64 GPU tensors (B symmetric).  Z is returned as a
    column-major tensor (stride(0) == 1) holding Z itself; with `residuals`,
    also the n_it values ||A - B Z_k||_F / ||A||_F (k = 0 .. iterations-1)."""
    n = A.shape[0]
    if A.shape != (n, n) or B.shape != (n, n):
        raise ValueError("A and B must be square and of the same order")
    Ac, lda = _colmajor(A)
    Bc, ldb = _colmajor(B)
    L = load_library()
    need = ctypes.c_size_t(0)
    _check(L.pfsm_g2s_workspace_size(n, ctypes.byref(need)))
    work = torch.empty(need.value + 256, dtype=torch.uint8, device=A.device)
    wp = (work.data_ptr() + 255) // 256 * 256
    Z = out if out is not None else torch.empty((n, n), dtype=torch.float64, device=A.device).t()
    if Z.stride(0) != 1:
        raise ValueError("out must be column-major (stride(0) == 1)")
    res = torch.empty(max(iterations, 1), dtype=torch.float64, device=A.device) if residuals else None
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _check(L.pfsm_generalized_to_standard(n, Ac.data_ptr(), lda, Bc.data_ptr(), ldb, int(iterations), Z.data_ptr(),
                                          Z.stride(1), wp, need.value, res.data_ptr() if res is not None else None,
                                          info.data_ptr(), _stream_handle()))
    if check:
        code = int(info.item())
        if code != 0:
            raise RuntimeError("pfsm device info %d: %s" % (code, INFO_TEXT.get(code, "error")))
    if residuals:
        return Z, res[:iterations], info
    return Z, info
