"""Thin Python binding of libjacobi (include/jacobi.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Functions take and return torch tensors on the current HIP device;
the current torch stream is passed to the library.  Matrices follow the usual
torch (row-major) semantics at this level and are handed to the library in
its column-major layout: a column-major M is stored as the row-major buffer of
M^T, so symmetric inputs pass through unchanged and outputs are returned as
transposed views.

Importing this module never falls back to anything: if libjacobi.so is
missing, load() raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjacobi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "jacobi.h")

PRECOND = {"none": 0, "fp32": 1, "mlp": 2}
VARIANT = {"auto": 0, "element": 1, "blocked": 2}
STAGE1 = {"auto": 0, "jacobi": 1, "tridiag": 2}
SVD_QR = {"auto": 0, "off": 1, "on": 2}
PREC = {"fp32": 0, "fp16": 1, "bf16": 2}
JAC_HIST = 65


class JacOpts(ctypes.Structure):
    _fields_ = [("precond", ctypes.c_int), ("variant", ctypes.c_int), ("block_b", ctypes.c_int),
                ("max_sweeps", ctypes.c_int), ("fp32_tol", ctypes.c_double),
                ("fp32_max_sweeps", ctypes.c_int), ("mlp", ctypes.c_void_p),
                ("theta", ctypes.c_void_p), ("fallback_tol", ctypes.c_double),
                ("inner_sweeps", ctypes.c_int), ("profile", ctypes.c_int), ("stage1", ctypes.c_int),
                ("svd_qr", ctypes.c_int), ("stage1_prec", ctypes.c_int)]


class JacBatchedOpts(ctypes.Structure):
    _fields_ = [("precond", ctypes.c_int), ("fp32_tol", ctypes.c_double), ("max_sweeps", ctypes.c_int),
                ("reserved", ctypes.c_int)]


class JacBatchedStats(ctypes.Structure):
    _fields_ = [("topup_sweeps", ctypes.c_int), ("series_failed", ctypes.c_int), ("graph_built", ctypes.c_int),
                ("classes", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class JacStats(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int), ("fp32_sweeps", ctypes.c_int),
                ("rotations", ctypes.c_longlong), ("fp32_rotations", ctypes.c_longlong),
                ("used_fallback", ctypes.c_int), ("nrmA", ctypes.c_double),
                ("off0", ctypes.c_double), ("off_final", ctypes.c_double),
                ("off_hist", ctypes.c_double * JAC_HIST), ("stage_ms", ctypes.c_float * 8),
                ("step_ms", ctypes.c_double), ("step_launches", ctypes.c_longlong),
                ("fp32_step_ms", ctypes.c_double), ("fp32_step_launches", ctypes.c_longlong),
                ("kern_ms", ctypes.c_double * 8), ("kern_launches", ctypes.c_longlong * 8),
                ("kern_work", ctypes.c_longlong * 8), ("start_resid", ctypes.c_double),
                ("fp32_method", ctypes.c_int), ("svd_qr_used", ctypes.c_int), ("qr_ms", ctypes.c_float)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_
             if f not in ("off_hist", "stage_ms", "kern_ms", "kern_launches", "kern_work")}
        names = ["inner64", "update64", "inner32", "update32", "elem64", "elem32", "tridiag_reduce",
                 "tridiag_rest"]
        d["kernels"] = {names[i]: {"ms": self.kern_ms[i], "launches": self.kern_launches[i],
                                   "tiles": self.kern_work[i] >> 32 if i < 4 else 0,
                                   "chunks": self.kern_work[i] & 0xFFFFFFFF if i < 4 else 0}
                        for i in range(8) if self.kern_launches[i]}
        d["off_hist"] = list(self.off_hist[: self.sweeps + 1])
        d["stage_ms"] = dict(zip(["start", "mgs", "similarity", "sweeps", "output", "total", "checks"],
                                 list(self.stage_ms)[:7]))
        return d


class JacobiError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} returned {code}: {msg}")
        self.code = code


_lib = None
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double


def load():
    """Load libjacobi.so from the package directory (raises if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "syev_jacobi": (_i, [_vp, _i, _i, _vp, _vp, _d, ctypes.POINTER(_i)]),
        "syev_jacobi_ex": (_i, [_vp, _i, _i, _vp, _vp, _i, _d, ctypes.POINTER(JacOpts),
                                ctypes.POINTER(JacStats), _vp]),
        "syev_jacobi_noalloc": (_i, [_vp, _i, _i, _vp, _vp, _i, _d, ctypes.POINTER(JacOpts),
                                     ctypes.POINTER(JacStats), _vp]),
        "syev_jacobi_warm": (_i, [_vp, _i, _i, _vp, _i, _vp, _vp, _i, _d, ctypes.POINTER(JacOpts),
                                  ctypes.POINTER(JacStats), _vp]),
        "gesvd_jacobi": (_i, [_vp, _i, _i, _i, _vp, _vp, _i, _vp, _i, _d, ctypes.POINTER(_i)]),
        "gesvd_jacobi_ex": (_i, [_vp, _i, _i, _i, _vp, _vp, _i, _vp, _i, _d, ctypes.POINTER(JacOpts),
                                 ctypes.POINTER(JacStats), _vp]),
        "syev_jacobi_batched": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(_vp), ctypes.POINTER(_i),
                                     ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i), _d, _vp, _vp,
                                     _vp]),
        "syev_jacobi_batched_ex": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(_vp), ctypes.POINTER(_i),
                                        ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i), _d, _vp, _vp,
                                        _vp, ctypes.POINTER(JacBatchedOpts), ctypes.POINTER(JacBatchedStats), _vp]),
        "jac_autotune_batched": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(_vp), ctypes.POINTER(_i), _d, _vp]),
        "jac_autotune_batched_ex": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(_vp), ctypes.POINTER(_i), _d,
                                         ctypes.POINTER(JacBatchedOpts), _vp]),
        "jac_tune_entry": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "jac_tune_entry_ex": (_i, [_i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "jac_tune_clear": (_i, []),
        "jac_parallel_steps": (_i, [_vp, _i, _i, _vp, _i, _i, _i, _d,
                                    ctypes.POINTER(ctypes.c_longlong), _vp]),
        "jac_round_robin_pairs": (_i, [_i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
        "jac_mgs": (_i, [_vp, _i, _i, _i, _vp]),
        "jac_similarity": (_i, [_vp, _i, _i, _vp, _i, _vp, _i, _vp]),
        "jac_qr_orth": (_i, [_vp, _i, _i, ctypes.POINTER(_i), _vp]),
        "jac_eig_fp32": (_i, [_vp, _i, _i, _vp, _i, _vp, _d, _i, ctypes.POINTER(_i), _vp]),
        "jac_sytrd_f32": (_i, [_vp, _i, _i, _vp, _vp, _vp, _vp, _i, _vp]),
        "jac_tridiag_eig": (_i, [_vp, _vp, _i, _vp, _vp, _i, _vp]),
        "jac_tridiag_backtransform": (_i, [_vp, _i, _vp, _i, _vp, _i, _vp]),
        "jac_eig_fp32_tridiag": (_i, [_vp, _i, _i, _vp, _i, _vp, _vp]),
        "jac_gemm_f64": (_i, [_i, _i, _i, _i, _i, _d, _vp, _i, _vp, _i, _d, _vp, _i, _vp]),
        "jac_gemm_f32": (_i, [_i, _i, _i, _i, _i, ctypes.c_float, _vp, _i, _vp, _i, ctypes.c_float,
                              _vp, _i, _vp]),
        "jac_mlp_create": (_i, [_i, _i, _i, _i, ctypes.c_ulonglong, ctypes.POINTER(_vp)]),
        "jac_mlp_free": (None, [_vp]),
        "jac_mlp_num_params": (ctypes.c_longlong, [_vp]),
        "jac_mlp_shape": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i),
                               ctypes.POINTER(ctypes.c_longlong)]),
        "jac_mlp_get": (_i, [_vp, _i, _vp]),
        "jac_mlp_set": (_i, [_vp, _i, _vp]),
        "jac_mlp_set_adam": (_i, [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_longlong]),
        "jac_mlp_forward": (_i, [_vp, _vp, _i, _vp, _i, _vp]),
        "jac_mlp_predict": (_i, [_vp, _vp, _vp, _i, _vp]),
        "jac_mlp_grads": (_i, [_vp, _vp, _vp, ctypes.c_longlong, _i, _vp, _vp]),
        "jac_mlp_adamw": (_i, [_vp, ctypes.c_float, ctypes.c_float, _vp]),
        "jac_mlp_train_step": (_i, [_vp, _vp, _vp, ctypes.c_longlong, _i, ctypes.c_float, ctypes.c_float, _vp,
                                    _vp]),
        "jac_mlp_pack_targets": (_i, [_vp, _i, _i, ctypes.c_longlong, _i, _vp, ctypes.c_longlong, _vp]),
        "jac_mlp_pack_targets_ex": (_i, [_vp, _i, _i, ctypes.c_longlong, _i, _vp, ctypes.c_longlong, _i, _vp]),
        "jac_mlp_save": (_i, [_vp, ctypes.c_char_p]),
        "jac_mlp_load": (_i, [_vp, ctypes.c_char_p]),
        "jac_workspace_bytes": (ctypes.c_size_t, [_i, ctypes.POINTER(JacOpts)]),
        "jac_release_workspace": (None, []),
        "jac_last_error": (ctypes.c_char_p, []),
        "jac_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_symbols():
    """Function names declared in include/jacobi.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", txt)) - {"sizeof"})


def last_error() -> str:
    return load().jac_last_error().decode()


def _check(fn, code, ok=(0,)):
    if code not in ok:
        raise JacobiError(fn, code, last_error())
    return code


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x: torch.Tensor, dtype=torch.float64):
    if not x.is_cuda:
        raise ValueError("expected a device tensor")
    if x.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {x.dtype}")
    return x


def _colmajor(M: torch.Tensor) -> torch.Tensor:
    """Buffer whose column-major reading is M (the row-major buffer of M^T)."""
    return M.t().contiguous()


def _opts(precond="fp32", variant="auto", block_b=0, max_sweeps=0, fp32_tol=0.0, fp32_max_sweeps=0,
          fallback_tol=0.0, inner_sweeps=0, profile=0, mlp=None, theta=None, stage1="auto", stage1_prec="fp32"):
    o = JacOpts()
    o.stage1 = STAGE1[stage1] if isinstance(stage1, str) else int(stage1)
    o.stage1_prec = PREC[stage1_prec] if isinstance(stage1_prec, str) else int(stage1_prec)
    if mlp is not None:
        o.mlp = mlp.h.value
    if theta is not None:
        o.theta = _dev(theta, torch.float32).data_ptr()
    o.precond = PRECOND[precond] if isinstance(precond, str) else int(precond)
    o.variant = VARIANT[variant] if isinstance(variant, str) else int(variant)
    o.block_b = block_b
    o.max_sweeps = max_sweeps
    o.fp32_tol = fp32_tol
    o.fp32_max_sweeps = fp32_max_sweeps
    o.fallback_tol = fallback_tol
    o.inner_sweeps = inner_sweeps
    o.profile = profile
    return o


def syev_jacobi(A: torch.Tensor, tol: float = 0.0):
    """Algorithm 4.1 (FP32 start), library's variant: returns (W, V, sweeps)."""
    L = load()
    A = _dev(A)
    n = A.shape[0]
    Ac = _colmajor(A)
    W = torch.empty(n, dtype=torch.float64, device=A.device)
    Vb = torch.empty((n, n), dtype=torch.float64, device=A.device)
    sw = ctypes.c_int(0)
    torch.cuda.synchronize()
    code = L.syev_jacobi(_vp(Ac.data_ptr()), n, max(n, 1), _vp(W.data_ptr()), _vp(Vb.data_ptr()), tol,
                         ctypes.byref(sw))
    _check("syev_jacobi", code, ok=(0, 1))
    return W, Vb.t(), sw.value, code


def syev_jacobi_ex(A: torch.Tensor, tol: float = 0.0, precond="fp32", variant="auto", max_sweeps=0,
                   fp32_tol=0.0, fp32_max_sweeps=0, block_b=0, allow_unconverged=False, inner_sweeps=0,
                   mlp=None, theta=None, fallback_tol=0.0, profile=0, stage1="auto", stage1_prec="fp32"):
    """Returns (W, V, stats dict, info).  precond="mlp" takes the network `mlp` (Mlp) and its
    input `theta` (device float32 tensor of n_in values)."""
    if theta is not None:
        theta = _dev(theta, torch.float32).contiguous()
    L = load()
    A = _dev(A)
    n = A.shape[0]
    Ac = _colmajor(A)
    W = torch.empty(n, dtype=torch.float64, device=A.device)
    Vb = torch.empty((n, n), dtype=torch.float64, device=A.device)
    o = _opts(precond, variant, block_b, max_sweeps, fp32_tol, fp32_max_sweeps, fallback_tol=fallback_tol,
              inner_sweeps=inner_sweeps, profile=profile, mlp=mlp, theta=theta, stage1=stage1,
              stage1_prec=stage1_prec)
    st = JacStats()
    code = L.syev_jacobi_ex(_vp(Ac.data_ptr()), n, max(n, 1), _vp(W.data_ptr()), _vp(Vb.data_ptr()),
                            max(n, 1), tol, ctypes.byref(o), ctypes.byref(st), _stream())
    _check("syev_jacobi_ex", code, ok=(0, 1) if allow_unconverged else (0,))
    return W, Vb.t(), st.as_dict(), code


def noalloc_bytes() -> int:
    """JAC_NOALLOC_BYTES of include/jacobi.h: the fixed device array of syev_jacobi_noalloc."""
    m = re.search(r"#define\s+JAC_NOALLOC_BYTES\s+\(\(size_t\)(\d+)\s*<<\s*(\d+)\)", open(HEADER).read())
    return int(m.group(1)) << int(m.group(2))


def syev_jacobi_noalloc(A: torch.Tensor, tol: float = 0.0, precond="fp32", variant="auto", max_sweeps=0,
                        fp32_tol=0.0, inner_sweeps=0, check=True, stage1="auto"):
    """The allocation-free variant of syev_jacobi_ex (workspace in the library's fixed device array).
    Returns (W, V, stats dict, info); with check=False the return code is passed back unchecked."""
    L = load()
    A = _dev(A)
    n = A.shape[0]
    Ac = _colmajor(A)
    W = torch.empty(n, dtype=torch.float64, device=A.device)
    Vb = torch.empty((n, n), dtype=torch.float64, device=A.device)
    o = _opts(precond, variant, 0, max_sweeps, fp32_tol, inner_sweeps=inner_sweeps, stage1=stage1)
    st = JacStats()
    code = L.syev_jacobi_noalloc(_vp(Ac.data_ptr()), n, max(n, 1), _vp(W.data_ptr()), _vp(Vb.data_ptr()),
                                 max(n, 1), tol, ctypes.byref(o), ctypes.byref(st), _stream())
    if check:
        _check("syev_jacobi_noalloc", code)
    return W, Vb.t(), st.as_dict(), code


def syev_jacobi_raw(A_ptr, n, lda, W_ptr, V_ptr, ldv, tol, opts: JacOpts, stats: JacStats | None = None,
                    stream=None):
    """Direct call with raw device pointers (used by the benchmark's timed loop)."""
    L = load()
    return L.syev_jacobi_ex(_vp(A_ptr), n, lda, _vp(W_ptr), _vp(V_ptr), ldv, tol, ctypes.byref(opts),
                            ctypes.byref(stats) if stats is not None else None,
                            stream if stream is not None else _stream())


def syev_jacobi_warm(A: torch.Tensor, Q0: torch.Tensor, tol: float = 0.0, max_sweeps=0):
    L = load()
    A = _dev(A)
    n = A.shape[0]
    Ac = _colmajor(A)
    Qc = _colmajor(_dev(Q0))
    W = torch.empty(n, dtype=torch.float64, device=A.device)
    Vb = torch.empty((n, n), dtype=torch.float64, device=A.device)
    o = _opts("fp32", "auto", 0, max_sweeps)
    st = JacStats()
    code = L.syev_jacobi_warm(_vp(Ac.data_ptr()), n, max(n, 1), _vp(Qc.data_ptr()), max(n, 1),
                              _vp(W.data_ptr()), _vp(Vb.data_ptr()), max(n, 1), tol, ctypes.byref(o),
                              ctypes.byref(st), _stream())
    _check("syev_jacobi_warm", code)
    return W, Vb.t(), st.as_dict(), code


def gesvd_jacobi(A: torch.Tensor, tol: float = 0.0):
    """Algorithm 5.2 (FP32 Gram start) with default options on the null stream: returns
    (S descending, U, V, sweeps, info)."""
    L = load()
    A = _dev(A)
    m, n = A.shape
    Ac = _colmajor(A)
    S = torch.empty(n, dtype=torch.float64, device=A.device)
    Ub = torch.empty((n, m), dtype=torch.float64, device=A.device)
    Vb = torch.empty((n, n), dtype=torch.float64, device=A.device)
    sw = ctypes.c_int(0)
    torch.cuda.synchronize()
    code = L.gesvd_jacobi(_vp(Ac.data_ptr()), m, n, max(m, 1), _vp(S.data_ptr()), _vp(Ub.data_ptr()), max(m, 1),
                          _vp(Vb.data_ptr()), max(n, 1), tol, ctypes.byref(sw))
    _check("gesvd_jacobi", code, ok=(0, 1))
    return S, Ub.t(), Vb.t(), sw.value, code


def gesvd_jacobi_ex(A: torch.Tensor, tol: float = 0.0, precond="fp32", max_sweeps=0, variant="auto",
                    allow_unconverged=False, stage1="auto", svd_qr="auto"):
    """Thin SVD A = U diag(S) V^T (m >= n): returns (S descending, U, V, stats, info).
    svd_qr: "auto" / "off" / "on" (QR first, for m >> n)."""
    L = load()
    A = _dev(A)
    m, n = A.shape
    Ac = _colmajor(A)
    S = torch.empty(n, dtype=torch.float64, device=A.device)
    Ub = torch.empty((n, m), dtype=torch.float64, device=A.device)
    Vb = torch.empty((n, n), dtype=torch.float64, device=A.device)
    o = _opts(precond, variant, 0, max_sweeps, stage1=stage1)
    o.svd_qr = SVD_QR[svd_qr]
    st = JacStats()
    code = L.gesvd_jacobi_ex(_vp(Ac.data_ptr()), m, n, max(m, 1), _vp(S.data_ptr()), _vp(Ub.data_ptr()),
                             max(m, 1), _vp(Vb.data_ptr()), max(n, 1), tol, ctypes.byref(o), ctypes.byref(st),
                             _stream())
    _check("gesvd_jacobi_ex", code, ok=(0, 1) if allow_unconverged else (0,))
    d = st.as_dict()
    d["rotations_per_sweep"] = list(st.off_hist[1: st.sweeps + 1])
    d.pop("off_hist")
    return S, Ub.t(), Vb.t(), d, code


class Batch:
    """Device buffers and pointer arrays for the batched entry points over a list of symmetric
    matrices (kept alive so that repeated calls replay the same graph)."""

    def __init__(self, mats):
        self.A = [_dev(a).contiguous() for a in mats]    # symmetric: row/column-major agree
        self.n = [a.shape[0] for a in self.A]
        dev = self.A[0].device
        self.W = [torch.empty(n, dtype=torch.float64, device=dev) for n in self.n]
        self.V = [torch.empty((n, n), dtype=torch.float64, device=dev) for n in self.n]
        b = len(self.A)
        self.sweeps = torch.zeros(b, dtype=torch.int32, device=dev)
        self.sweeps32 = torch.zeros(b, dtype=torch.int32, device=dev)
        self.info = torch.zeros(b, dtype=torch.int32, device=dev)
        self.c_n = (_i * b)(*self.n)
        self.c_A = (_vp * b)(*[a.data_ptr() for a in self.A])
        self.c_W = (_vp * b)(*[w.data_ptr() for w in self.W])
        self.c_V = (_vp * b)(*[v.data_ptr() for v in self.V])
        self.c_ld = (_i * b)(*self.n)
        self.stats = {}

    @staticmethod
    def _opts(precond, fp32_tol, max_sweeps):
        return JacBatchedOpts(PRECOND[precond], float(fp32_tol), int(max_sweeps), 0)

    def run(self, tol: float = 0.0, stream=None, precond: str = "none", fp32_tol: float = 0.0, max_sweeps: int = 0,
            plain_api: bool = False):
        """One batched solve.  plain_api: through syev_jacobi_batched (no options) instead of the _ex
        entry point."""
        L = load()
        st = stream if stream is not None else _stream()
        if plain_api:
            code = L.syev_jacobi_batched(len(self.A), self.c_n, self.c_A, self.c_ld, self.c_W, self.c_V, self.c_ld,
                                         tol, _vp(self.sweeps.data_ptr()), _vp(self.info.data_ptr()), st)
            _check("syev_jacobi_batched", code)
            return
        o = self._opts(precond, fp32_tol, max_sweeps)
        s = JacBatchedStats()
        code = L.syev_jacobi_batched_ex(len(self.A), self.c_n, self.c_A, self.c_ld, self.c_W, self.c_V, self.c_ld,
                                        tol, _vp(self.sweeps.data_ptr()), _vp(self.info.data_ptr()),
                                        _vp(self.sweeps32.data_ptr()), ctypes.byref(o), ctypes.byref(s), st)
        _check("syev_jacobi_batched_ex", code)
        self.stats = s.as_dict()

    def autotune(self, tol: float = 0.0, precond: str = "none", fp32_tol: float = 0.0):
        L = load()
        if precond == "none" and fp32_tol == 0.0:
            code = L.jac_autotune_batched(len(self.A), self.c_n, self.c_A, self.c_ld, tol, _stream())
        else:
            o = self._opts(precond, fp32_tol, 0)
            code = L.jac_autotune_batched_ex(len(self.A), self.c_n, self.c_A, self.c_ld, tol, ctypes.byref(o),
                                             _stream())
        _check("jac_autotune_batched", code)

    def results(self):
        """(W list, V list (columns = eigenvectors), sweeps, info) after the call."""
        return self.W, [v.t() for v in self.V], self.sweeps.cpu().numpy(), self.info.cpu().numpy()


def jac_tune_clear():
    """Forget the batched path's tuned table of this process."""
    load().jac_tune_clear()


def jac_tune_entry(n: int, precond: str = "none"):
    """(inner-sweep cap, FP64 sweeps, FP32 sweeps) of the batched path's table for order n."""
    a, b, c = _i(0), _i(0), _i(0)
    _check("jac_tune_entry_ex", load().jac_tune_entry_ex(n, PRECOND[precond], ctypes.byref(a), ctypes.byref(b),
                                                        ctypes.byref(c)))
    return a.value, b.value, c.value


def jac_parallel_steps(T: torch.Tensor, V: torch.Tensor | None, r0: int, nsteps: int, skip_abs: float = 0.0):
    """Apply round-robin steps r0.. to copies of T (symmetric) and V; returns (T, V, rotations)."""
    L = load()
    n = T.shape[0]
    Tc = _colmajor(_dev(T))
    Vc = None if V is None else _colmajor(_dev(V))
    rot = ctypes.c_longlong(0)
    code = L.jac_parallel_steps(_vp(Tc.data_ptr()), n, max(n, 1),
                                None if Vc is None else _vp(Vc.data_ptr()), max(n, 1), r0, nsteps,
                                skip_abs, ctypes.byref(rot), _stream())
    _check("jac_parallel_steps", code)
    return Tc.t(), None if Vc is None else Vc.t(), rot.value


def jac_round_robin_pairs(ne: int, r: int):
    L = load()
    p = (ctypes.c_int * (ne // 2))()
    q = (ctypes.c_int * (ne // 2))()
    code = L.jac_round_robin_pairs(ne, r, p, q)
    _check("jac_round_robin_pairs", code)
    return list(p), list(q)


def jac_mgs(Z: torch.Tensor):
    """Modified Gram-Schmidt of the columns of Z (m x n); returns Q."""
    L = load()
    m, n = Z.shape
    Qc = _colmajor(_dev(Z))
    code = L.jac_mgs(_vp(Qc.data_ptr()), m, n, max(m, 1), _stream())
    _check("jac_mgs", code)
    return Qc.t()


def jac_qr_orth(Z: torch.Tensor):
    """Step 2 as the pipeline runs it: returns (Q, method) with method 1 (series) or 2 (block MGS)."""
    L = load()
    n = Z.shape[0]
    Qb = _colmajor(_dev(Z))
    meth = ctypes.c_int(0)
    code = L.jac_qr_orth(_vp(Qb.data_ptr()), n, max(n, 1), ctypes.byref(meth), _stream())
    _check("jac_qr_orth", code)
    return Qb.t(), meth.value


def jac_similarity(A: torch.Tensor, Q: torch.Tensor):
    L = load()
    n = A.shape[0]
    Ac = _colmajor(_dev(A))
    Qc = _colmajor(_dev(Q))
    Tb = torch.empty((n, n), dtype=torch.float64, device=A.device)
    code = L.jac_similarity(_vp(Ac.data_ptr()), n, max(n, 1), _vp(Qc.data_ptr()), max(n, 1),
                            _vp(Tb.data_ptr()), max(n, 1), _stream())
    _check("jac_similarity", code)
    return Tb.t()


def jac_eig_fp32(A: torch.Tensor, tol: float = 0.0, max_sweeps: int = 0):
    """FP32 step 1: returns (W ascending, Z with matching columns, sweeps)."""
    L = load()
    n = A.shape[0]
    Ac = _colmajor(_dev(A))
    W = torch.empty(n, dtype=torch.float64, device=A.device)
    Zb = torch.empty((n, n), dtype=torch.float64, device=A.device)
    sw = ctypes.c_int(0)
    code = L.jac_eig_fp32(_vp(Ac.data_ptr()), n, max(n, 1), _vp(Zb.data_ptr()), max(n, 1),
                          _vp(W.data_ptr()), tol, max_sweeps, ctypes.byref(sw), _stream())
    _check("jac_eig_fp32", code)
    return W, Zb.t(), sw.value


def jac_sytrd_f32(A: torch.Tensor):
    """FP32 Householder tridiagonalization of the symmetric A: returns (d, e, tau, U) with U's
    column k the reflector u_k (device tensors; d, e FP64, tau, U FP32)."""
    L = load()
    A = _dev(A)
    n = A.shape[0]
    Ac = _colmajor(A)
    d = torch.empty(n, dtype=torch.float64, device=A.device)
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=A.device)
    tau = torch.empty(max(n - 2, 1), dtype=torch.float32, device=A.device)
    Ub = torch.zeros((max(n - 2, 1), n), dtype=torch.float32, device=A.device)
    code = L.jac_sytrd_f32(_vp(Ac.data_ptr()), n, max(n, 1), _vp(d.data_ptr()), _vp(e.data_ptr()),
                           _vp(tau.data_ptr()), _vp(Ub.data_ptr()), max(n, 1), _stream())
    _check("jac_sytrd_f32", code)
    torch.cuda.synchronize()
    return d, e[: max(n - 1, 0)], tau[: max(n - 2, 0)], Ub[: max(n - 2, 0)].t()


def jac_tridiag_eig(d: torch.Tensor, e: torch.Tensor, vectors: bool = True):
    """Eigenvalues (ascending) and, with vectors=True, eigenvectors of the tridiagonal (d, e)."""
    L = load()
    d = _dev(d).contiguous()
    n = d.shape[0]
    e = _dev(e).contiguous() if n > 1 else torch.zeros(1, dtype=torch.float64, device=d.device)
    w = torch.empty(n, dtype=torch.float64, device=d.device)
    Zb = torch.empty((n, n), dtype=torch.float64, device=d.device) if vectors else None
    code = L.jac_tridiag_eig(_vp(d.data_ptr()), _vp(e.data_ptr()), n, _vp(w.data_ptr()),
                             _vp(Zb.data_ptr()) if vectors else None, max(n, 1), _stream())
    _check("jac_tridiag_eig", code)
    return (w, Zb.t()) if vectors else w


def jac_tridiag_backtransform(U: torch.Tensor, tau: torch.Tensor, Y: torch.Tensor):
    """H_0 ... H_{n-3} Y for reflectors (U, tau) as from jac_sytrd_f32 (FP32 arithmetic)."""
    L = load()
    n = Y.shape[0]
    Uc = _colmajor(_dev(U, torch.float32)) if n > 2 else torch.zeros(1, dtype=torch.float32, device=Y.device)
    tau = _dev(tau, torch.float32).contiguous() if n > 2 else Uc
    Yb = _colmajor(_dev(Y)).clone()
    code = L.jac_tridiag_backtransform(_vp(Uc.data_ptr()), max(n, 1), _vp(tau.data_ptr()), n,
                                       _vp(Yb.data_ptr()), max(n, 1), _stream())
    _check("jac_tridiag_backtransform", code)
    return Yb.t()


def jac_eig_fp32_tridiag(A: torch.Tensor):
    """The tridiagonal FP32 step 1: returns (W ascending, Z with matching columns)."""
    L = load()
    n = A.shape[0]
    Ac = _colmajor(_dev(A))
    W = torch.empty(n, dtype=torch.float64, device=A.device)
    Zb = torch.empty((n, n), dtype=torch.float64, device=A.device)
    code = L.jac_eig_fp32_tridiag(_vp(Ac.data_ptr()), n, max(n, 1), _vp(Zb.data_ptr()), max(n, 1),
                                  _vp(W.data_ptr()), _stream())
    _check("jac_eig_fp32_tridiag", code)
    return W, Zb.t()


def jac_gemm(A: torch.Tensor, B: torch.Tensor, transa=False, transb=False):
    """op(A) @ op(B) on the matrix cores (float64 or float32)."""
    L = load()
    dt = A.dtype
    Ac = _colmajor(_dev(A, dt))
    Bc = _colmajor(_dev(B, dt))
    m = A.shape[1] if transa else A.shape[0]
    k = A.shape[0] if transa else A.shape[1]
    n = B.shape[0] if transb else B.shape[1]
    Cb = torch.zeros((n, m), dtype=dt, device=A.device)
    fn = L.jac_gemm_f64 if dt == torch.float64 else L.jac_gemm_f32
    code = fn(int(transa), int(transb), m, n, k, 1.0, _vp(Ac.data_ptr()), max(A.shape[0], 1),
              _vp(Bc.data_ptr()), max(B.shape[0], 1), 0.0, _vp(Cb.data_ptr()), max(m, 1), _stream())
    _check("jac_gemm", code)
    return Cb.t()


# ------------------------------------------------------------------ learned warm start
MLP_PARAMS, MLP_GRADS, MLP_MOMENT1, MLP_MOMENT2 = 0, 1, 2, 3


class Mlp:
    """Handle of a jac_mlp network (theta -> n x n eigenvector guess).  Buffers are
    exchanged as numpy float32 arrays (host); theta, targets and outputs as device tensors."""

    def __init__(self, n_in: int, hidden: int, n: int, max_batch: int, seed: int = 0):
        L = load()
        h = _vp()
        _check("jac_mlp_create", L.jac_mlp_create(n_in, hidden, n, max_batch, seed, ctypes.byref(h)))
        self.h = h
        self.n_in, self.hidden, self.n, self.max_batch = n_in, hidden, n, max_batch
        self.P = int(L.jac_mlp_num_params(h))

    def close(self):
        if self.h is not None and self.h.value:
            load().jac_mlp_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self):
        a, b, c, d = _i(), _i(), _i(), _i()
        t = ctypes.c_longlong()
        _check("jac_mlp_shape", load().jac_mlp_shape(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                                      ctypes.byref(d), ctypes.byref(t)))
        return a.value, b.value, c.value, d.value, t.value

    def get(self, which: int = MLP_PARAMS):
        import numpy as np
        out = np.empty(self.P, dtype=np.float32)
        _check("jac_mlp_get", load().jac_mlp_get(self.h, which, out.ctypes.data_as(_vp)))
        return out

    def set(self, values, which: int = MLP_PARAMS):
        import numpy as np
        v = np.ascontiguousarray(values, dtype=np.float32)
        if v.size != self.P:
            raise ValueError(f"expected {self.P} values, got {v.size}")
        _check("jac_mlp_set", load().jac_mlp_set(self.h, which, v.ctypes.data_as(_vp)))

    def set_adam(self, beta1=0.9, beta2=0.999, eps=1e-8, steps=0):
        _check("jac_mlp_set_adam", load().jac_mlp_set_adam(self.h, beta1, beta2, eps, steps))

    def forward(self, theta: torch.Tensor) -> torch.Tensor:
        theta = _dev(theta, torch.float32).contiguous()
        B = theta.shape[0]
        Y = torch.empty((B, self.n * self.n), dtype=torch.float32, device=theta.device)
        _check("jac_mlp_forward", load().jac_mlp_forward(self.h, _vp(theta.data_ptr()), B, _vp(Y.data_ptr()),
                                                          self.n * self.n, _stream()))
        return Y

    def predict(self, theta: torch.Tensor) -> torch.Tensor:
        """Z (n x n FP64) for one theta; columns are the predicted eigenvectors."""
        theta = _dev(theta, torch.float32).contiguous()
        Zc = torch.empty((self.n, self.n), dtype=torch.float64, device=theta.device)
        _check("jac_mlp_predict", load().jac_mlp_predict(self.h, _vp(theta.data_ptr()), _vp(Zc.data_ptr()),
                                                          self.n, _stream()))
        return Zc.t()

    def grads(self, theta: torch.Tensor, target: torch.Tensor, loss: torch.Tensor | None = None):
        theta = _dev(theta, torch.float32).contiguous()
        target = _dev(target, torch.int16)
        _check("jac_mlp_grads", load().jac_mlp_grads(self.h, _vp(theta.data_ptr()), _vp(target.data_ptr()),
                                                      target.stride(0), theta.shape[0],
                                                      None if loss is None else _vp(loss.data_ptr()), _stream()))

    def adamw(self, lr: float, weight_decay: float = 0.0):
        _check("jac_mlp_adamw", load().jac_mlp_adamw(self.h, lr, weight_decay, _stream()))

    def train_step(self, theta: torch.Tensor, target: torch.Tensor, lr: float, weight_decay: float = 0.0,
                   loss: torch.Tensor | None = None):
        """theta: (B, n_in) float32; target: (B, >= n^2) int16 holding bfloat16 bits (row stride
        target.stride(0)); loss: optional device float32 scalar written with the batch loss."""
        _check("jac_mlp_train_step", load().jac_mlp_train_step(
            self.h, _vp(theta.data_ptr()), _vp(target.data_ptr()), target.stride(0), theta.shape[0], lr,
            weight_decay, None if loss is None else _vp(loss.data_ptr()), _stream()))

    def save(self, path: str):
        _check("jac_mlp_save", load().jac_mlp_save(self.h, path.encode()))

    def load_file(self, path: str):
        _check("jac_mlp_load", load().jac_mlp_load(self.h, path.encode()))


def jac_mlp_pack_targets(V: torch.Tensor, out: torch.Tensor | None = None, canonical: bool = True) -> torch.Tensor:
    """bfloat16 training targets of a stack of eigenvector matrices.  V: (count, n, n) FP64,
    V[c][:, j] = eigenvector j.  Returns (count, n*n) int16 bfloat16 bits, row c = column-major
    entries of V[c], with every column's largest-|entry| made positive (canonical) or as given."""
    V = _dev(V)
    count, n, _ = V.shape
    Vc = V.transpose(1, 2).contiguous()          # row-major buffer of V^T = column-major V
    if out is None:
        out = torch.empty((count, n * n), dtype=torch.int16, device=V.device)
    _check("jac_mlp_pack_targets", load().jac_mlp_pack_targets_ex(_vp(Vc.data_ptr()), n, n, n * n, count,
                                                                   _vp(out.data_ptr()), out.stride(0),
                                                                   0 if canonical else 1, _stream()))
    return out
