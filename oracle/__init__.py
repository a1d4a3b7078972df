"""CPU oracle for the mixed-precision preconditioned Jacobi eigensolver.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or executes anything here, and nothing here imports the product.

The arithmetic lives in plain C (``oracle.c``: the Jacobi methods, MGS, GEMM,
one-sided SVD; ``tridiag.c``: Householder tridiagonalization, Sturm bisection,
inverse iteration and the back-transformation, the parts of the tridiagonal
eigensolver the paper takes for step 1), FP64, single-threaded; this module
compiles it with gcc on first use and wraps it with ctypes and numpy.  See the
two C files for the paper passage each routine follows.  ``mlp.py``
holds the FP64 reference of the learned warm-start network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "tridiag.c"), os.path.join(_HERE, "jacobi_body.h")]

U64 = 2.0 ** -53
U32 = 2.0 ** -24
DEFAULT_TOL = 20.0 * U64  # epsilon = 20 omega, Section 6 setup


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, no fast-math, no FMA contraction)."""
    fresh = os.path.exists(_SO) and all(
        os.path.getmtime(_SO) >= os.path.getmtime(s) for s in _SRC)
    if force or not fresh:
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, _SRC[0], _SRC[1], "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int)
        llp = ctypes.POINTER(ctypes.c_longlong)
        c_int, c_d = ctypes.c_int, ctypes.c_double
        L.or_syev.argtypes = [c_int, dp, c_int, c_d, c_int, c_int, dp, dp, c_int, ip, llp, dp, c_int]
        L.or_syev.restype = c_int
        L.or_syev_f32.argtypes = [c_int, fp, c_int, c_d, c_int, c_int, fp, fp, c_int, ip, llp]
        L.or_syev_f32.restype = c_int
        L.or_jacobi_from.argtypes = [c_int, dp, c_int, dp, c_int, c_int, c_d, c_d, c_int, c_int,
                                     ip, llp, dp, c_int]
        L.or_jacobi_from.restype = c_int
        L.or_round_robin.argtypes = [c_int, c_int, ip, ip]
        L.or_round_robin.restype = None
        L.or_parallel_step.argtypes = [c_int, dp, c_int, dp, c_int, c_int, c_int, ip, ip, c_d]
        L.or_parallel_step.restype = ctypes.c_longlong
        L.or_angle.argtypes = [c_d, c_d, c_d, dp, dp, dp]
        L.or_angle.restype = None
        L.or_fro.argtypes = [c_int, c_int, dp, c_int]
        L.or_fro.restype = c_d
        L.or_off.argtypes = [c_int, dp, c_int]
        L.or_off.restype = c_d
        L.or_mgs.argtypes = [c_int, c_int, dp, c_int, dp, c_int, dp, c_int]
        L.or_mgs.restype = c_int
        L.or_gemm.argtypes = [c_int, c_int, c_int, c_int, c_int, dp, c_int, dp, c_int, dp, c_int]
        L.or_gemm.restype = None
        L.or_svd_onesided.argtypes = [c_int, c_int, dp, c_int, dp, c_int, c_d, c_d, c_int, c_int,
                                      ip, llp]
        L.or_svd_onesided.restype = c_int
        L.or_svd_finish.argtypes = [c_int, c_int, dp, c_int, dp, c_int, dp, dp, c_int, dp, c_int]
        L.or_svd_finish.restype = None
        L.or_sytrd.argtypes = [c_int, dp, c_int, dp, dp, dp, dp, c_int]
        L.or_sytrd.restype = c_int
        L.or_sturm_count.argtypes = [c_int, dp, dp, c_d]
        L.or_sturm_count.restype = c_int
        L.or_tridiag_eigvals.argtypes = [c_int, dp, dp, dp]
        L.or_tridiag_eigvals.restype = None
        L.or_tridiag_vector.argtypes = [c_int, dp, dp, c_d, dp]
        L.or_tridiag_vector.restype = c_int
        L.or_apply_reflectors.argtypes = [c_int, dp, c_int, dp, dp, c_int, c_int]
        L.or_apply_reflectors.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _colmajor(a, dtype=np.float64):
    return np.asfortranarray(np.asarray(a, dtype=dtype))


class Result:
    """Outcome of an oracle solve: W ascending, V (columns = eigenvectors)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def syev(A, tol: float = DEFAULT_TOL, max_sweeps: int = 64, order: str = "row",
         hist_len: int = 64) -> Result:
    """Algorithm 3.2 in FP64 from T = A, P = I (order 'row' or 'rr')."""
    A = _colmajor(A)
    n = A.shape[0]
    W = np.zeros(n)
    V = np.zeros((n, n), order="F")
    sw = ctypes.c_int(0)
    rot = ctypes.c_longlong(0)
    hist = np.zeros(hist_len)
    info = lib().or_syev(n, _dp(A), max(n, 1), tol, max_sweeps, 0 if order == "row" else 1,
                         _dp(W), _dp(V), max(n, 1), ctypes.byref(sw), ctypes.byref(rot),
                         _dp(hist), hist_len)
    return Result(W=W, V=V, info=info, sweeps=sw.value, rotations=rot.value,
                  off_hist=hist[: sw.value + 1].copy())


def syev_f32(A, tol: float = 1e-6, max_sweeps: int = 64, order: str = "row") -> Result:
    """The same cyclic Jacobi carried out in FP32 (reference for step 1)."""
    A = _colmajor(A, np.float32)
    n = A.shape[0]
    W = np.zeros(n, np.float32)
    V = np.zeros((n, n), np.float32, order="F")
    sw = ctypes.c_int(0)
    rot = ctypes.c_longlong(0)
    info = lib().or_syev_f32(n, _fp(A), max(n, 1), tol, max_sweeps, 0 if order == "row" else 1,
                             _fp(W), _fp(V), max(n, 1), ctypes.byref(sw), ctypes.byref(rot))
    return Result(W=W, V=V, info=info, sweeps=sw.value, rotations=rot.value)


def jacobi_from(T, P, tol: float, nrmA: float, max_sweeps: int = 64, order: str = "rr",
                hist_len: int = 64) -> Result:
    """Step 4 of Algorithm 4.1: sweeps from the given T, P (copies are updated)."""
    T = _colmajor(T).copy(order="F")
    P = _colmajor(P).copy(order="F")
    n = T.shape[0]
    sw = ctypes.c_int(0)
    rot = ctypes.c_longlong(0)
    hist = np.zeros(hist_len)
    info = lib().or_jacobi_from(n, _dp(T), max(n, 1), _dp(P), max(P.shape[0], 1), P.shape[0],
                                tol, nrmA, max_sweeps, 0 if order == "row" else 1,
                                ctypes.byref(sw), ctypes.byref(rot), _dp(hist), hist_len)
    return Result(T=T, P=P, info=info, sweeps=sw.value, rotations=rot.value,
                  off_hist=hist[: sw.value + 1].copy())


def round_robin(n_even: int, r: int):
    p = np.zeros(n_even // 2, np.int32)
    q = np.zeros(n_even // 2, np.int32)
    lib().or_round_robin(n_even, r, _ip(p), _ip(q))
    return p, q


def parallel_step(T, P, p, q, skip_abs: float):
    """Apply one step of disjoint rotations (angles from T before the step)."""
    T = _colmajor(T).copy(order="F")
    P = None if P is None else _colmajor(P).copy(order="F")
    n = T.shape[0]
    p = np.ascontiguousarray(p, np.int32)
    q = np.ascontiguousarray(q, np.int32)
    np_rows = 0 if P is None else P.shape[0]
    applied = lib().or_parallel_step(
        n, _dp(T), max(n, 1), None if P is None else _dp(P), max(np_rows, 1), np_rows,
        len(p), _ip(p), _ip(q), skip_abs)
    return T, P, applied


def angle(aii: float, ajj: float, aij: float):
    c, s, t = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().or_angle(aii, ajj, aij, ctypes.byref(c), ctypes.byref(s), ctypes.byref(t))
    return c.value, s.value, t.value


def fro(A) -> float:
    A = _colmajor(A)
    return lib().or_fro(A.shape[0], A.shape[1], _dp(A), max(A.shape[0], 1))


def off(T) -> float:
    T = _colmajor(T)
    return lib().or_off(T.shape[0], _dp(T), max(T.shape[0], 1))


def mgs(Z):
    """Modified Gram-Schmidt: returns (Q, R, info)."""
    Z = _colmajor(Z)
    m, n = Z.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    info = lib().or_mgs(m, n, _dp(Z), max(m, 1), _dp(Q), max(m, 1), _dp(R), max(n, 1))
    return Q, R, info


def gemm(A, B, ta: bool = False, tb: bool = False):
    A = _colmajor(A)
    B = _colmajor(B)
    m = A.shape[1] if ta else A.shape[0]
    k = A.shape[0] if ta else A.shape[1]
    n = B.shape[0] if tb else B.shape[1]
    C = np.zeros((m, n), order="F")
    lib().or_gemm(int(ta), int(tb), m, n, k, _dp(A), max(A.shape[0], 1), _dp(B),
                  max(B.shape[0], 1), _dp(C), max(m, 1))
    return C


def similarity(A, Q):
    """T = Q^T (A Q), step 3 of Algorithm 4.1."""
    return gemm(Q, gemm(A, Q), ta=True)


def svd_onesided(C, V, tol: float = U64, ratio_stop: float = 2e-4, max_sweeps: int = 64,
                 order: str = "row") -> Result:
    C = _colmajor(C).copy(order="F")
    V = _colmajor(V).copy(order="F")
    m, n = C.shape
    sw = ctypes.c_int(0)
    rot = ctypes.c_longlong(0)
    info = lib().or_svd_onesided(m, n, _dp(C), max(m, 1), _dp(V), max(n, 1), tol, ratio_stop,
                                 max_sweeps, 0 if order == "row" else 1, ctypes.byref(sw),
                                 ctypes.byref(rot))
    return Result(C=C, V=V, info=info, sweeps=sw.value, rotations=rot.value)


def svd_finish(C, Vin):
    C = _colmajor(C)
    Vin = _colmajor(Vin)
    m, n = C.shape
    S = np.zeros(n)
    U = np.zeros((m, n), order="F")
    V = np.zeros((n, n), order="F")
    lib().or_svd_finish(m, n, _dp(C), max(m, 1), _dp(Vin), max(n, 1), _dp(S), _dp(U), max(m, 1),
                        _dp(V), max(n, 1))
    return S, U, V


def gesvd(A, tol: float = U64, ratio_stop: float = 2e-4, max_sweeps: int = 64,
          order: str = "row") -> Result:
    """Algorithm 5.1 (plain one-sided Jacobi SVD) end to end."""
    A = _colmajor(A)
    m, n = A.shape
    r = svd_onesided(A, np.eye(n), tol, ratio_stop, max_sweeps, order)
    S, U, V = svd_finish(r.C, r.V)
    return Result(S=S, U=U, V=V, info=r.info, sweeps=r.sweeps, rotations=r.rotations)


# ---------------------------------------------------------------- tridiagonal route (tridiag.c)
def sytrd(A):
    """Householder tridiagonalization A = Q T Q^T: returns (d, e, tau, U) with U's column k the
    reflector vector u_k (u_k(k+1) = 1, zero above) and Q = H_0 ... H_{n-3}."""
    A = _colmajor(A)
    n = A.shape[0]
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 0) + 1)
    tau = np.zeros(max(n, 1))
    U = np.zeros((n, n), order="F")
    if n:
        lib().or_sytrd(n, _dp(A), max(n, 1), _dp(d), _dp(e), _dp(tau), _dp(U), max(n, 1))
    return d, e[: max(n - 1, 0)], tau[: max(n - 2, 0)], U


def _de(d, e):
    d = np.ascontiguousarray(d, np.float64)
    e = np.ascontiguousarray(np.append(np.asarray(e, np.float64), 0.0))
    return d, e


def sturm_count(d, e, x: float) -> int:
    d, e = _de(d, e)
    return lib().or_sturm_count(d.size, _dp(d), _dp(e), x)


def tridiag_eigvals(d, e):
    """All eigenvalues of the symmetric tridiagonal (d, e), ascending, by bisection."""
    d, e = _de(d, e)
    w = np.zeros(d.size)
    lib().or_tridiag_eigvals(d.size, _dp(d), _dp(e), _dp(w))
    return w


def tridiag_vectors(d, e, w):
    """Eigenvectors (columns) of (d, e) for the eigenvalues w, by inverse iteration."""
    d, e = _de(d, e)
    n = d.size
    Z = np.zeros((n, len(w)), order="F")
    z = np.zeros(n)
    for k, lam in enumerate(w):
        lib().or_tridiag_vector(n, _dp(d), _dp(e), float(lam), _dp(z))
        Z[:, k] = z
    return Z


def apply_reflectors(U, tau, Y):
    """Z = H_0 H_1 ... H_{n-3} Y (reflectors from sytrd)."""
    U = _colmajor(U)
    Z = _colmajor(Y).copy(order="F")
    n, ncol = Z.shape
    t = np.zeros(max(n, 1))
    t[: len(tau)] = tau
    lib().or_apply_reflectors(n, _dp(U), max(n, 1), _dp(t), _dp(Z), max(n, 1), ncol)
    return Z


def syev_tridiag(A):
    """Eigendecomposition through the three parts: tridiagonalization, bisection and inverse
    iteration on T, back-transformation.  Returns (W ascending, Z)."""
    d, e, tau, U = sytrd(A)
    w = tridiag_eigvals(d, e)
    return w, apply_reflectors(U, tau, tridiag_vectors(d, e, w))
