"""ctypes wrapper of the plain-C FP64 oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It builds ``bilu_oracle.c`` with gcc into
``oracle/_build`` and exposes each oracle step as a numpy function.
Nothing here is shared with the GPU library.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bilu_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libbilu_oracle.so")

OK, NOT_CONVERGED, BREAKDOWN, SINGULAR = 0, 2, 3, 1
SWEEP_L, SWEEP_U, SWEEP_UT, SWEEP_LT = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (plain loops, no SIMD intrinsics)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                           "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ct.CDLL(_LIB)
        P, I, D, LL = ct.c_void_p, ct.c_int, ct.c_double, ct.c_longlong
        L.orc_check_pattern.argtypes = [I, P, P]
        L.orc_symbolic.argtypes = [I, P, P, I, ct.POINTER(ct.c_void_p)]
        L.orc_pattern_nnz.argtypes = [P]
        L.orc_pattern_nnz.restype = LL
        L.orc_pattern_export.argtypes = [P, P, P, P]
        L.orc_pattern_free.argtypes = [P]
        L.orc_levels.argtypes = [I, P, P, I, P]
        L.orc_level_sets.argtypes = [I, P, I, P, P]
        L.orc_factor.argtypes = [I, I, P, P, P, P, P, P, P, ct.POINTER(I)]
        L.orc_split.argtypes = [I, I, P, P, P, P, P]
        for f in (L.orc_apply, L.orc_apply_t):
            f.argtypes = [I, I, P, P, P, P, P, P]
        L.orc_apply_f32.argtypes = [I, I, P, P, P, P, P, P]
        L.orc_round_f32.argtypes = [LL, P, P]
        for f in (L.orc_spmv, L.orc_spmv_t):
            f.argtypes = [I, I, P, P, P, P, P]
        L.orc_solve.argtypes = [I, I, P, P, P, P, P, P, P, P, P, P, P,
                                I, I, D, I, I, ct.POINTER(I), ct.POINTER(D)]
        L.orc_grad_A.argtypes = [I, I, P, P, P, P, P]
        L.orc_last_restarts.restype = I
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, code, row=-1):
        super().__init__(f"oracle status {code} (row {row})")
        self.code = code
        self.row = row


def check_pattern(nb, Ap, Aj):
    Ap, Aj = _i32(Ap), _i32(Aj)
    return lib().orc_check_pattern(nb, _p(Ap), _p(Aj))


def symbolic(nb, Ap, Aj, k):
    """Algorithm 3 on the point-wise view of the block pattern.

    Returns (Pp, Pj, lev): the kept pattern and the level of fill of each
    kept entry."""
    Ap, Aj = _i32(Ap), _i32(Aj)
    h = ct.c_void_p()
    st = lib().orc_symbolic(nb, _p(Ap), _p(Aj), int(k), ct.byref(h))
    if st != 0:
        raise OracleError(st)
    nnz = lib().orc_pattern_nnz(h)
    Pp = np.zeros(nb + 1, np.int32)
    Pj = np.zeros(nnz, np.int32)
    lev = np.zeros(nnz, np.int32)
    lib().orc_pattern_export(h, _p(Pp), _p(Pj), _p(lev))
    lib().orc_pattern_free(h)
    return Pp, Pj, lev


def levels(nb, Pp, Pj, which):
    """0-based level of each row for sweep ``which`` (Eq 4); returns (lvl, nlev)."""
    Pp, Pj = _i32(Pp), _i32(Pj)
    lvl = np.zeros(nb, np.int32)
    nlev = lib().orc_levels(nb, _p(Pp), _p(Pj), int(which), _p(lvl))
    return lvl, nlev


def level_sets(lvl, nlev):
    lvl = _i32(lvl)
    ptr = np.zeros(nlev + 1, np.int32)
    rows = np.zeros(lvl.shape[0], np.int32)
    lib().orc_level_sets(lvl.shape[0], _p(lvl), nlev, _p(ptr), _p(rows))
    return ptr, rows


def factor(nb, bs, Ap, Aj, Ax, Pp, Pj):
    """Backfill A into P and run block ILU(0) (Algorithms 4-5).

    Returns (LU, Dinv); raises OracleError(SINGULAR, row) on a singular pivot."""
    Ap, Aj, Pp, Pj = _i32(Ap), _i32(Aj), _i32(Pp), _i32(Pj)
    Ax = _f64(Ax)
    bb = bs * bs
    LU = np.zeros(int(Pp[-1]) * bb)
    Dinv = np.zeros(nb * bb)
    bad = ct.c_int(-1)
    st = lib().orc_factor(nb, bs, _p(Ap), _p(Aj), _p(Ax), _p(Pp), _p(Pj), _p(LU),
                          _p(Dinv), ct.byref(bad))
    if st != 0:
        raise OracleError(st, bad.value)
    return LU, Dinv


def split(nb, bs, Pp, Pj, LU, Dinv):
    """U = D U' (Eq 5): F holds L below, U' above and I on the diagonal."""
    Pp, Pj = _i32(Pp), _i32(Pj)
    F = np.zeros(int(Pp[-1]) * bs * bs)
    lib().orc_split(nb, bs, _p(Pp), _p(Pj), _p(_f64(LU)), _p(_f64(Dinv)), _p(F))
    return F


def round_f32(a):
    a = _f64(a)
    out = np.zeros(a.shape[0], np.float32)
    lib().orc_round_f32(a.shape[0], _p(a), _p(out))
    return out


def apply(nb, bs, Pp, Pj, F, Dinv, r, transpose=False):
    Pp, Pj = _i32(Pp), _i32(Pj)
    r = _f64(r)
    z = np.zeros_like(r)
    if F.dtype == np.float32:
        assert not transpose
        lib().orc_apply_f32(nb, bs, _p(Pp), _p(Pj), _p(np.ascontiguousarray(F)),
                            _p(np.ascontiguousarray(Dinv, dtype=np.float32)), _p(r), _p(z))
        return z
    f = lib().orc_apply_t if transpose else lib().orc_apply
    f(nb, bs, _p(Pp), _p(Pj), _p(_f64(F)), _p(_f64(Dinv)), _p(r), _p(z))
    return z


def spmv(nb, bs, Ap, Aj, Ax, x, transpose=False):
    Ap, Aj = _i32(Ap), _i32(Aj)
    x = _f64(x)
    y = np.zeros_like(x)
    f = lib().orc_spmv_t if transpose else lib().orc_spmv
    f(nb, bs, _p(Ap), _p(Aj), _p(_f64(Ax)), _p(x), _p(y))
    return y


def solve(nb, bs, Ap, Aj, Ax, Pp, Pj, F, Dinv, b, method=0, restart=30, rtol=1e-8,
          maxit=2000, transpose=False, F32=None, Dinv32=None):
    """BiCGSTAB (method 0), GMRES(restart) (method 1) or ORTHOMIN(k = restart)
    (method 2), right-preconditioned.

    Returns (x, iters, relres, status)."""
    Ap, Aj, Pp, Pj = _i32(Ap), _i32(Aj), _i32(Pp), _i32(Pj)
    b = _f64(b)
    x = np.zeros_like(b)
    it = ct.c_int(0)
    rr = ct.c_double(0.0)
    F32 = None if F32 is None else np.ascontiguousarray(F32, np.float32)
    Dinv32 = None if Dinv32 is None else np.ascontiguousarray(Dinv32, np.float32)
    st = lib().orc_solve(nb, bs, _p(Ap), _p(Aj), _p(_f64(Ax)), _p(Pp), _p(Pj),
                         _p(_f64(F)) if F is not None else None,
                         _p(_f64(Dinv)) if Dinv is not None else None,
                         _p(F32), _p(Dinv32), _p(b), _p(x), int(method), int(restart),
                         float(rtol), int(maxit), int(bool(transpose)),
                         ct.byref(it), ct.byref(rr))
    return x, it.value, rr.value, st


def last_restarts():
    """True-residual restarts taken by the last BiCGSTAB solve (a counter)."""
    return int(lib().orc_last_restarts())


def grad_A(nb, bs, Ap, Aj, lam, x):
    """dL/dA_ij = -lambda_i x_j^T on A's block pattern."""
    Ap, Aj = _i32(Ap), _i32(Aj)
    out = np.zeros(int(Ap[-1]) * bs * bs)
    lib().orc_grad_A(nb, bs, _p(Ap), _p(Aj), _p(_f64(lam)), _p(_f64(x)), _p(out))
    return out


class OracleILU:
    """The whole oracle pipeline for one block system: symbolic phase and
    level sets at construction, numeric factorisation and split on demand."""

    def __init__(self, nb, bs, Ap, Aj, k):
        self.nb, self.bs, self.k = nb, bs, k
        self.Ap, self.Aj = _i32(Ap), _i32(Aj)
        self.Pp, self.Pj, self.lev = symbolic(nb, Ap, Aj, k)
        self.F = self.Dinv = self.LU = None

    def level_sets(self, which):
        lvl, nlev = levels(self.nb, self.Pp, self.Pj, which)
        return level_sets(lvl, nlev)

    def factor(self, Ax):
        self.LU, self.Dinv = factor(self.nb, self.bs, self.Ap, self.Aj, Ax, self.Pp, self.Pj)
        self.F = split(self.nb, self.bs, self.Pp, self.Pj, self.LU, self.Dinv)
        return self

    def apply(self, r, transpose=False):
        return apply(self.nb, self.bs, self.Pp, self.Pj, self.F, self.Dinv, r, transpose)

    def solve(self, Ax, b, **kw):
        return solve(self.nb, self.bs, self.Ap, self.Aj, Ax, self.Pp, self.Pj, self.F,
                     self.Dinv, b, **kw)
