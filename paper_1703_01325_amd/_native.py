"""ctypes binding of libbilu.so (argument marshalling only).

Every function here has the name of the C entry point it calls and does
nothing but convert arguments: numpy arrays for host structure, raw device
pointers (ints) and HIP stream handles (ints) for device data.  All
computation happens in the library.  Importing fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libbilu.so")

OK = 0
ERR_ARG, ERR_ALLOC, ERR_HIP, ERR_MISSING_DIAG, ERR_PATTERN, ERR_TIMEOUT, ERR_STATE = -1, -2, -3, -4, -5, -6, -7
SINGULAR_PIVOT, NOT_CONVERGED, BREAKDOWN, NONFINITE = 1, 2, 3, 4
SWEEP_L, SWEEP_U, SWEEP_UT, SWEEP_LT = 0, 1, 2, 3
FACTORS_FP64, FACTORS_FP32 = 0, 1
BICGSTAB, GMRES, ORTHOMIN = 0, 1, 2
WANT_TRANSPOSE = 1
DEVICE_SYMBOLIC = 2

# every symbol declared in include/bilu.h
EXPORTS = (
    "bilu_analyze", "bilu_get_pattern", "bilu_get_levels", "bilu_get_info", "bilu_validate",
    "bilu_symbolic_device", "bilu_levels_device",
    "bilu_factor_numeric", "bilu_factor_diag", "bilu_get_factors", "bilu_get_factors_f32",
    "bilu_apply", "bilu_apply_noalloc", "bilu_apply_point", "bilu_apply_transpose", "bilu_spmv", "bilu_solve", "bilu_grad_A",
    "bilu_tune", "bilu_autotune", "bilu_check", "bilu_timing", "bilu_timing_read",
    "bilu_destroy", "bilu_status_string",
    "bilu_batch_create", "bilu_batch_offsets", "bilu_batch_factor", "bilu_batch_apply",
    "bilu_batch_spmv", "bilu_batch_solve", "bilu_batch_autotune", "bilu_batch_member", "bilu_batch_destroy",
)
K_SWEEP_L, K_SWEEP_U, K_SWEEP_UT, K_SWEEP_LT, K_SPMV, K_FACTOR, K_SPLIT, K_SWEEP_U_SPMV, K_COUNT = range(9)
K_NAMES = ("sweep_L", "sweep_U", "sweep_UT", "sweep_LT", "spmv", "factor", "split", "sweep_U_spmv")


class BiluInfo(ct.Structure):
    _fields_ = [("nb", ct.c_int), ("bs", ct.c_int), ("k", ct.c_int),
                ("nnzb_A", ct.c_int64), ("nnzb_P", ct.c_int64), ("nnzb_L", ct.c_int64),
                ("nnzb_U", ct.c_int64), ("nlev", ct.c_int * 4), ("rows_per_chunk", ct.c_int),
                ("sweep_slots", ct.c_int64 * 4), ("tile_rows", ct.c_int),
                ("tile_group", ct.c_int), ("lds_ring", ct.c_int * 4), ("tile_block", ct.c_int * 4),
                ("line_sweep", ct.c_int * 2)]


class KernelTime(ct.Structure):
    _fields_ = [("launches", ct.c_int64), ("total_ms", ct.c_double)]


class SolveOpts(ct.Structure):
    _fields_ = [("method", ct.c_int), ("restart", ct.c_int), ("rtol", ct.c_double),
                ("maxit", ct.c_int)]


class RhsInfo(ct.Structure):
    _fields_ = [("status", ct.c_int), ("iters", ct.c_int), ("relres", ct.c_double),
                ("restarts", ct.c_int), ("reserved", ct.c_int)]


class TuneResult(ct.Structure):
    _fields_ = [("sweep_mode", ct.c_int), ("tile_rows", ct.c_int), ("rhs_tile", ct.c_int),
                ("candidates", ct.c_int), ("apply_us", ct.c_double), ("default_us", ct.c_double),
                ("tile_group", ct.c_int)]


class BatchTuneInfo(ct.Structure):
    _fields_ = [("tile_scale", ct.c_double), ("pair_us", ct.c_double), ("default_us", ct.c_double),
                ("candidates", ct.c_int), ("reserved", ct.c_int)]


class SysDesc(ct.Structure):
    _fields_ = [("nb", ct.c_int), ("bs", ct.c_int), ("Ap", ct.c_void_p), ("Aj", ct.c_void_p)]


class BiluError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} ({code})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950) first")
    L = ct.CDLL(LIB_PATH)
    P, I, VP = ct.c_void_p, ct.c_int, ct.c_void_p
    L.bilu_analyze.argtypes = [I, I, P, P, I, I, ct.POINTER(VP)]
    L.bilu_get_pattern.argtypes = [VP, ct.POINTER(ct.c_int64), ct.POINTER(P), ct.POINTER(P), ct.POINTER(P)]
    L.bilu_get_levels.argtypes = [VP, I, ct.POINTER(I), ct.POINTER(P), ct.POINTER(P)]
    L.bilu_get_info.argtypes = [VP, ct.POINTER(BiluInfo)]
    L.bilu_validate.argtypes = [VP]
    L.bilu_symbolic_device.argtypes = [I, P, P, I, P, P, P, ct.c_int64, ct.POINTER(ct.c_int64), P]
    L.bilu_levels_device.argtypes = [I, P, P, I, P, P, P, ct.POINTER(I), P]
    L.bilu_factor_numeric.argtypes = [VP, P, P, ct.POINTER(I)]
    L.bilu_factor_diag.argtypes = [VP, I, P]
    L.bilu_get_factors.argtypes = [VP, P, P, P]
    L.bilu_get_factors_f32.argtypes = [VP, P, P, P]
    L.bilu_apply.argtypes = [VP, P, P, I, P]
    L.bilu_apply_transpose.argtypes = [VP, P, P, I, P]
    L.bilu_apply_noalloc.argtypes = [VP, P, P, I, P]
    L.bilu_apply_point.argtypes = [VP, P, P, P]
    L.bilu_spmv.argtypes = [VP, P, P, P, I, I, P]
    L.bilu_solve.argtypes = [VP, P, P, P, I, ct.POINTER(SolveOpts), ct.POINTER(RhsInfo), I, P]
    L.bilu_grad_A.argtypes = [VP, P, P, P, P]
    L.bilu_tune.argtypes = [VP, I, I]
    L.bilu_autotune.argtypes = [VP, I, P, ct.POINTER(TuneResult)]
    L.bilu_check.argtypes = [VP, P]
    L.bilu_timing.argtypes = [VP, I]
    L.bilu_timing_read.argtypes = [VP, P, ct.POINTER(KernelTime)]
    L.bilu_destroy.argtypes = [VP]
    L.bilu_destroy.restype = None
    L.bilu_status_string.argtypes = [I]
    L.bilu_status_string.restype = ct.c_char_p
    L.bilu_batch_create.argtypes = [I, ct.POINTER(SysDesc), I, ct.POINTER(VP), ct.POINTER(I)]
    L.bilu_batch_offsets.argtypes = [VP, ct.POINTER(P), ct.POINTER(ct.c_int64)]
    L.bilu_batch_factor.argtypes = [VP, ct.POINTER(P), I, P, ct.POINTER(I), ct.POINTER(I)]
    L.bilu_batch_apply.argtypes = [VP, P, P, P]
    L.bilu_batch_spmv.argtypes = [VP, P, P, P]
    L.bilu_batch_solve.argtypes = [VP, P, P, ct.POINTER(SolveOpts), ct.POINTER(RhsInfo), P]
    L.bilu_batch_autotune.argtypes = [VP, P, ct.POINTER(BatchTuneInfo)]
    L.bilu_batch_member.argtypes = [VP, I, ct.POINTER(VP)]
    L.bilu_batch_destroy.argtypes = [VP]
    L.bilu_batch_destroy.restype = None
    for name in EXPORTS:
        if name not in ("bilu_destroy", "bilu_status_string", "bilu_batch_destroy"):
            getattr(L, name).restype = I
    return L


lib = _load()


def status_string(code: int) -> str:
    return lib.bilu_status_string(int(code)).decode()


def _check(code, where, allow_positive=False):
    if code < 0 or (code > 0 and not allow_positive):
        raise BiluError(code, where)
    return code


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def bilu_analyze(nb, bs, Ap, Aj, k, flags=0):
    Ap, Aj = _i32(Ap), _i32(Aj)
    h = ct.c_void_p()
    _check(lib.bilu_analyze(int(nb), int(bs), _ptr(Ap), _ptr(Aj), int(k), int(flags), ct.byref(h)),
           "bilu_analyze")
    return h


def bilu_get_pattern(ctx):
    n = ct.c_int64()
    Pp, Pj, lev = ct.c_void_p(), ct.c_void_p(), ct.c_void_p()
    _check(lib.bilu_get_pattern(ctx, ct.byref(n), ct.byref(Pp), ct.byref(Pj), ct.byref(lev)),
           "bilu_get_pattern")
    info = bilu_get_info(ctx)
    nb = info.nb

    def view(p, count):
        if count == 0:
            return np.zeros(0, np.int32)
        return np.ctypeslib.as_array(ct.cast(p, ct.POINTER(ct.c_int32)), shape=(count,)).copy()

    return view(Pp, nb + 1), view(Pj, n.value), view(lev, n.value)


def bilu_get_levels(ctx, sweep):
    nlev = ct.c_int()
    ptr, rows = ct.c_void_p(), ct.c_void_p()
    _check(lib.bilu_get_levels(ctx, int(sweep), ct.byref(nlev), ct.byref(ptr), ct.byref(rows)),
           "bilu_get_levels")
    nb = bilu_get_info(ctx).nb
    lp = np.ctypeslib.as_array(ct.cast(ptr, ct.POINTER(ct.c_int32)), shape=(nlev.value + 1,)).copy()
    lr = np.ctypeslib.as_array(ct.cast(rows, ct.POINTER(ct.c_int32)), shape=(nb,)).copy()
    return lp, lr


def bilu_symbolic_device(nb, Ap_ptr, Aj_ptr, k, Pp_ptr, Pj_ptr, lev_ptr, cap, stream):
    """Device pointers in; returns the entry count of P (Pj_ptr = lev_ptr =
    None with cap 0: size query, only Pp is written)."""
    n = ct.c_int64()
    _check(lib.bilu_symbolic_device(int(nb), Ap_ptr, Aj_ptr, int(k), Pp_ptr, Pj_ptr, lev_ptr, int(cap),
                                    ct.byref(n), stream), "bilu_symbolic_device")
    return n.value


def bilu_levels_device(nb, Pp_ptr, Pj_ptr, sweep, lvl_ptr, level_ptr_ptr, level_rows_ptr, stream):
    """Device pointers in; returns the level count."""
    nlev = ct.c_int()
    _check(lib.bilu_levels_device(int(nb), Pp_ptr, Pj_ptr, int(sweep), lvl_ptr, level_ptr_ptr, level_rows_ptr,
                                  ct.byref(nlev), stream), "bilu_levels_device")
    return nlev.value


def bilu_get_info(ctx):
    info = BiluInfo()
    _check(lib.bilu_get_info(ctx, ct.byref(info)), "bilu_get_info")
    return info


def bilu_validate(ctx):
    _check(lib.bilu_validate(ctx), "bilu_validate")


def bilu_factor_numeric(ctx, Ax_ptr, stream):
    bad = ct.c_int(-1)
    st = _check(lib.bilu_factor_numeric(ctx, ct.c_void_p(Ax_ptr), ct.c_void_p(stream), ct.byref(bad)),
                "bilu_factor_numeric", allow_positive=True)
    return st, bad.value


def bilu_factor_diag(ctx, precision, stream):
    _check(lib.bilu_factor_diag(ctx, int(precision), ct.c_void_p(stream)), "bilu_factor_diag")


def bilu_get_factors(ctx, F_ptr, Dinv_ptr, stream):
    _check(lib.bilu_get_factors(ctx, ct.c_void_p(F_ptr), ct.c_void_p(Dinv_ptr), ct.c_void_p(stream)),
           "bilu_get_factors")


def bilu_get_factors_f32(ctx, F_ptr, Dinv_ptr, stream):
    _check(lib.bilu_get_factors_f32(ctx, ct.c_void_p(F_ptr), ct.c_void_p(Dinv_ptr), ct.c_void_p(stream)),
           "bilu_get_factors_f32")


def bilu_apply(ctx, r_ptr, z_ptr, nrhs, stream):
    _check(lib.bilu_apply(ctx, ct.c_void_p(r_ptr), ct.c_void_p(z_ptr), int(nrhs), ct.c_void_p(stream)),
           "bilu_apply")


def bilu_apply_point(ctx, r_ptr, z_ptr, stream):
    _check(lib.bilu_apply_point(ctx, ct.c_void_p(r_ptr), ct.c_void_p(z_ptr), ct.c_void_p(stream)),
           "bilu_apply_point")


def bilu_apply_noalloc(ctx, r_ptr, z_ptr, nrhs, stream):
    _check(lib.bilu_apply_noalloc(ctx, ct.c_void_p(r_ptr), ct.c_void_p(z_ptr), int(nrhs), ct.c_void_p(stream)),
           "bilu_apply_noalloc")


def bilu_apply_transpose(ctx, r_ptr, z_ptr, nrhs, stream):
    _check(lib.bilu_apply_transpose(ctx, ct.c_void_p(r_ptr), ct.c_void_p(z_ptr), int(nrhs),
                                    ct.c_void_p(stream)), "bilu_apply_transpose")


def bilu_spmv(ctx, Ax_ptr, x_ptr, y_ptr, nrhs, transpose, stream):
    _check(lib.bilu_spmv(ctx, ct.c_void_p(Ax_ptr), ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), int(nrhs),
                         int(transpose), ct.c_void_p(stream)), "bilu_spmv")


def bilu_solve(ctx, Ax_ptr, b_ptr, x_ptr, nrhs, method, restart, rtol, maxit, transpose, stream):
    opts = SolveOpts(int(method), int(restart), float(rtol), int(maxit))
    info = (RhsInfo * int(nrhs))()
    st = _check(lib.bilu_solve(ctx, ct.c_void_p(Ax_ptr), ct.c_void_p(b_ptr), ct.c_void_p(x_ptr), int(nrhs),
                               ct.byref(opts), info, int(transpose), ct.c_void_p(stream)),
                "bilu_solve", allow_positive=True)
    return st, [(i.status, i.iters, i.relres, i.restarts) for i in info]


def bilu_grad_A(ctx, lam_ptr, x_ptr, dA_ptr, stream):
    _check(lib.bilu_grad_A(ctx, ct.c_void_p(lam_ptr), ct.c_void_p(x_ptr), ct.c_void_p(dA_ptr),
                           ct.c_void_p(stream)), "bilu_grad_A")


TUNE_SWEEP_MODE, TUNE_TILE_ROWS, TUNE_BLOCKS, TUNE_RHS_TILE, TUNE_FUSE_SPMV, TUNE_TILE_GROUP = 0, 1, 3, 4, 5, 6
TUNE_TILE_BLOCK = 7
TUNE_LINE_SWEEP = 8
TUNE_HELPER = 9
TUNE_SPMV_STREAM = 10
TUNE_RHS_PAIRS = 11
TUNE_SPLIT_DINV = 12
TUNE_FACTOR = 13
TUNE_SPIN_LIMIT = 14


def bilu_tune(ctx, param, value):
    _check(lib.bilu_tune(ctx, int(param), int(value)), "bilu_tune")


def bilu_autotune(ctx, nrhs, stream):
    out = TuneResult()
    _check(lib.bilu_autotune(ctx, int(nrhs), ct.c_void_p(stream), ct.byref(out)), "bilu_autotune")
    return {"sweep_mode": out.sweep_mode, "tile_rows": out.tile_rows, "tile_group": out.tile_group,
            "rhs_tile": out.rhs_tile, "candidates": out.candidates, "apply_us": out.apply_us,
            "default_us": out.default_us}


def bilu_check(ctx, stream):
    _check(lib.bilu_check(ctx, ct.c_void_p(stream)), "bilu_check")


def bilu_timing(ctx, enable):
    _check(lib.bilu_timing(ctx, int(enable)), "bilu_timing")


def bilu_timing_read(ctx, stream):
    out = (KernelTime * K_COUNT)()
    _check(lib.bilu_timing_read(ctx, ct.c_void_p(stream), out), "bilu_timing_read")
    return {K_NAMES[i]: (out[i].launches, out[i].total_ms) for i in range(K_COUNT)}


def bilu_destroy(ctx):
    lib.bilu_destroy(ctx)


def bilu_batch_create(systems, k):
    """systems: sequence of (nb, bs, Ap, Aj) with host structure arrays."""
    keep = [(_i32(Ap), _i32(Aj)) for (_, _, Ap, Aj) in systems]
    descs = (SysDesc * len(systems))()
    for i, ((nb, bs, _, _), (Ap, Aj)) in enumerate(zip(systems, keep)):
        descs[i] = SysDesc(int(nb), int(bs), Ap.ctypes.data, Aj.ctypes.data)
    h = ct.c_void_p()
    bad = ct.c_int(-1)
    st = lib.bilu_batch_create(len(systems), descs, int(k), ct.byref(h), ct.byref(bad))
    if st != OK:
        raise BiluError(st, f"bilu_batch_create (system {bad.value})")
    return h


def bilu_batch_offsets(batch):
    off = ct.c_void_p()
    n = ct.c_int64()
    _check(lib.bilu_batch_offsets(batch, ct.byref(off), ct.byref(n)), "bilu_batch_offsets")
    return off, n.value


def bilu_batch_factor(batch, Ax_ptrs, precision, stream):
    arr = (ct.c_void_p * len(Ax_ptrs))(*[ct.c_void_p(int(p)) for p in Ax_ptrs])
    bad_sys, bad_row = ct.c_int(-1), ct.c_int(-1)
    st = _check(lib.bilu_batch_factor(batch, arr, int(precision), ct.c_void_p(stream), ct.byref(bad_sys),
                                      ct.byref(bad_row)), "bilu_batch_factor", allow_positive=True)
    return st, bad_sys.value, bad_row.value


def bilu_batch_apply(batch, r_ptr, z_ptr, stream):
    _check(lib.bilu_batch_apply(batch, ct.c_void_p(r_ptr), ct.c_void_p(z_ptr), ct.c_void_p(stream)),
           "bilu_batch_apply")


def bilu_batch_spmv(batch, x_ptr, y_ptr, stream):
    _check(lib.bilu_batch_spmv(batch, ct.c_void_p(x_ptr), ct.c_void_p(y_ptr), ct.c_void_p(stream)),
           "bilu_batch_spmv")


def bilu_batch_solve(batch, nsys, b_ptr, x_ptr, rtol, maxit, stream):
    opts = SolveOpts(BICGSTAB, 0, float(rtol), int(maxit))
    info = (RhsInfo * int(nsys))()
    st = _check(lib.bilu_batch_solve(batch, ct.c_void_p(b_ptr), ct.c_void_p(x_ptr), ct.byref(opts), info,
                                     ct.c_void_p(stream)), "bilu_batch_solve", allow_positive=True)
    return st, [(i.status, i.iters, i.relres, i.restarts) for i in info]


def bilu_batch_autotune(batch, stream):
    info = BatchTuneInfo()
    _check(lib.bilu_batch_autotune(batch, ct.c_void_p(stream), ct.byref(info)), "bilu_batch_autotune")
    return {"tile_scale": info.tile_scale, "pair_us": info.pair_us, "default_us": info.default_us,
            "candidates": info.candidates}


def bilu_batch_member(batch, s):
    h = ct.c_void_p()
    _check(lib.bilu_batch_member(batch, int(s), ct.byref(h)), "bilu_batch_member")
    return h


def bilu_batch_destroy(batch):
    lib.bilu_batch_destroy(batch)
