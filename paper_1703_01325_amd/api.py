"""Torch-facing wrapper over the C ABI: torch tensors in, pointers out.

torch provides device memory and the current HIP stream; every step of
the preconditioner and the solvers runs in libbilu.so's kernels.  There is
no CPU fallback: the native library must be built and a GPU present.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _native as N


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _dev_f64(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    return t


def _dev_i32(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous int32 CUDA tensor")
    return t


def symbolic_device(Ap: torch.Tensor, Aj: torch.Tensor, k: int):
    """Symbolic phase on the GPU (Algorithm 3, Eq 1-2): (Pp, Pj, lev) of the
    ILU(k) pattern as int32 CUDA tensors, from A's block pattern on the GPU."""
    _dev_i32(Ap, "Ap")
    _dev_i32(Aj, "Aj")
    nb = Ap.numel() - 1
    Pp = torch.empty(nb + 1, dtype=torch.int32, device=Ap.device)
    nnz = N.bilu_symbolic_device(nb, Ap.data_ptr(), Aj.data_ptr(), k, Pp.data_ptr(), None, None, 0, _stream())
    Pj = torch.empty(max(nnz, 1), dtype=torch.int32, device=Ap.device)
    lev = torch.empty(max(nnz, 1), dtype=torch.int32, device=Ap.device)
    N.bilu_symbolic_device(nb, Ap.data_ptr(), Aj.data_ptr(), k, Pp.data_ptr(), Pj.data_ptr(), lev.data_ptr(),
                           nnz, _stream())
    return Pp, Pj[:nnz], lev[:nnz]


def levels_device(Pp: torch.Tensor, Pj: torch.Tensor, sweep: int):
    """Level sets of one sweep on the GPU (Eq 4): (lvl, level_ptr, level_rows)
    as int32 CUDA tensors, level_ptr of length nlev + 1."""
    _dev_i32(Pp, "Pp")
    _dev_i32(Pj, "Pj")
    nb = Pp.numel() - 1
    lvl = torch.empty(nb, dtype=torch.int32, device=Pp.device)
    ptr = torch.empty(nb + 1, dtype=torch.int32, device=Pp.device)
    rows = torch.empty(nb, dtype=torch.int32, device=Pp.device)
    nlev = N.bilu_levels_device(nb, Pp.data_ptr(), Pj.data_ptr(), sweep, lvl.data_ptr(), ptr.data_ptr(),
                                rows.data_ptr(), _stream())
    return lvl, ptr[:nlev + 1], rows


class BlockILU:
    """Decoupled block ILU(k) of one block pattern (Algorithm 5, Eq 5).

    ``BlockILU(nb, bs, Ap, Aj, k)`` runs the symbolic phase and the level
    sets on the host (``device_symbolic=True``: on the GPU, the same
    results); ``factor(Ax)`` runs the numeric phase and the diagonal split
    on the GPU; ``apply``/``spmv``/``solve`` run the hot path.
    """

    def __init__(self, nb, bs, Ap, Aj, k, transpose=False, device_symbolic=False):
        self.nb, self.bs, self.k = int(nb), int(bs), int(k)
        self.n = self.nb * self.bs
        self.Ap = np.ascontiguousarray(Ap, np.int32)
        self.Aj = np.ascontiguousarray(Aj, np.int32)
        flags = (N.WANT_TRANSPOSE if transpose else 0) | (N.DEVICE_SYMBOLIC if device_symbolic else 0)
        self._ctx = N.bilu_analyze(nb, bs, self.Ap, self.Aj, k, flags)
        self.transpose = bool(transpose)
        self.precision = None
        self._owned = True

    # ---- host views -------------------------------------------------------
    def info(self):
        return N.bilu_get_info(self._ctx)

    def pattern(self):
        return N.bilu_get_pattern(self._ctx)

    def levels(self, sweep):
        return N.bilu_get_levels(self._ctx, sweep)

    def set_sweep_mode(self, mode):
        N.bilu_tune(self._ctx, N.TUNE_SWEEP_MODE, mode)

    def tune(self, mode=None, tile_rows=None, blocks=None, rhs_tile=None, fuse_spmv=None, tile_group=None,
             tile_block=None, line_sweep=None, helper=None, spmv_stream=None, rhs_pairs=None, split_dinv=None,
             factor=None, spin_limit=None):
        """Launch knobs of the sweeps and the factorisation (results are
        bit-identical for all).  ``factor``: "waves" (one persistent launch,
        8 rows per workgroup where the LDS allows), "levels" (one launch per
        L level), "waves16" / "waves4" (16 where the LDS allows / at most 4
        rows per workgroup).  ``spin_limit``: polls of a bounded wait before
        the call fails with a time-out (0: the default)."""
        for key, val in ((N.TUNE_SWEEP_MODE, mode), (N.TUNE_TILE_ROWS, tile_rows), (N.TUNE_BLOCKS, blocks),
                         (N.TUNE_RHS_TILE, rhs_tile), (N.TUNE_TILE_GROUP, tile_group),
                         (N.TUNE_TILE_BLOCK, None if tile_block is None else
                          (0 if not tile_block else tile_block[0] + 256 * tile_block[1])),
                         (N.TUNE_LINE_SWEEP, None if line_sweep is None else
                          (0 if not line_sweep else line_sweep[0] + 256 * line_sweep[1])),
                         (N.TUNE_HELPER, None if helper is None else
                          (0 if helper == "auto" else 1 if helper else 2)),
                         (N.TUNE_SPMV_STREAM, None if spmv_stream is None else
                          (0 if spmv_stream == "auto" else 1 if spmv_stream else 2)),
                         (N.TUNE_RHS_PAIRS, None if rhs_pairs is None else
                          (0 if rhs_pairs == "auto" else 2 if rhs_pairs else 1)),
                         (N.TUNE_SPLIT_DINV, None if split_dinv is None else
                          (0 if split_dinv == "auto" else 2 if split_dinv else 1)),
                         (N.TUNE_FACTOR, None if factor is None else {"waves": 0, "levels": 1, "waves16": 2, "waves4": 3}[factor]),
                         (N.TUNE_SPIN_LIMIT, spin_limit),
                         (N.TUNE_FUSE_SPMV, None if fuse_spmv is None else int(bool(fuse_spmv)))):
            if val is not None:
                N.bilu_tune(self._ctx, key, val)

    def autotune(self, nrhs: int = 1):
        """Times candidate launch configurations on the device and keeps the
        fastest (after factor); returns the choice and its timings."""
        return N.bilu_autotune(self._ctx, nrhs, _stream())

    # ---- GPU --------------------------------------------------------------
    def factor(self, Ax: torch.Tensor, precision: str = "fp64"):
        """Numeric factorisation + U = D U'.  Returns the block row of a
        singular pivot, or -1."""
        _dev_f64(Ax, "Ax")
        st, bad = N.bilu_factor_numeric(self._ctx, Ax.data_ptr(), _stream())
        if st == N.SINGULAR_PIVOT:
            return bad
        prec = N.FACTORS_FP32 if precision == "fp32" else N.FACTORS_FP64
        N.bilu_factor_diag(self._ctx, prec, _stream())
        self.precision = precision
        return -1

    def _vec_shape(self, v):
        if v.dim() == 1:
            return 1
        return v.shape[1]

    def apply(self, r: torch.Tensor, out: torch.Tensor | None = None, transpose=False):
        _dev_f64(r, "r")
        z = torch.empty_like(r) if out is None else out
        fn = N.bilu_apply_transpose if transpose else N.bilu_apply
        fn(self._ctx, r.data_ptr(), z.data_ptr(), self._vec_shape(r), _stream())
        return z

    def apply_point(self, r: torch.Tensor, out: torch.Tensor | None = None):
        """z = M^{-1} r through the point-granularity sweeps (one column)."""
        _dev_f64(r, "r")
        z = torch.empty_like(r) if out is None else out
        N.bilu_apply_point(self._ctx, r.data_ptr(), z.data_ptr(), _stream())
        return z

    def spmv(self, Ax: torch.Tensor, x: torch.Tensor, out=None, transpose=False):
        _dev_f64(Ax, "Ax")
        _dev_f64(x, "x")
        y = torch.empty_like(x) if out is None else out
        N.bilu_spmv(self._ctx, Ax.data_ptr(), x.data_ptr(), y.data_ptr(), self._vec_shape(x),
                    int(transpose), _stream())
        return y

    def solve(self, Ax, b, method="bicgstab", restart=30, rtol=1e-8, maxit=2000, transpose=False,
              out=None):
        """x = A^{-1} b (or A^{-T} b); returns (x, status, [(status, iters, relres, restarts)] per RHS)."""
        _dev_f64(Ax, "Ax")
        _dev_f64(b, "b")
        x = torch.empty_like(b) if out is None else out
        m = {"bicgstab": N.BICGSTAB, "gmres": N.GMRES, "orthomin": N.ORTHOMIN}[method]
        st, info = N.bilu_solve(self._ctx, Ax.data_ptr(), b.data_ptr(), x.data_ptr(), self._vec_shape(b),
                                m, restart, rtol, maxit, int(transpose), _stream())
        return x, st, info

    def grad_A(self, lam, x):
        _dev_f64(lam, "lambda")
        _dev_f64(x, "x")
        info = self.info()
        dA = torch.empty(int(info.nnzb_A) * self.bs * self.bs, dtype=torch.float64, device=x.device)
        N.bilu_grad_A(self._ctx, lam.data_ptr(), x.data_ptr(), dA.data_ptr(), _stream())
        return dA

    def factors(self):
        """FP64 factors in pattern order (L below, U' above, I on the diagonal) and D^{-1}."""
        info = self.info()
        bb = self.bs * self.bs
        F = torch.empty(int(info.nnzb_P) * bb, dtype=torch.float64, device="cuda")
        D = torch.empty(self.nb * bb, dtype=torch.float64, device="cuda")
        N.bilu_get_factors(self._ctx, F.data_ptr(), D.data_ptr(), _stream())
        return F, D

    def factors_f32(self):
        info = self.info()
        bb = self.bs * self.bs
        F = torch.empty(int(info.nnzb_P) * bb, dtype=torch.float32, device="cuda")
        D = torch.empty(self.nb * bb, dtype=torch.float32, device="cuda")
        N.bilu_get_factors_f32(self._ctx, F.data_ptr(), D.data_ptr(), _stream())
        return F, D

    def timing(self, enable: bool):
        N.bilu_timing(self._ctx, int(enable))

    def timing_read(self):
        """{kernel class: (launches, total ms)} from HIP events on the launch stream."""
        return N.bilu_timing_read(self._ctx, _stream())

    def check(self):
        N.bilu_check(self._ctx, _stream())

    def close(self):
        if self._ctx is not None:
            if self._owned:
                N.bilu_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BlockILUBatch:
    """Independent systems of uneven sizes and block sizes, preconditioned
    and solved together: one sweep launch, one SpMV launch and one launch
    per vector step serve every member.

    ``systems`` is a sequence of ``(nb, bs, Ap, Aj)``.  Batch vectors are the
    members' vectors laid end to end (``offsets``).
    """

    def __init__(self, systems, k):
        self.k = int(k)
        self.systems = [(int(nb), int(bs), np.ascontiguousarray(Ap, np.int32), np.ascontiguousarray(Aj, np.int32))
                        for (nb, bs, Ap, Aj) in systems]
        self.nsys = len(self.systems)
        self._b = N.bilu_batch_create(self.systems, k)
        off_p, self.n = N.bilu_batch_offsets(self._b)
        import ctypes as ct
        self.offsets = np.ctypeslib.as_array(ct.cast(off_p, ct.POINTER(ct.c_int64)), shape=(self.nsys + 1,)).copy()
        self._Ax = None

    def factor(self, Ax_list, precision: str = "fp64"):
        """Factor every member; ``Ax_list[s]`` stays referenced for the SpMVs.
        Returns (system, block row) of a singular pivot, or None."""
        for s, Ax in enumerate(Ax_list):
            _dev_f64(Ax, f"Ax[{s}]")
        self._Ax = list(Ax_list)
        prec = N.FACTORS_FP32 if precision == "fp32" else N.FACTORS_FP64
        st, bad_sys, bad_row = N.bilu_batch_factor(self._b, [a.data_ptr() for a in self._Ax], prec, _stream())
        if st == N.SINGULAR_PIVOT:
            return bad_sys, bad_row
        return None

    def apply(self, r: torch.Tensor, out: torch.Tensor | None = None):
        _dev_f64(r, "r")
        z = torch.empty_like(r) if out is None else out
        N.bilu_batch_apply(self._b, r.data_ptr(), z.data_ptr(), _stream())
        return z

    def spmv(self, x: torch.Tensor, out: torch.Tensor | None = None):
        _dev_f64(x, "x")
        y = torch.empty_like(x) if out is None else out
        N.bilu_batch_spmv(self._b, x.data_ptr(), y.data_ptr(), _stream())
        return y

    def solve(self, b: torch.Tensor, rtol=1e-8, maxit=2000, out=None):
        """BiCGSTAB on every member; returns (x, worst status, per-member
        (status, iterations, true relative residual))."""
        _dev_f64(b, "b")
        x = torch.empty_like(b) if out is None else out
        st, info = N.bilu_batch_solve(self._b, self.nsys, b.data_ptr(), x.data_ptr(), rtol, maxit, _stream())
        return x, st, info

    def autotune(self):
        """Device-timed choice of the members' tile sizes (results unchanged)."""
        return N.bilu_batch_autotune(self._b, _stream())

    def member(self, s: int) -> BlockILU:
        """Member s as a BlockILU view (owned by the batch)."""
        nb, bs, Ap, Aj = self.systems[s]
        m = object.__new__(BlockILU)
        m.nb, m.bs, m.k, m.n = nb, bs, self.k, nb * bs
        m.Ap, m.Aj = Ap, Aj
        m._ctx = N.bilu_batch_member(self._b, s)
        m.transpose = False
        m.precision = None
        m._owned = False
        return m

    def close(self):
        if self._b is not None:
            N.bilu_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
