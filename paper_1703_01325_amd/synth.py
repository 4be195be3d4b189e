"""Seeded synthetic reservoir-shaped block systems.

This module only draws inputs: block sparsity patterns, block values and
right-hand sides.  It holds none of the preconditioner's arithmetic (no
factorisation, no triangular solve, no matrix-vector product); a right-hand
side of the form b = A x* is formed by the caller with its own product.

Matrix recipe (one cell = one block row, ``b`` unknowns per cell, the
block-wise setting of Section 2.3, Eq 3):

* grid ``nx x ny x nz``, natural order ``cell = x + nx*(y + ny*z)``;
* 7-point stencil pattern, columns of a block row sorted ascending, the
  diagonal block always stored;
* cell permeability ``K = exp(mu + sigma*Z)``, ``Z ~ N(0,1)`` per cell
  (``mu`` may vary per z-layer);
* face transmissibility ``T_ij = 2 K_i K_j / (K_i + K_j)``;
* off-diagonal block ``A_ij = -T_ij I + 0.1 G_ij`` with ``G_ij ~ N(0,1)``
  drawn independently for ``(i,j)`` and ``(j,i)`` (non-symmetric values);
* diagonal block ``A_ii = diag(s_i) + I + R_i`` with ``s_i[r]`` the sum of
  ``|A_ij[r,c]|`` over the off-diagonal blocks of the block row and
  ``R_i ~ U[-0.2, 0.2]``.

Draw order from one ``numpy.random.Generator(PCG64(seed))``: optional
per-layer means, then ``Z`` per cell, then all ``G`` blocks (block rows
ascending, off-diagonal blocks in ascending column order, each block filled
column by column), then all ``R_i``, then ``x*`` (``U[-1,1]``), then any
workload-specific extras.

Block values are stored column by column inside each block (Section 2.1):
element ``(r, c)`` of block ``e`` is ``Ax[e*b*b + c*b + r]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class BlockSystem:
    """A block sparse system in the block-CSR layout of Section 2.1."""

    nb: int                 # block rows (cells)
    bs: int                 # block size b (unknowns per cell)
    Ap: np.ndarray          # int32 [nb+1] row starts, in blocks
    Aj: np.ndarray          # int32 [nnzb] block column indices, sorted per row
    Ax: np.ndarray          # float64 [nnzb*b*b], column-major inside each block
    xstar: np.ndarray       # float64 [nb*b], exact solution used to form b = A x*
    grid: tuple = (0, 0, 0)
    seed: int = 0
    extras: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nb * self.bs

    @property
    def nnzb(self) -> int:
        return int(self.Ap[-1])


def stencil7_pattern(nx: int, ny: int, nz: int):
    """Block pattern of the 7-point stencil in natural order.

    Returns ``(Ap, Aj)`` int32 with ascending columns per block row.
    """
    nb = nx * ny * nz
    cell = np.arange(nb, dtype=np.int64)
    x = cell % nx
    y = (cell // nx) % ny
    z = cell // (nx * ny)
    # Offsets in ascending order, so the per-row column list comes out sorted.
    offs = np.array([-nx * ny, -nx, -1, 0, 1, nx, nx * ny], dtype=np.int64)
    valid = np.stack([z > 0, y > 0, x > 0, np.ones(nb, bool),
                      x < nx - 1, y < ny - 1, z < nz - 1], axis=1)
    cols = cell[:, None] + offs[None, :]
    counts = valid.sum(axis=1)
    Ap = np.zeros(nb + 1, dtype=np.int64)
    np.cumsum(counts, out=Ap[1:])
    Aj = cols[valid]
    return Ap.astype(np.int32), Aj.astype(np.int32)


def _reservoir_values(rng, Ap, Aj, bs, K):
    nb = Ap.shape[0] - 1
    nnzb = int(Ap[-1])
    rows = np.repeat(np.arange(nb, dtype=np.int64), np.diff(Ap).astype(np.int64))
    offd = Aj.astype(np.int64) != rows
    n_off = int(offd.sum())
    bb = bs * bs
    G = rng.standard_normal(n_off * bb).reshape(n_off, bb)
    R = rng.uniform(-0.2, 0.2, size=nb * bb).reshape(nb, bb)
    Ki = K[rows[offd]]
    Kj = K[Aj[offd].astype(np.int64)]
    T = 2.0 * Ki * Kj / (Ki + Kj)
    eye = np.eye(bs).reshape(bb)          # symmetric, so layout-independent
    vals = np.zeros((nnzb, bb), dtype=np.float64)
    vals[offd] = -T[:, None] * eye[None, :] + 0.1 * G
    # s_i[r] = sum over off-diagonal blocks of the row and over c of |A_ij[r,c]|.
    absoff = np.abs(vals[offd]).reshape(n_off, bs, bs)   # [blk][c][r]
    per_blk = absoff.sum(axis=1)                          # [blk][r]
    s = np.zeros((nb, bs), dtype=np.float64)
    np.add.at(s, rows[offd], per_blk)
    diag = np.zeros((nb, bs, bs), dtype=np.float64)      # [row][c][r]
    idx = np.arange(bs)
    diag[:, idx, idx] = s + 1.0
    diag += R.reshape(nb, bs, bs)
    vals[~offd] = diag.reshape(nb, bb)
    return vals.reshape(-1)


def reservoir(nx, ny, nz, bs, seed, mu=0.0, sigma=1.0, layer_mu=None):
    """Reservoir-shaped 7-point block system.

    ``layer_mu=(lo, hi)`` draws one log-mean per z-layer from ``U[lo, hi]``
    before anything else (layered permeability); otherwise ``mu`` is used.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = nx * ny * nz
    if layer_mu is not None:
        mus = rng.uniform(layer_mu[0], layer_mu[1], size=nz)
        mu_cell = np.repeat(mus, nx * ny)
    else:
        mu_cell = np.full(nb, float(mu))
    Z = rng.standard_normal(nb)
    K = np.exp(mu_cell + sigma * Z)
    Ap, Aj = stencil7_pattern(nx, ny, nz)
    Ax = _reservoir_values(rng, Ap, Aj, bs, K)
    xstar = rng.uniform(-1.0, 1.0, size=nb * bs)
    sysm = BlockSystem(nb=nb, bs=bs, Ap=Ap, Aj=Aj, Ax=Ax, xstar=xstar,
                       grid=(nx, ny, nz), seed=seed)
    sysm.extras["rng"] = rng
    return sysm


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def small_10cube(seed: int = 1) -> BlockSystem:
    """10x10x10 grid, b=3, lognormal(0, 1) permeability."""
    return reservoir(10, 10, 10, 3, seed, mu=0.0, sigma=1.0)


def mid_64cube(seed: int = 2, bs: int = 3) -> BlockSystem:
    """64^3 grid, b=3, lognormal(0, 2) permeability."""
    return reservoir(64, 64, 64, bs, seed, mu=0.0, sigma=2.0)


def layered_60x220x85(seed: int = 3) -> BlockSystem:
    """60x220x85 grid, b=3, per-layer log-mean U[-2,3], sigma 1.5."""
    return reservoir(60, 220, 85, 3, seed, sigma=1.5, layer_mu=(-2.0, 3.0))


def poisson7(n: int, bs: int, seed: int = 6, nx: int | None = None, ny: int | None = None) -> BlockSystem:
    """Scalar 7-point Poisson matrix on an ``nx x ny x n`` grid (``nx``,
    ``ny`` default to ``n``), unknowns in natural order ``u = x + nx*(y +
    ny*z)``, regrouped into block rows of ``bs`` consecutive unknowns (the
    block-size study of Section 3, Table 1).

    Scalar entries: 6 on the diagonal, -1 for each grid neighbour inside the
    domain (homogeneous Dirichlet boundary eliminated, so boundary rows keep
    the 6).  ``bs`` must divide ``nx``: block row ``I`` then holds the ``bs``
    x-consecutive unknowns of one grid line segment, and the block pattern is
    the 7-point stencil of the ``nx/bs x ny x n`` block grid.  The diagonal
    block is tridiagonal (-1, 6, -1); the block of the x-neighbour segment
    before holds a single -1 at (0, bs-1), the one after at (bs-1, 0), and
    the y and z neighbour blocks are -I.  The explicit zeros of the
    x-neighbour blocks are stored, as the block format does.

    The exact solution ``x*`` is drawn ``U[-1, 1]`` from ``PCG64(seed)``.
    """
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    if bs < 1 or nx % bs:
        raise ValueError(f"block size {bs} must divide the x extent {nx}")
    gx = nx // bs
    Ap, Aj = stencil7_pattern(gx, ny, n)
    nb = gx * ny * n
    bb = bs * bs
    rows = np.repeat(np.arange(nb, dtype=np.int64), np.diff(Ap).astype(np.int64))
    d = Aj.astype(np.int64) - rows
    vals = np.zeros((int(Ap[-1]), bs, bs), dtype=np.float64)   # [blk][c][r]
    idx = np.arange(bs)
    diag = np.zeros((bs, bs))
    diag[idx, idx] = 6.0
    diag[idx[:-1], idx[1:]] = -1.0
    diag[idx[1:], idx[:-1]] = -1.0
    vals[d == 0] = diag                      # symmetric: layout-independent
    vals[d == -1, bs - 1, 0] = -1.0          # (r=0, c=bs-1), column-major
    vals[d == 1, 0, bs - 1] = -1.0           # (r=bs-1, c=0)
    far = np.nonzero(np.abs(d) > 1)[0]
    vals[far[:, None], idx[None, :], idx[None, :]] = -1.0
    rng = np.random.Generator(np.random.PCG64(seed))
    xstar = rng.uniform(-1.0, 1.0, size=nb * bs)
    return BlockSystem(nb=nb, bs=bs, Ap=Ap, Aj=Aj, Ax=vals.reshape(-1), xstar=xstar,
                       grid=(gx, ny, n), seed=seed)


def poisson_120cube(bs: int, seed: int = 6) -> BlockSystem:
    """The 120^3 Poisson matrix (n = 1,728,000) with blocks of ``bs``."""
    return poisson7(120, bs, seed)


def multi_rhs(n: int, nrhs: int, seed: int = 41) -> np.ndarray:
    """(n, nrhs) right-hand sides, entries U[-1,1], row-major."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=(n, nrhs))


BATCH_BLOCK_SIZES = (2, 3, 4, 6, 8)


def uneven_batch_member(s: int, side_lo: int = 8, side_hi: int = 40) -> BlockSystem:
    """System ``s`` of the uneven batch: sides U{lo..hi}, b from {2,3,4,6,8}."""
    rng = np.random.Generator(np.random.PCG64(4200 + s))
    nx, ny, nz = (int(v) for v in rng.integers(side_lo, side_hi + 1, size=3))
    bs = int(rng.choice(np.array(BATCH_BLOCK_SIZES)))
    sub_seed = int(rng.integers(0, 2**63 - 1))
    return reservoir(nx, ny, nz, bs, sub_seed, mu=0.0, sigma=1.0)


def thermal_64cube(seed: int = 5) -> BlockSystem:
    """64^3 grid, b=4, lognormal(0, 2); adds the adjoint workload extras.

    extras: ``sel`` (sorted distinct unknowns, 1% of n), ``d`` ~ N(0,1),
    ``fd_blocks``/``fd_rc`` (20 stored scalar entries of A: block uniform,
    then (r, c) uniform) and ``fd_b`` (20 entries of b).
    """
    sysm = reservoir(64, 64, 64, 4, seed, mu=0.0, sigma=2.0)
    add_adjoint_extras(sysm)
    return sysm


def add_adjoint_extras(sysm: BlockSystem, frac: float = 0.01, n_fd: int = 20):
    rng = sysm.extras["rng"]
    n = sysm.n
    m = max(1, int(np.floor(frac * n)))
    sel = np.sort(rng.choice(n, size=m, replace=False))
    d = rng.standard_normal(m)
    fd_blocks = rng.integers(0, sysm.nnzb, size=n_fd)
    fd_rc = rng.integers(0, sysm.bs, size=(n_fd, 2))
    fd_b = rng.choice(n, size=n_fd, replace=False)
    sysm.extras.update(sel=sel, d=d, fd_blocks=fd_blocks, fd_rc=fd_rc, fd_b=fd_b)
    return sysm


def random_block_pattern(nb: int, density: float, seed: int, symmetric=False):
    """Random block pattern with a stored diagonal, sorted unique columns."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = rng.random((nb, nb)) < density
    if symmetric:
        M = M | M.T
    np.fill_diagonal(M, True)
    Ap = np.zeros(nb + 1, dtype=np.int32)
    Ap[1:] = np.cumsum(M.sum(axis=1))
    Aj = np.nonzero(M)[1].astype(np.int32)
    return Ap, Aj


def graded_block_pattern(nb: int, lo: float, hi: float, seed: int):
    """Random block pattern whose row density rises linearly from lo (first
    row) to hi (last row): short and long rows in one matrix.  Stored
    diagonal, sorted unique columns."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dens = np.linspace(lo, hi, nb)[:, None]
    M = rng.random((nb, nb)) < dens
    np.fill_diagonal(M, True)
    Ap = np.zeros(nb + 1, dtype=np.int32)
    Ap[1:] = np.cumsum(M.sum(axis=1))
    Aj = np.nonzero(M)[1].astype(np.int32)
    return Ap, Aj


def random_block_values(Ap, Aj, bs, seed, dominance=1.0):
    """Random block values; diagonal blocks made row diagonally dominant."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = Ap.shape[0] - 1
    nnzb = int(Ap[-1])
    bb = bs * bs
    vals = rng.uniform(-1.0, 1.0, size=(nnzb, bs, bs))   # [blk][c][r]
    rows = np.repeat(np.arange(nb), np.diff(Ap))
    absrow = np.zeros((nb, bs))
    np.add.at(absrow, rows, np.abs(vals).sum(axis=1))
    dpos = np.nonzero(Aj == rows)[0]
    idx = np.arange(bs)
    vals[dpos[:, None], idx[None, :], idx[None, :]] += absrow + dominance
    return vals.reshape(nnzb * bb)
