"""The 3D Poisson workload of Section 3, Experiment 1 (Table 1): the
generator and the oracle on it, pinned by facts that do not come from the
oracle.

* The regrouped block matrix equals the textbook 7-point Laplacian, built
  here as a Kronecker sum of 1D second differences.
* At 120^3 it has the dimension and nonzero count that the paper prints for
  the matrix of Table 1 (n = 1,728,000, nnz = 12,009,600).
* Block ILU(0) on the x-line block grid: a block of the 7-point block
  stencil has no two neighbours that are neighbours of each other, so the
  elimination never updates an off-diagonal block and the factors follow
  the classic diagonal recurrence D_I = A_II - sum_J A_IJ D_J^{-1} A_JI over
  the lower neighbours J of I (for b = 1 the scalar ILU(0) recurrence of
  the 7-point stencil); L_IJ = A_IJ D_J^{-1} and U'_IJ = D_I^{-1} A_IJ.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1703_01325_amd import synth


def scalar_matrix(s):
    """Scalar CSR matrix of a block system (column-major blocks)."""
    b = s.bs
    data = s.Ax.reshape(-1, b, b).transpose(0, 2, 1)
    return sp.bsr_matrix((data, s.Aj, s.Ap), shape=(s.n, s.n)).tocsr()


def laplacian(nx, ny, nz):
    def T(m):
        return sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])

    def I(m):
        return sp.identity(m)

    return (sp.kron(I(nz), sp.kron(I(ny), T(nx))) + sp.kron(I(nz), sp.kron(T(ny), I(nx)))
            + sp.kron(T(nz), sp.kron(I(ny), I(nx)))).tocsr()


@pytest.mark.parametrize("bs", [1, 2, 4, 8])
def test_generator_is_the_7_point_laplacian(bs):
    s = synth.poisson7(5, bs, nx=16, ny=3)
    assert s.grid == (16 // bs, 3, 5) and s.n == 16 * 3 * 5
    D = (scalar_matrix(s) - laplacian(16, 3, 5)).toarray()
    assert np.abs(D).max() == 0.0


def test_table1_dimension_and_nonzeros():
    # Section 3, Experiment 1: n = 1,728,000 and 12,009,600 nonzeros
    for bs in (1, 8):
        s = synth.poisson_120cube(bs)
        assert s.n == 1_728_000
        assert np.count_nonzero(s.Ax) == 12_009_600
        assert s.nnzb == 7 * s.nb - 2 * (s.grid[1] * s.grid[2] + s.grid[0] * s.grid[2] + s.grid[0] * s.grid[1])


def test_rejects_block_size_not_dividing_x():
    with pytest.raises(ValueError):
        synth.poisson7(6, 4)


def block(X, e, b):
    return np.asarray(X[e * b * b:(e + 1) * b * b]).reshape(b, b).T


@pytest.mark.parametrize("bs", [1, 2, 4])
def test_block_ilu0_diagonal_recurrence(oracle_mod, bs):
    s = synth.poisson7(4, bs, nx=8, ny=5)
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, 0).factor(s.Ax)
    assert np.array_equal(O.Pp, s.Ap) and np.array_equal(O.Pj, s.Aj)
    b = bs
    pos = {}
    for i in range(s.nb):
        for e in range(s.Ap[i], s.Ap[i + 1]):
            pos[(i, int(s.Aj[e]))] = e
    D = [None] * s.nb
    for i in range(s.nb):
        Di = block(s.Ax, pos[(i, i)], b).copy()
        for e in range(s.Ap[i], s.Ap[i + 1]):
            j = int(s.Aj[e])
            if j < i:
                Di -= block(s.Ax, e, b) @ np.linalg.solve(D[j], block(s.Ax, pos[(j, i)], b))
        D[i] = Di
    for i in range(s.nb):
        Dinv = block(O.Dinv, i, b)
        assert np.abs(Dinv @ D[i] - np.eye(b)).max() <= 1e-13
        for e in range(s.Ap[i], s.Ap[i + 1]):
            j = int(s.Aj[e])
            F = block(O.F, e, b)
            if j < i:
                ref = block(s.Ax, e, b) @ np.linalg.inv(D[j])
            elif j > i:
                ref = np.linalg.solve(D[i], block(s.Ax, e, b))
            else:
                continue
            assert np.abs(F - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_point_ilu0_first_pivots(oracle_mod):
    # scalar recurrence on the first grid line: d_0 = 6, d_x = 6 - 1/d_{x-1}
    s = synth.poisson7(3, 1, nx=6, ny=4)
    O = oracle_mod.OracleILU(s.nb, 1, s.Ap, s.Aj, 0).factor(s.Ax)
    d = 6.0
    for x in range(6):
        assert abs(1.0 / O.Dinv[x] - d) <= 1e-14 * d
        d = 6.0 - 1.0 / d
