"""Pins of the oracle's ORTHOMIN(k) (the reservoir Krylov method the paper's
introduction names), independent of its code:

* with every direction kept (k at least the number of iterations) the method
  is a minimal-residual method on the right-preconditioned Krylov space, so
  after j iterations ||b - A x_j|| equals the least-squares minimum over
  x in span{M^{-1} u_0, ..., M^{-1} u_{j-1}}, u_i = (A M^{-1})^i b, found
  here by numpy on an explicit (orthonormalised) basis;
* k = 0 is the minimal-residual iteration: one step is x = alpha M^{-1} b
  with alpha = (b, q) / (q, q), q = A M^{-1} b;
* ORTHOMIN(5) reaches the tolerance with a true residual scipy confirms.
The preconditioner inside the brute force is the oracle's own application,
pinned by its own tests; what these pins check is the Krylov loop."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1703_01325_amd import synth


def dense_A(s):
    data = s.Ax.reshape(-1, s.bs, s.bs).transpose(0, 2, 1)
    return sp.bsr_matrix((data, s.Aj, s.Ap), shape=(s.n, s.n)).toarray()


def system():
    Ap, Aj = synth.random_block_pattern(24, 0.15, seed=301)
    Ax = synth.random_block_values(Ap, Aj, 2, seed=302, dominance=0.5)
    s = synth.BlockSystem(nb=24, bs=2, Ap=Ap, Aj=Aj, Ax=Ax, xstar=np.zeros(48))
    return s


@pytest.mark.parametrize("j", [1, 2, 3, 5, 8])
def test_full_orthomin_is_minimal_residual(oracle_mod, j):
    s = system()
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, 0).factor(s.Ax)
    A = dense_A(s)
    b = np.random.default_rng(303).standard_normal(s.n)
    x, it, rr, st = O.solve(s.Ax, b, method=2, restart=50, rtol=1e-300, maxit=j)
    assert it == j and st == 2
    res = np.linalg.norm(b - A @ x)
    # explicit Krylov basis of A M^{-1} from b, orthonormalised
    U = np.zeros((s.n, j))
    u = b / np.linalg.norm(b)
    for i in range(j):
        U[:, i] = u
        Q, _ = np.linalg.qr(U[:, :i + 1])
        u = A @ O.apply(Q[:, i])
        u = u - Q @ (Q.T @ u)
        u = u / np.linalg.norm(u)
    Q, _ = np.linalg.qr(U)
    W = np.column_stack([O.apply(Q[:, i]) for i in range(j)])
    y, *_ = np.linalg.lstsq(A @ W, b, rcond=None)
    best = np.linalg.norm(b - A @ W @ y)
    assert abs(res - best) <= 1e-10 * np.linalg.norm(b), (res, best)


def test_orthomin0_first_step_closed_form(oracle_mod):
    s = system()
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, 1).factor(s.Ax)
    A = dense_A(s)
    b = np.random.default_rng(304).standard_normal(s.n)
    x, it, rr, st = O.solve(s.Ax, b, method=2, restart=0, rtol=1e-300, maxit=1)
    z = O.apply(b)
    q = A @ z
    alpha = (b @ q) / (q @ q)
    assert np.abs(x - alpha * z).max() <= 1e-14 * np.abs(alpha * z).max()


def test_orthomin_converges_true_residual(oracle_mod):
    s = synth.small_10cube()
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, 0).factor(s.Ax)
    b = oracle_mod.spmv(s.nb, s.bs, s.Ap, s.Aj, s.Ax, s.xstar)
    x, it, rr, st = O.solve(s.Ax, b, method=2, restart=5, rtol=1e-8)
    assert st == 0 and rr <= 1e-8
    A = sp.bsr_matrix((s.Ax.reshape(-1, 3, 3).transpose(0, 2, 1), s.Aj, s.Ap), shape=(s.n, s.n))
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
    assert np.linalg.norm(x - s.xstar) / np.linalg.norm(s.xstar) <= 1e-6
