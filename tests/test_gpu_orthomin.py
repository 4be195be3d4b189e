"""GPU parity of ORTHOMIN(k) (right-preconditioned, every decision on the
device) against the oracle's ORTHOMIN on the same inputs: iterations within
+-1 and the solution within relative 1e-10 at rtol 1e-8 (1e-9 at the
looser Poisson tolerance), k from 0 (minimal residual) to 16, transposed
too, at small and full sizes; and the status paths."""
import numpy as np
import pytest
import torch

from paper_1703_01325_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1703_01325_amd import api as A
    return A


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def nrel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.mark.parametrize("ilu", [0, 1])
@pytest.mark.parametrize("k", [0, 1, 5, 16])
def test_orthomin_small(api, oracle_mod, ilu, k):
    s = synth.small_10cube()
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, ilu).factor(s.Ax)
    rhs = oracle_mod.spmv(s.nb, s.bs, s.Ap, s.Aj, s.Ax, s.xstar)
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, ilu, transpose=True)
    Ax = cuda(s.Ax)
    assert M.factor(Ax) == -1
    x, st, info = M.solve(Ax, cuda(rhs), method="orthomin", restart=k, rtol=1e-8)
    xo, ito, rro, sto = O.solve(s.Ax, rhs, method=2, restart=k, rtol=1e-8)
    assert st == 0 and sto == 0 and info[0][2] <= 1e-8
    assert abs(info[0][1] - ito) <= 1, (info, ito)
    assert nrel(x.cpu().numpy(), xo) <= 1e-10
    g = np.random.default_rng(5 + k).standard_normal(s.n)
    lt, st, info = M.solve(Ax, cuda(g), method="orthomin", restart=k, rtol=1e-8, transpose=True)
    lo, ito, rro, sto = O.solve(s.Ax, g, method=2, restart=k, rtol=1e-8, transpose=True)
    assert st == 0 and sto == 0 and abs(info[0][1] - ito) <= 1
    assert nrel(lt.cpu().numpy(), lo) <= 1e-10
    M.check()
    M.close()


def test_orthomin_poisson_truncation(api, oracle_mod):
    s = synth.poisson7(11, 2, nx=24, ny=13)
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, 0).factor(s.Ax)
    b = np.ones(s.n)
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 0)
    Ax = cuda(s.Ax)
    assert M.factor(Ax) == -1
    for k in (2, 8):
        x, st, info = M.solve(Ax, cuda(b), method="orthomin", restart=k, rtol=1e-6, maxit=4000)
        xo, ito, rro, sto = O.solve(s.Ax, b, method=2, restart=k, rtol=1e-6, maxit=4000)
        print(f"ORTHOMIN({k}): GPU {info[0][1]} iterations, oracle {ito}")
        assert st == 0 and sto == 0 and abs(info[0][1] - ito) <= 1
        assert nrel(x.cpu().numpy(), xo) <= 1e-9
    M.close()


def test_orthomin_mid_full_size(api, oracle_mod):
    s = synth.mid_64cube()
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, 1).factor(s.Ax)
    rhs = oracle_mod.spmv(s.nb, s.bs, s.Ap, s.Aj, s.Ax, s.xstar)
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 1)
    Ax = cuda(s.Ax)
    assert M.factor(Ax) == -1
    x, st, info = M.solve(Ax, cuda(rhs), method="orthomin", restart=10, rtol=1e-8)
    xo, ito, rro, sto = O.solve(s.Ax, rhs, method=2, restart=10, rtol=1e-8)
    assert st == 0 and sto == 0 and info[0][2] <= 1e-8 and abs(info[0][1] - ito) <= 1
    assert nrel(x.cpu().numpy(), xo) <= 1e-10
    M.close()


def test_orthomin_status(api):
    from paper_1703_01325_amd import _native as N
    s = synth.small_10cube()
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 0)
    Ax = cuda(s.Ax)
    assert M.factor(Ax) == -1
    b = cuda(np.random.default_rng(1).standard_normal(s.n))
    x, st, info = M.solve(Ax, b, method="orthomin", restart=5, rtol=1e-8, maxit=1)
    assert st == N.NOT_CONVERGED and info[0][0] == N.NOT_CONVERGED and info[0][1] == 1
    x, st, info = M.solve(Ax, torch.zeros_like(b), method="orthomin", restart=5, rtol=1e-8)
    assert st == 0 and info[0][1] == 0 and float(x.abs().max()) == 0.0
    with pytest.raises(N.BiluError):
        M.solve(Ax, b, method="orthomin", restart=17)
    M.close()
