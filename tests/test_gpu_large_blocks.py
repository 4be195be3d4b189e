"""Block sizes above the block-row kernels (9..32; the paper's Table 2 uses
b = 25): the factorisation by blocks with the block size a run-time value,
the split, the SpMV and an application at point granularity, each against
the oracle (factors, applications and SpMVs relative 1e-12, solves within
+-1 iteration and relative 1e-10), and the calls such systems refuse."""
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


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def nrel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [(bs, k) for bs in (9, 16, 25) for k in (0, 1)]


@pytest.mark.parametrize("bs,k", CASES, ids=[f"b{b}_k{k}" for b, k in CASES])
def test_large_block_parity(api, oracle_mod, bs, k):
    s = synth.reservoir(6, 5, 4, bs, seed=200 + bs)
    print(f"b={bs} ILU({k})", flush=True)
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, k).factor(s.Ax)
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, k)
    Ax = cuda(s.Ax)
    assert M.factor(Ax) == -1
    F, D = M.factors()
    rows = np.repeat(np.arange(s.nb), np.diff(O.Pp))
    bb = bs * bs
    Fg, Fo = F.cpu().numpy().reshape(-1, bb), np.asarray(O.F).reshape(-1, bb)
    assert rel(Fg[O.Pj < rows], Fo[O.Pj < rows]) <= 1e-12
    assert rel(Fg[O.Pj > rows], Fo[O.Pj > rows]) <= 1e-12
    assert rel(D.cpu().numpy(), O.Dinv) <= 1e-12
    r = np.random.default_rng(bs).standard_normal(s.n)
    z = M.apply(cuda(r))
    assert rel(z.cpu().numpy(), O.apply(r)) <= 1e-12
    assert torch.equal(M.apply_point(cuda(r)), z)
    y = M.spmv(Ax, cuda(r))
    assert rel(y.cpu().numpy(), oracle_mod.spmv(s.nb, s.bs, s.Ap, s.Aj, s.Ax, r)) <= 1e-13
    rhs = oracle_mod.spmv(s.nb, s.bs, s.Ap, s.Aj, s.Ax, s.xstar)
    for method, m_id, m in (("bicgstab", 0, 20), ("gmres", 1, 20), ("orthomin", 2, 10)):
        x, st, info = M.solve(Ax, cuda(rhs), method=method, restart=m, rtol=1e-8)
        xo, ito, rro, sto = O.solve(s.Ax, rhs, method=m_id, restart=m, rtol=1e-8)
        assert st == 0 and sto == 0 and info[0][2] <= 1e-8, (method, info)
        assert abs(info[0][1] - ito) <= 1, (method, info, ito)
        assert nrel(x.cpu().numpy(), xo) <= 1e-10, method
    M.check()
    M.close()


def test_large_block_refusals(api):
    from paper_1703_01325_amd import _native as N
    s = synth.reservoir(4, 3, 3, 25, seed=250)
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 0, transpose=True)
    Ax = cuda(s.Ax)
    with pytest.raises(N.BiluError):
        M.factor(Ax, precision="fp32")
    assert M.factor(Ax) == -1
    with pytest.raises(N.BiluError):
        M.apply(cuda(np.ones((s.n, 2))))
    with pytest.raises(N.BiluError):
        M.apply(cuda(np.ones(s.n)), transpose=True)
    with pytest.raises(N.BiluError):
        api.BlockILUBatch([(s.nb, s.bs, s.Ap, s.Aj)], 0)
    M.close()
