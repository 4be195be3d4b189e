"""GPU parity on the 3D Poisson workload of Section 3, Experiment 1
(Table 1): the 7-point Laplacian regrouped into blocks of b consecutive
unknowns, b in {1, 2, 4, 8}, ILU(k) for k = 0..3, GMRES(20).

Small grids (every b and k, several tiles and ragged tails): factors and one
application within relative 1e-12 of the oracle, GMRES(20) to rtol 1e-6
within +-1 iteration of the oracle and relative 1e-9 of its solution.  The
full 120^3 size (b = 2, ILU(1), the fastest row of the table): one
application against the oracle within 1e-12 and a GMRES(20) solve whose
true residual the oracle's own product confirms."""
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


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [(bs, k) for bs in (1, 2, 4, 8) for k in (0, 1, 2, 3)]


@pytest.mark.parametrize("bs,k", CASES, ids=[f"b{b}_k{k}" for b, k in CASES])
def test_poisson_small_parity(api, oracle_mod, bs, k):
    s = synth.poisson7(11, bs, nx=24, ny=13)
    print(f"poisson 24x13x11 b={bs} ILU({k})", flush=True)
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, k).factor(s.Ax)
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, k)
    Ax = cuda(s.Ax)
    assert M.factor(Ax) == -1
    F, Dinv = M.factors()
    rows = np.repeat(np.arange(s.nb), np.diff(O.Pp))
    off = O.Pj != rows
    bb = bs * bs
    assert rel(F.cpu().numpy().reshape(-1, bb)[off], np.asarray(O.F).reshape(-1, bb)[off]) <= 1e-12
    assert rel(Dinv.cpu().numpy(), O.Dinv) <= 1e-12
    r = np.random.default_rng(7 + bs + 10 * k).uniform(-1, 1, s.n)
    z = M.apply(cuda(r))
    assert rel(z.cpu().numpy(), O.apply(r)) <= 1e-12
    b = np.ones(s.n)
    x, st, info = M.solve(Ax, cuda(b), method="gmres", restart=20, rtol=1e-6)
    xo, ito, rro, sto = O.solve(s.Ax, b, method=1, restart=20, rtol=1e-6)
    assert st == 0 and sto == 0
    assert abs(info[0][1] - ito) <= 1 and info[0][2] <= 1e-6
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-9
    M.close()


def test_poisson_120_b2_ilu1(api, oracle_mod):
    s = synth.poisson_120cube(2)
    print("poisson 120^3 b=2 ILU(1)", flush=True)
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, 1).factor(s.Ax)
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 1)
    Ax = cuda(s.Ax)
    assert M.factor(Ax) == -1
    r = np.random.default_rng(12).uniform(-1, 1, s.n)
    assert rel(M.apply(cuda(r)).cpu().numpy(), O.apply(r)) <= 1e-12
    b = np.ones(s.n)
    x, st, info = M.solve(Ax, cuda(b), method="gmres", restart=20, rtol=1e-6)
    assert st == 0 and info[0][0] == 0
    res = b - oracle_mod.spmv(s.nb, s.bs, s.Ap, s.Aj, s.Ax, x.cpu().numpy())
    rr = np.linalg.norm(res) / np.linalg.norm(b)
    print(f"GMRES(20): {info[0][1]} iterations, relres {info[0][2]:.3e} (oracle product {rr:.3e})")
    assert rr <= 1e-6 and abs(rr - info[0][2]) <= 1e-9
    M.close()
