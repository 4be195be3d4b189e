"""bilu_apply_noalloc through the C ABI: the same result bits as bilu_apply,
on calls in a row that share the device scratch (the second with a smaller
input), straight after the factorisation and after other applications;
sizes beyond the scratch and calls before the layouts exist are refused."""
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


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _noalloc(N, M, r):
    z = torch.empty_like(r)
    N.bilu_apply_noalloc(M._ctx, r.data_ptr(), z.data_ptr(), 1 if r.dim() == 1 else r.shape[1], _stream())
    return z


def test_noalloc_matches_apply(api, oracle_mod):
    from paper_1703_01325_amd import _native as N
    cases = [(synth.small_10cube(), 1, 4, "fp64"),                      # 3000 x 4
             (synth.reservoir(6, 5, 4, 3, seed=19), 0, 1, "fp32")]      # 360 x 1
    for s, k, R, prec in cases:
        M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, k)
        assert M.factor(torch.from_numpy(s.Ax).cuda(), precision=prec) == -1
        rng = np.random.default_rng(R)
        r = torch.from_numpy(rng.standard_normal(s.n if R == 1 else (s.n, R))).cuda()
        if R == 1:
            # the layouts for one column exist after the factorisation
            z0 = _noalloc(N, M, r)
        ref = M.apply(r)
        z1 = _noalloc(N, M, r)
        z2 = _noalloc(N, M, r)
        torch.cuda.synchronize()
        assert torch.equal(z1, ref) and torch.equal(z2, ref)
        if R == 1:
            assert torch.equal(z0, ref)
        if prec == "fp64":
            O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, k).factor(s.Ax)
            rc = r.cpu().numpy()
            for j in range(R):
                zo = O.apply(rc[:, j] if R > 1 else rc)
                zg = z1.cpu().numpy()
                zg = zg[:, j] if R > 1 else zg
                assert np.abs(zg - zo).max() <= 1e-12 * np.abs(zo).max()
        M.check()
        M.close()


def test_noalloc_refusals(api):
    from paper_1703_01325_amd import _native as N
    # 64^3 block rows of size 3 with 8 columns: 50 MB of intermediate vector
    s = synth.mid_64cube()
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 0)
    r = torch.zeros((s.n, 8), dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    with pytest.raises(N.BiluError) as ei:
        N.bilu_apply_noalloc(M._ctx, r.data_ptr(), z.data_ptr(), 8, _stream())
    assert ei.value.code == N.ERR_ARG
    # one column fits, but nothing is factored yet
    with pytest.raises(N.BiluError) as ei:
        N.bilu_apply_noalloc(M._ctx, r.data_ptr(), z.data_ptr(), 1, _stream())
    assert ei.value.code == N.ERR_STATE
    M.close()
